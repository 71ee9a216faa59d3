// Per-tile front-to-back alpha blending (Eq. (rendering), Sec. 3) with the
// dominant Gaussian map (Eq. (dominant-map), Sec. 4.1) and the per-pixel L1
// error of Eq. (l1map) fused into the same traversal, and the matching reverse
// pass.
//
// One 16x16 tile per 256-thread block; each wave64 owns an 8x8 quadrant.
// Gaussian records are staged through LDS in batches of 256.  A staged
// record carries the Gaussian's pixel box as two 16-bit masks over the tile's
// columns and rows: a wave skips a Gaussian whose box misses its quadrant
// (wave-uniform branch), and a pixel outside the box never composites it, so
// the contributor set is exactly {box holds the pixel, alpha >= 1/255}.  A
// block stops fetching once all 256 pixels have saturated.
//
// Alpha is evaluated as exp2(q) with q = a' dx^2 + b' dx dy + c' dy^2 + log2(o)
// (conic pre-scaled by -log2(e)/2, opacity folded into the exponent); the
// forward and the reverse pass share the staged values and the helper below,
// so they take identical alpha decisions.
#include "internal.h"

namespace {

constexpr float ALPHA_MIN = 1.0f / 255.0f;
constexpr float ALPHA_MAX = 0.99f;
constexpr float T_STOP = 1e-4f;
constexpr float LOG2E = 1.4426950408889634f;
constexpr float LN2 = 0.6931471805599453f;

struct StagedRec {
    float4 mc;  // mean x, mean y (tile-relative), a', b'
    float4 cc;  // c', log2(o), r, g
};

__device__ __forceinline__ float blend_exponent(float dx, float dy, const StagedRec &r) {
#pragma clang fp contract(off)
    return __fmaf_rn(r.mc.z * dx, dx, __fmaf_rn(r.cc.x * dy, dy, __fmaf_rn(r.mc.w * dx, dy, r.cc.y)));
}

__device__ __forceinline__ uint32_t span_mask(int lo, int hi) {   // bits lo..hi of 16, clamped
    lo = lo < 0 ? 0 : lo;
    hi = hi > 15 ? 15 : hi;
    if (hi < lo) return 0u;
    return ((2u << hi) - 1u) & ~((1u << lo) - 1u);
}

// Stage Gaussian `id` for the tile at (ox, oy).
__device__ __forceinline__ void stage_record(const BlendRec *__restrict__ rec, const short4 *__restrict__ box,
                                             uint32_t id, int ox, int oy, StagedRec &s, float &blue,
                                             uint32_t &mask) {
#pragma clang fp contract(off)
    const BlendRec r = rec[id];
    const short4 b = box[id];
    const float mx = (r.m.x - (float)ox) + r.m.z;
    const float my = (r.m.y - (float)oy) + r.m.w;
    const float k = -0.5f * LOG2E;
    s.mc = make_float4(mx, my, k * r.c.x, -LOG2E * r.c.y);
    s.cc = make_float4(k * r.c.z, __log2f(r.c.w), r.rgb.x, r.rgb.y);
    blue = r.rgb.z;
    mask = span_mask(b.x - ox, b.z - ox) | (span_mask(b.y - oy, b.w - oy) << 16);
}

__global__ void __launch_bounds__(AS_BLOCK) k_blend_fwd(const uint32_t *__restrict__ ranges,
                                                        const uint32_t *__restrict__ vals,
                                                        const BlendRec *__restrict__ rec,
                                                        const short4 *__restrict__ box, DevCam cam, int tiles_x,
                                                        const float *__restrict__ gt, float *__restrict__ image,
                                                        float *__restrict__ t_final, uint32_t *__restrict__ last_out,
                                                        uint32_t *__restrict__ ncontrib_out,
                                                        int32_t *__restrict__ dom_out, double *__restrict__ err,
                                                        unsigned long long *__restrict__ minmax) {
    __shared__ StagedRec s_rec[AS_BLOCK];
    __shared__ float s_blue[AS_BLOCK];
    __shared__ int32_t s_id[AS_BLOCK];
    __shared__ uint32_t s_mask[AS_BLOCK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int tile = blockIdx.x;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int qx = (w & 1) * 8, qy = (w >> 1) * 8;
    const int lx = qx + (lane & 7), ly = qy + (lane >> 3);
    const int ox = tx * AS_TILE_W, oy = ty * AS_TILE_H;
    const int x = ox + lx, y = oy + ly;
    const bool inside = x < cam.W && y < cam.H;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const uint32_t qmx = 0xFFu << qx, qmy = (0xFFu << qy) << 16;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

    float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, wbest = 0.f;
    int32_t dom = -1;
    uint32_t last = 0, nc = 0;
    int done = inside ? 0 : 1;

    for (uint32_t b0 = start; b0 < end; b0 += AS_BLOCK) {
        if (__syncthreads_count(done) == AS_BLOCK) break;
        const uint32_t idx = b0 + tid;
        if (idx < end) {
            const uint32_t id = vals[idx];
            StagedRec sr;
            float blue;
            uint32_t m;
            stage_record(rec, box, id, ox, oy, sr, blue, m);
            s_rec[tid] = sr;
            s_blue[tid] = blue;
            s_id[tid] = (int32_t)id;
            s_mask[tid] = m;
        }
        __syncthreads();
        if (!done) {
            const int cnt = (int)min((uint32_t)AS_BLOCK, end - b0);
            for (int j = 0; j < cnt; j++) {
                const uint32_t m = s_mask[j];
                if (!(m & qmx) || !(m & qmy)) continue;            // box misses this quadrant
                if (!((m >> lx) & (m >> (16 + ly)) & 1u)) continue;  // box misses this pixel
                const StagedRec r = s_rec[j];
                const float dx = r.mc.x - px, dy = r.mc.y - py;
                const float araw = __builtin_amdgcn_exp2f(blend_exponent(dx, dy, r));
                const float alpha = fminf(ALPHA_MAX, araw);
                if (alpha < ALPHA_MIN) continue;
                const float testT = T * (1.0f - alpha);
                if (testT < T_STOP) {
                    done = 1;
                    break;
                }
                const float wgt = alpha * T;
                C0 += wgt * r.cc.z;
                C1 += wgt * r.cc.w;
                C2 += wgt * s_blue[j];
                if (wgt > wbest) {
                    wbest = wgt;
                    dom = s_id[j];
                }
                T = testT;
                last = b0 + (uint32_t)j;
                nc++;
            }
        }
    }

    double e = 0.0;
    if (inside) {
        const int64_t P = (int64_t)cam.W * cam.H;
        const int64_t pix = (int64_t)y * cam.W + x;
        const float r0 = C0 + T * cam.bg[0];
        const float r1 = C1 + T * cam.bg[1];
        const float r2 = C2 + T * cam.bg[2];
        image[pix] = r0;
        image[P + pix] = r1;
        image[2 * P + pix] = r2;
        t_final[pix] = T;
        last_out[pix] = last;
        ncontrib_out[pix] = nc;
        dom_out[pix] = dom;
        if (gt) {
            const double d0 = fabs((double)r0 - (double)gt[pix]);
            const double d1 = fabs((double)r1 - (double)gt[P + pix]);
            const double d2 = fabs((double)r2 - (double)gt[2 * P + pix]);
            e = (d0 + d1) + d2;
            err[pix] = e;
        }
    }
    if (gt) {
        // e >= 0, so the IEEE bit patterns order like the values
        const double emin = wave_min_d(inside ? e : __longlong_as_double(0x7ff0000000000000ll));
        const double emax = wave_max_d(inside ? e : 0.0);
        if (lane == 0) {
            atomicMin(&minmax[0], (unsigned long long)__double_as_longlong(emin));
            atomicMax(&minmax[1], (unsigned long long)__double_as_longlong(emax));
        }
    }
}

// Reverse pass.  For contributor k of a pixel with alpha a_k and transmittance
// T_k in front of it, dC/dc_k = a_k T_k and
//   dC/da_k = T_k (c_k - A_k) - T_final bg / (1 - a_k),
// where A_k is the colour composited behind k normalised by T_{k+1}; walking
// the list backwards from the last contributor restores T_k = T_{k+1}/(1-a_k)
// and A_k incrementally.  Gradients reach (o, conic, mean) only where
// alpha = o G is below the 0.99 clamp.  Each wave reduces its 64 pixels'
// gradients of a Gaussian before one set of atomics.
__global__ void __launch_bounds__(AS_BLOCK) k_blend_bwd(const uint32_t *__restrict__ ranges,
                                                        const uint32_t *__restrict__ vals,
                                                        const BlendRec *__restrict__ rec,
                                                        const short4 *__restrict__ box, DevCam cam, int tiles_x,
                                                        const float *__restrict__ t_final,
                                                        const uint32_t *__restrict__ last_in,
                                                        const uint32_t *__restrict__ ncontrib_in,
                                                        const float *__restrict__ dL_dimage, float *__restrict__ grad2d,
                                                        int64_t stride) {
    __shared__ StagedRec s_rec[AS_BLOCK];
    __shared__ float s_blue[AS_BLOCK];
    __shared__ int32_t s_id[AS_BLOCK];
    __shared__ uint32_t s_mask[AS_BLOCK];
    __shared__ uint32_t s_maxlast;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int tile = blockIdx.x;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int qx = (w & 1) * 8, qy = (w >> 1) * 8;
    const int lx = qx + (lane & 7), ly = qy + (lane >> 3);
    const int ox = tx * AS_TILE_W, oy = ty * AS_TILE_H;
    const int x = ox + lx, y = oy + ly;
    const bool inside = x < cam.W && y < cam.H;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const uint32_t qmx = 0xFFu << qx, qmy = (0xFFu << qy) << 16;
    const uint32_t start = ranges[2 * tile];

    const int64_t P = (int64_t)cam.W * cam.H;
    const int64_t pix = (int64_t)y * cam.W + x;
    float T = 1.0f, Tfin = 1.0f, dL0 = 0.f, dL1 = 0.f, dL2 = 0.f;
    uint32_t lastp = 0;
    bool has = false;
    if (inside) {
        Tfin = t_final[pix];
        T = Tfin;
        has = ncontrib_in[pix] > 0;
        lastp = last_in[pix];
        dL0 = dL_dimage[pix];
        dL1 = dL_dimage[P + pix];
        dL2 = dL_dimage[2 * P + pix];
    }
    const float bgdot = cam.bg[0] * dL0 + cam.bg[1] * dL1 + cam.bg[2] * dL2;
    if (tid == 0) s_maxlast = 0;
    __syncthreads();
    if (has) atomicMax(&s_maxlast, lastp + 1);
    __syncthreads();
    const uint32_t hi_end = s_maxlast > start ? s_maxlast : start;   // one past the block's last contributor
    // one past the wave's last contributor (wave-uniform)
    uint32_t wlast = has ? lastp + 1 : 0;
    for (int o = 32; o > 0; o >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, o, 64));

    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, last_alpha = 0.f, lc0 = 0.f, lc1 = 0.f, lc2 = 0.f;

    for (uint32_t b1 = hi_end; b1 > start;) {
        const uint32_t b0 = b1 - start > (uint32_t)AS_BLOCK ? b1 - AS_BLOCK : start;
        const uint32_t idx = b0 + tid;
        if (idx < b1) {
            const uint32_t id = vals[idx];
            StagedRec sr;
            float blue;
            uint32_t m;
            stage_record(rec, box, id, ox, oy, sr, blue, m);
            s_rec[tid] = sr;
            s_blue[tid] = blue;
            s_id[tid] = (int32_t)id;
            s_mask[tid] = m;
        }
        __syncthreads();
        for (int j = (int)(b1 - b0) - 1; j >= 0; j--) {
            const uint32_t gidx = b0 + (uint32_t)j;
            if (gidx >= wlast) continue;                        // beyond every pixel of this wave
            const uint32_t m = s_mask[j];
            if (!(m & qmx) || !(m & qmy)) continue;             // box misses this quadrant
            float g[9];
#pragma unroll
            for (int k = 0; k < 9; k++) g[k] = 0.f;
            bool contrib = false;
            if (has && gidx <= lastp && ((m >> lx) & (m >> (16 + ly)) & 1u)) {
                const StagedRec r = s_rec[j];
                const float dx = r.mc.x - px, dy = r.mc.y - py;
                const float araw = __builtin_amdgcn_exp2f(blend_exponent(dx, dy, r));
                const float alpha = fminf(ALPHA_MAX, araw);
                if (alpha >= ALPHA_MIN) {
                    contrib = true;
                    const float om = 1.0f - alpha;
                    T = T / om;
                    const float wgt = alpha * T;
                    const float c0 = r.cc.z, c1 = r.cc.w, c2 = s_blue[j];
                    acc0 = last_alpha * lc0 + (1.0f - last_alpha) * acc0;
                    acc1 = last_alpha * lc1 + (1.0f - last_alpha) * acc1;
                    acc2 = last_alpha * lc2 + (1.0f - last_alpha) * acc2;
                    lc0 = c0; lc1 = c1; lc2 = c2;
                    float dLda = (c0 - acc0) * dL0 + (c1 - acc1) * dL1 + (c2 - acc2) * dL2;
                    dLda *= T;
                    last_alpha = alpha;
                    dLda += (-Tfin / om) * bgdot;
                    g[6] = wgt * dL0;
                    g[7] = wgt * dL1;
                    g[8] = wgt * dL2;
                    if (araw < ALPHA_MAX) {
                        // alpha = o exp(p): dalpha/do = alpha/o, dalpha/dp = alpha;
                        // p = -(a dx^2 + c dy^2)/2 - b dx dy with the unscaled conic
                        const float o = exp2f(r.cc.y);
                        g[5] = dLda * araw / o;
                        const float dp = dLda * araw;
                        const float a = -2.0f * LN2 * r.mc.z, b = -LN2 * r.mc.w, c = -2.0f * LN2 * r.cc.x;
                        g[0] = dp * (-(a * dx + b * dy));
                        g[1] = dp * (-(c * dy + b * dx));
                        g[2] = dp * (-0.5f * dx * dx);
                        g[3] = dp * (-dx * dy);
                        g[4] = dp * (-0.5f * dy * dy);
                    }
                }
            }
            if (__ballot(contrib)) {
#pragma unroll
                for (int k = 0; k < 9; k++) g[k] = wave_sum(g[k]);
                if (lane == 0) {
                    const int64_t id = s_id[j];
#pragma unroll
                    for (int k = 0; k < 9; k++) atomicAdd(&grad2d[k * stride + id], g[k]);
                }
            }
        }
        __syncthreads();
        b1 = b0;
    }
}

}  // namespace

void launch_blend_fwd(const as_frame *f, const uint32_t *vals, const DevCam &cam, const float *gt, float *image,
                      hipStream_t s) {
    const int tiles = f->tiles_x * f->tiles_y;
    hipLaunchKernelGGL(k_blend_fwd, dim3(tiles), dim3(AS_BLOCK), 0, s, f->ranges, vals, f->rec,
                       reinterpret_cast<const short4 *>(f->box), cam, f->tiles_x, gt, image, f->t_final, f->last,
                       f->n_contrib, f->dom, f->err, reinterpret_cast<unsigned long long *>(f->err_minmax));
}

void launch_blend_bwd(const as_frame *f, const uint32_t *vals, const DevCam &cam, const float *dL_dimage,
                      float *grad2d, int64_t g2d_stride, hipStream_t s) {
    const int tiles = f->tiles_x * f->tiles_y;
    hipLaunchKernelGGL(k_blend_bwd, dim3(tiles), dim3(AS_BLOCK), 0, s, f->ranges, vals, f->rec,
                       reinterpret_cast<const short4 *>(f->box), cam, f->tiles_x, f->t_final, f->last, f->n_contrib,
                       dL_dimage, grad2d, g2d_stride);
}
