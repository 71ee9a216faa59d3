// Error region partitioning of one sampled view (Sec. 4.1): normalised L1 error
// (Eq. (l1map)), metric map, attribution counts, erosion, error bands, 8-connected
// regions of equal (dominant candidate, band) (Eq. (error-region)), the area
// filter (Eq. (min_region_area)) and the region statistics.
//
// Decision quantities (E, M, B, the region set and its integer moments) are
// computed in FP64 / exact integers; this file is compiled with
// -ffp-contract=off.  Connected components use a lock-free union-find whose
// roots are always the smallest pixel index of their component, so labels are
// canonical and independent of thread scheduling: first inside 16x16 tiles in
// LDS (fused with the classification and the erosion), then across tile
// borders in global memory.  Kept regions take their record slots from per-block
// counts scanned by one block, so records stay in ascending label order.
#include <mutex>

#include "internal.h"

namespace {

enum { ES_B, ES_LABEL, ES_MOM, ES_KEEP, ES_KIDX, ES_COUNT };

// Bytes of each scratch slot for a view of P pixels: bands, labels, the six
// integer moments per (root) pixel, keep flags, and two words per block of
// 256 pixels.
void es_need(int64_t P, size_t need[ES_COUNT]) {
    const size_t p = (size_t)(P > 0 ? P : 1);
    need[ES_B] = p;
    need[ES_LABEL] = p * 4;
    need[ES_MOM] = p * 48;
    need[ES_KEEP] = p;
    need[ES_KIDX] = (p + 255) / 256 * 8;
}

__device__ __forceinline__ double dev_bits_to_double(unsigned long long b) { return __longlong_as_double((long long)b); }

// Per-pixel L1 error and its range.  A bounded grid strides over the pixels
// and each block issues one pair of range atomics: device-wide atomics on the
// same two words serialise at the memory side, so there are few of them.
__global__ void __launch_bounds__(256) k_error_map(int W, int H, const float *__restrict__ img,
                                                   const float *__restrict__ gt, double *__restrict__ err,
                                                   unsigned long long *__restrict__ minmax) {
    __shared__ double s_mn[4], s_mx[4];
    const int64_t P = (int64_t)W * H;
    double mn = __longlong_as_double(0x7ff0000000000000ll), mx = 0.0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < P; u += (int64_t)gridDim.x * blockDim.x) {
        const double d0 = fabs((double)img[u] - (double)gt[u]);
        const double d1 = fabs((double)img[P + u] - (double)gt[P + u]);
        const double d2 = fabs((double)img[2 * P + u] - (double)gt[2 * P + u]);
        const double e = (d0 + d1) + d2;
        err[u] = e;
        mn = fmin(mn, e);
        mx = fmax(mx, e);
    }
    mn = wave_min_d(mn);
    mx = wave_max_d(mx);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_mn[w] = mn;
        s_mx[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; k++) {
            mn = fmin(mn, s_mn[k]);
            mx = fmax(mx, s_mx[k]);
        }
        atomicMin(&minmax[0], (unsigned long long)__double_as_longlong(mn));
        atomicMax(&minmax[1], (unsigned long long)__double_as_longlong(mx));
    }
}

// E = normalised error (Eq. (l1map)), M = [E > tau], band B = floor((E - tau) L / (1 - tau)) clamped to L - 1
__device__ __forceinline__ bool classify_px(double e, double emin, double emax, double tau, int L, uint8_t *band) {
    const double E = (emax == emin) ? 0.0 : (e - emin) / (emax - emin);
    const bool m = E > tau;
    uint8_t b = 0;
    if (m) {
        double bb = floor(((E - tau) * (double)L) / (1.0 - tau));
        if (bb > (double)(L - 1)) bb = (double)(L - 1);
        b = (uint8_t)bb;
    }
    *band = b;
    return m;
}

__device__ __forceinline__ int32_t uf_load(const int32_t *L, int32_t x) {
    return __hip_atomic_load(L + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t uf_find(const int32_t *L, int32_t x) {
    int32_t p = uf_load(L, x);
    while (p != x) {
        x = p;
        p = uf_load(L, x);
    }
    return x;
}

// Link the components of a and b; a root only ever points to a smaller index.
__device__ __forceinline__ void uf_unite(int32_t *L, int32_t a, int32_t b) {
    while (true) {
        a = uf_find(L, a);
        b = uf_find(L, b);
        if (a == b) return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicMin(L + a, b);
        if (old == a) return;
        a = old;
    }
}

// The same union-find on a block's LDS array.
__device__ __forceinline__ int lds_find(int32_t *L, int x) {
    int p = __hip_atomic_load(L + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (p != x) {
        x = p;
        p = __hip_atomic_load(L + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    return x;
}

__device__ __forceinline__ void lds_unite(int32_t *L, int a, int b) {
    while (true) {
        a = lds_find(L, a);
        b = lds_find(L, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(L + a, b);
        if (old == a) return;
        a = old;
    }
}

constexpr int ET = 16;      // pixel tile of the erosion / local components
constexpr int EMAX_R = 8;   // erosion radii up to this use an LDS tile with halo
constexpr int ES = ET + 2 * EMAX_R;

// M' = erosion of M with a square element of offsets [-lo, hi] per axis
// ((2r+1)^2: lo = hi = r; pixels outside the image count as set); active = M'
// and a candidate dominates the pixel.  Then the
// 8-connected components of equal (D, B) inside the block's 16x16 tile, with
// an LDS union-find whose roots are the smallest tile-local index, which is
// also the smallest image index of the tile's part of the component.  Writes
// label = image index of that root (-1 inactive).
__global__ void __launch_bounds__(ET * ET) k_erode_ccl_local(int W, int H, int tiles_x, int r, int lo, int hi,
                                                             const double *__restrict__ err,
                                                             const unsigned long long *__restrict__ minmax, double tau,
                                                             int L, const int32_t *__restrict__ dom,
                                                             uint8_t *__restrict__ B,
                                                             const uint8_t *__restrict__ is_cand,
                                                             int32_t *__restrict__ attr,
                                                             int32_t *__restrict__ label,
                                                             unsigned long long *__restrict__ mom) {
    __shared__ uint8_t s_m[ES * ES];
    __shared__ uint8_t s_row[ES * ET];
    __shared__ int32_t s_par[ET * ET];
    __shared__ int32_t s_dom[ET * ET];
    __shared__ uint8_t s_b[ET * ET];
    const int tid = threadIdx.x;
    const int tx = (int)blockIdx.x % tiles_x, ty = (int)blockIdx.x / tiles_x;
    const int ox = tx * ET, oy = ty * ET;
    const int lx = tid % ET, ly = tid / ET, x = ox + lx, y = oy + ly;
    const bool inside = x < W && y < H;
    const int64_t u = (int64_t)y * W + x;
    const double emin = dev_bits_to_double(minmax[0]), emax = dev_bits_to_double(minmax[1]);
    uint8_t scratch_band;
    // this pixel's class and band (written for the later passes), and the
    // attribution count before erosion: attr[D] += 1 per high-error pixel
    // dominated by a candidate, one atomic per wave when all hits share D
    uint8_t b = 0;
    const bool m_own = inside && classify_px(err[u], emin, emax, tau, L, &b);
    if (inside) B[u] = b;
    const int32_t d = inside ? dom[u] : -1;
    {
        const bool hit = m_own && d >= 0 && is_cand[d];
        const uint64_t hits = __ballot(hit);
        if (hits) {
            const int leader = __ffsll((unsigned long long)hits) - 1;
            const int32_t d0 = __shfl(d, leader, 64);
            const uint64_t same = __ballot(hit && d == d0);
            if (same == hits) {
                if ((int)__lane_id() == leader) atomicAdd(&attr[d0], (int32_t)__popcll(hits));
            } else if (hit) {
                atomicAdd(&attr[d], 1);
            }
        }
    }
    bool e;
    if (r <= EMAX_R) {   // lo, hi <= r
        const int S = ET + lo + hi;
        for (int i = tid; i < S * S; i += ET * ET) {
            const int hx = i % S, hy = i / S, gx = ox + hx - lo, gy = oy + hy - lo;
            s_m[i] = (gx < 0 || gy < 0 || gx >= W || gy >= H)
                         ? 1
                         : classify_px(err[(int64_t)gy * W + gx], emin, emax, tau, L, &scratch_band);
        }
        __syncthreads();
        for (int i = tid; i < S * ET; i += ET * ET) {   // AND along rows
            const int cx = i % ET, hy = i / ET;
            uint8_t a = 1;
            for (int k = 0; k <= lo + hi; k++) a &= s_m[hy * S + cx + k];
            s_row[i] = a;
        }
        __syncthreads();
        uint8_t a = 1;                                  // then along columns
        for (int k = 0; k <= lo + hi; k++) a &= s_row[(ly + k) * ET + lx];
        e = a != 0;
    } else {
        e = m_own;
        for (int dy = -lo; dy <= hi && e; dy++) {
            const int yy = y + dy;
            if (yy < 0 || yy >= H) continue;
            for (int dx = -lo; dx <= hi; dx++) {
                const int xx = x + dx;
                if (xx < 0 || xx >= W) continue;
                if (!classify_px(err[(int64_t)yy * W + xx], emin, emax, tau, L, &scratch_band)) {
                    e = false;
                    break;
                }
            }
        }
    }
    const bool active = inside && e && d >= 0 && is_cand[d];
    s_par[tid] = active ? tid : -1;
    s_dom[tid] = d;
    s_b[tid] = b;
    __syncthreads();
    if (active) {
        const int nx[4] = {-1, -1, 0, 1};
        const int ny[4] = {0, -1, -1, -1};
        for (int k = 0; k < 4; k++) {
            const int qx = lx + nx[k], qy = ly + ny[k];
            if (qx < 0 || qy < 0 || qx >= ET) continue;
            const int q = qy * ET + qx;
            if (s_par[q] < 0 || s_dom[q] != d || s_b[q] != b) continue;   // activity never changes here
            lds_unite(s_par, tid, q);
        }
    }
    __syncthreads();
    if (inside) {
        int32_t lab = -1;
        if (active) {
            const int rt = lds_find(s_par, tid);
            lab = (int32_t)((int64_t)(oy + rt / ET) * W + ox + rt % ET);
            // every component's final root (its smallest index) is the local
            // root of its part in that tile: the moments are cleared there
            if (rt == tid)
                for (int k = 0; k < 6; k++) mom[u * 6 + k] = 0ull;
        }
        label[u] = lab;
    }
}

// Join the tile-local components across tile borders: only pixels whose W,
// NW, N or NE neighbour lies in another tile link (a tile's top row, left
// and right columns: 3 ET - 2 pixels, one thread each), with the global
// union-find (roots are the smallest image index).
constexpr int ES_BORDER = 3 * ET - 2;
__global__ void k_ccl_border(int W, int H, int tiles_x, int64_t n_tiles, const int32_t *__restrict__ dom,
                             const uint8_t *__restrict__ B, int32_t *label) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tiles * ES_BORDER) return;
    const int64_t t = i / ES_BORDER;
    const int j = (int)(i - t * ES_BORDER);
    // j < ET: top row; then the left and the right column below it
    const int lx = j < ET ? j : (j < 2 * ET - 1 ? 0 : ET - 1);
    const int ly = j < ET ? 0 : (j < 2 * ET - 1 ? j - ET + 1 : j - 2 * ET + 2);
    const int x = (int)(t % tiles_x) * ET + lx, y = (int)(t / tiles_x) * ET + ly;
    if (x >= W || y >= H) return;
    const int64_t u = (int64_t)y * W + x;
    // a label's sign (active or not) never changes in this pass, only the
    // values of roots do: plain loads decide activity, the union-find reads
    // coherently
    const volatile int32_t *lv = label;
    if (lv[u] < 0) return;
    const int32_t d = dom[u];
    const uint8_t b = B[u];
    const int nx[4] = {-1, -1, 0, 1};
    const int ny[4] = {0, -1, -1, -1};
    for (int k = 0; k < 4; k++) {
        const int xx = x + nx[k], yy = y + ny[k];
        if (xx < 0 || yy < 0 || xx >= W) continue;
        if (xx / ET == x / ET && yy / ET == y / ET) continue;   // joined by the local pass
        const int64_t q = (int64_t)yy * W + xx;
        if (dom[q] != d || B[q] != b || lv[q] < 0) continue;
        uf_unite(label, (int32_t)u, (int32_t)q);
    }
}

// Exact integer moments A, Sx, Sy, Sxx, Sxy, Syy per component, stored at the
// component's root pixel (the end of the pixel's parent chain: the labels no
// longer change, so plain loads follow it).
__global__ void k_moments(int W, int H, const int32_t *__restrict__ label, unsigned long long *__restrict__ mom) {
    const int64_t P = (int64_t)W * H;
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t s = -1;
    int64_t v[6] = {0, 0, 0, 0, 0, 0};
    if (u < P) {
        int32_t l = label[u];
        if (l >= 0) {
            for (int32_t p = label[l]; p != l; p = label[l]) l = p;
            s = l;
            const int64_t x = u % W, y = u / W;
            v[0] = 1; v[1] = x; v[2] = y; v[3] = x * x; v[4] = x * y; v[5] = y * y;
        }
    }
    // one set of atomics per distinct region among the wave's 64 pixels (a
    // wave spans one image row segment, which few regions cross)
    uint64_t pending = __ballot(s >= 0);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int64_t s0 = __shfl(s, leader, 64);
        const bool mine = s == s0;
        pending &= ~__ballot(mine);
        int64_t t[6];
#pragma unroll
        for (int k = 0; k < 6; k++) {
            t[k] = mine ? v[k] : 0;
            for (int o = 32; o > 0; o >>= 1) t[k] += __shfl_xor(t[k], o, 64);
        }
        if ((int)__lane_id() == leader)
            for (int k = 0; k < 6; k++) atomicAdd(&mom[s0 * 6 + k], (unsigned long long)t[k]);
    }
}

// A component is kept (Eq. (min_region_area)) at its root pixel.
// Kept components (roots with area >= m_min) and the number per block of 256
// pixels.
__global__ void __launch_bounds__(256) k_region_keep(int64_t P, const int32_t *__restrict__ label,
                                                     const unsigned long long *__restrict__ mom, int m_min,
                                                     uint8_t *__restrict__ keep, int64_t *__restrict__ part) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool k = u < P && label[u] == (int32_t)u && (int64_t)mom[u * 6] >= (int64_t)m_min;
    if (u < P) keep[u] = k;
    const int c = __syncthreads_count(k);
    if (threadIdx.x == 0) part[blockIdx.x] = c;
}

// One block: the per-block counts become the first record slot of each
// block (after the records already in the buffer), and the buffer's count
// advances by the total.
__global__ void __launch_bounds__(1024) k_region_slots(int64_t *__restrict__ part, int64_t nblk,
                                                       int64_t *__restrict__ count) {
    __shared__ int64_t s_w[16];
    __shared__ int64_t s_carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_carry = *count;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nblk; b0 += 1024) {
        const int64_t b = b0 + tid;
        const int64_t v = b < nblk ? part[b] : 0;
        int64_t inc = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (lane == 63) s_w[w] = inc;
        __syncthreads();
        int64_t pre = s_carry;
        for (int k = 0; k < w; k++) pre += s_w[k];
        if (b < nblk) part[b] = pre + inc - v;
        __syncthreads();
        if (tid == 1023) s_carry = pre + inc;
        __syncthreads();
    }
    if (tid == 0) *count = s_carry;
}

__device__ __forceinline__ double central_moment(int64_t A, int64_t sab, int64_t sa, int64_t sb) {
    const __int128 num = (__int128)A * sab - (__int128)sa * sb;
    double dnum;
    if (num >= (__int128)INT64_MIN && num <= (__int128)INT64_MAX) dnum = (double)(int64_t)num;
    else dnum = (double)num;
    const double dA = (double)A;
    return dnum / (dA * dA);
}

// One record per kept component, in ascending label order: a block's first
// slot (k_region_slots) plus the kept pixels before this one in the block.
__global__ void __launch_bounds__(256) k_region_emit(int W, int H, int view, const unsigned long long *__restrict__ mom,
                                                     const uint8_t *__restrict__ keep, const int64_t *__restrict__ slot,
                                                     const int32_t *__restrict__ dom, const uint8_t *__restrict__ B,
                                                     const float *__restrict__ gt, as_region *__restrict__ out,
                                                     int64_t out_cap) {
    __shared__ int s_w[4];
    const int64_t P = (int64_t)W * H;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool k = s < P && keep[s];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t bal = __ballot(k);
    if (lane == 0) s_w[w] = __popcll(bal);
    __syncthreads();
    int before = __popcll(bal & ((1ull << lane) - 1ull));
    for (int q = 0; q < w; q++) before += s_w[q];
    if (!k) return;
    const int64_t pos = slot[blockIdx.x] + before;
    if (pos >= out_cap) return;
    as_region r;
    const int32_t root = (int32_t)s;
    r.cand = dom[root];
    r.view = view;
    r.label = root;
    r.band = B[root];
    r.pad0 = 0;
    const int64_t A = (int64_t)mom[s * 6 + 0];
    r.area = (int32_t)A;
    r.sx = (int64_t)mom[s * 6 + 1];
    r.sy = (int64_t)mom[s * 6 + 2];
    r.sxx = (int64_t)mom[s * 6 + 3];
    r.sxy = (int64_t)mom[s * 6 + 4];
    r.syy = (int64_t)mom[s * 6 + 5];
    const double dA = (double)A;
    r.cx = (double)r.sx / dA + 0.5;
    r.cy = (double)r.sy / dA + 0.5;
    const double cxx = central_moment(A, r.sxx, r.sx, r.sx) + 1.0 / 12.0;
    const double cxy = central_moment(A, r.sxy, r.sx, r.sy);
    const double cyy = central_moment(A, r.syy, r.sy, r.sy) + 1.0 / 12.0;
    r.cov[0] = cxx;
    r.cov[1] = cxy;
    r.cov[2] = cyy;
    const double half_tr = 0.5 * (cxx + cyy);
    const double half_dif = 0.5 * (cxx - cyy);
    const double disc = sqrt(half_dif * half_dif + cxy * cxy);
    const double l1 = half_tr + disc, l2 = half_tr - disc;
    double ex, ey;
    if (disc == 0.0) {
        ex = 1.0; ey = 0.0;
    } else if (half_dif >= 0.0) {
        ex = half_dif + disc; ey = cxy;
    } else {
        ex = cxy; ey = -half_dif + disc;
    }
    const double en = sqrt(ex * ex + ey * ey);
    ex = ex / en;
    ey = ey / en;
    if (ex < 0.0 || (ex == 0.0 && ey < 0.0)) {
        ex = -ex;
        ey = -ey;
    }
    r.e1[0] = ex;
    r.e1[1] = ey;
    r.sigma1 = sqrt(l1);
    r.sigma2 = sqrt(l2 > 0.0 ? l2 : 0.0);
    const int64_t gx = (int64_t)floor(r.cx), gy = (int64_t)floor(r.cy);
    for (int ch = 0; ch < 3; ch++) r.rgb[ch] = gt[ch * P + gy * W + gx];
    r.pad1 = 0.f;
    out[pos] = r;
}


}  // namespace

void launch_error_map(int W, int H, const float *image, const float *gt, double *err, uint64_t *minmax, hipStream_t s) {
    const int64_t P = (int64_t)W * H;
    launch_fill_u64(minmax, 0x7ff0000000000000ull, 1, s);
    launch_fill_u64(minmax + 1, 0ull, 1, s);
    if (P == 0) return;
    int64_t g = (P + 255) / 256;
    if (g > 512) g = 512;
    hipLaunchKernelGGL(k_error_map, dim3((unsigned)g), dim3(256), 0, s, W, H, image, gt, err,
                       reinterpret_cast<unsigned long long *>(minmax));
}

size_t errstats_reserve_bytes(int64_t max_pixels) {
    if (max_pixels <= 0) return 0;
    size_t need[ES_COUNT], total = 0;
    es_need(max_pixels, need);
    for (int k = 0; k < ES_COUNT; k++) total += devbuf_size(need[k]);
    return total;
}

hipError_t errstats_reserve(as_ctx *ctx, int64_t max_pixels) {
    if (max_pixels <= 0) return hipSuccess;
    size_t need[ES_COUNT];
    es_need(max_pixels, need);
    hipError_t e = hipSuccess;
    for (int k = 0; k < ES_COUNT && e == hipSuccess; k++) e = devbuf_ensure(ctx->es[k], need[k]);
    return e;
}

namespace {
// The scratch of one error-statistics call (slots of es_need).
struct EsScratch {
    uint8_t *B;
    int32_t *label;
    unsigned long long *mom;
    uint8_t *keep;
    int64_t *kidx;   // per block of 256 pixels: kept roots, then first record slot
};

void es_launch(const EsScratch &sc, int W, int H, const double *err, const uint64_t *minmax, const int32_t *dom,
               const float *gt, int view, const uint8_t *is_cand, const as_split_params &p, as_region_buf &rb,
               int32_t *attr, hipStream_t s);
}  // namespace

as_status run_error_stats(as_ctx *ctx, int W, int H, const double *err, const uint64_t *minmax, const int32_t *dom,
                          const float *gt, int view, int64_t n, const uint8_t *is_cand, const as_split_params &p,
                          as_region_buf &rb, int32_t *attr, hipStream_t s) {
    (void)n;
    const int64_t P = (int64_t)W * H;
    if (P == 0) return AS_OK;
    if (P > ctx->res.max_pixels) {
        as_set_error("as_accumulate_error_stats: a %dx%d view needs max_pixels >= %lld in as_ctx_reserve (reserved "
                     "%lld)", W, H, (long long)P, (long long)ctx->res.max_pixels);
        return AS_ERR_CAPACITY;
    }
    DevBuf *es = ctx->es;
    const EsScratch sc{(uint8_t *)es[ES_B].p, (int32_t *)es[ES_LABEL].p, (unsigned long long *)es[ES_MOM].p,
                       (uint8_t *)es[ES_KEEP].p, (int64_t *)es[ES_KIDX].p};
    es_launch(sc, W, H, err, minmax, dom, gt, view, is_cand, p, rb, attr, s);
    return AS_OK;
}

// ---- the no-allocation variant ------------------------------------------------------
//
// For callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid hipMalloc): the same kernels with their
// scratch in one static device array, sized for views of up to
// AS_NOALLOC_MAX_PIXELS pixels.  The runtime gives every device its own copy
// of the array (held until the process ends); its address on a device is taken
// once, with that device current, when a context is created there
// (errstats_noalloc_init), and the kernels receive that address.  In host code
// the array's name is no device address, so it is never passed to a kernel.
// Every call on a device shares the one array: calls on that device must not
// overlap (they would race on it).  Nothing in it needs clearing: each kernel
// writes a slot before any kernel of the same call reads it.
namespace {
constexpr size_t es_slot(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
constexpr size_t ES_NA_PIX = (size_t)AS_NOALLOC_MAX_PIXELS;
constexpr size_t ES_NA_OFF_LABEL = es_slot(ES_NA_PIX);
constexpr size_t ES_NA_OFF_MOM = ES_NA_OFF_LABEL + es_slot(ES_NA_PIX * 4);
constexpr size_t ES_NA_OFF_KEEP = ES_NA_OFF_MOM + es_slot(ES_NA_PIX * 48);
constexpr size_t ES_NA_OFF_KIDX = ES_NA_OFF_KEEP + es_slot(ES_NA_PIX);
constexpr size_t ES_NA_BYTES = ES_NA_OFF_KIDX + es_slot((ES_NA_PIX + 255) / 256 * 8);
constexpr int ES_NA_MAX_DEVICES = 64;

std::mutex g_na_mutex;
unsigned char *g_na_ptr[ES_NA_MAX_DEVICES];   // the array's address on each device
}  // namespace

static __device__ __align__(256) unsigned char scratch[ES_NA_BYTES];

hipError_t errstats_noalloc_init(int device) {
    if (device < 0 || device >= ES_NA_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (g_na_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_na_ptr[device] = (unsigned char *)ptr;
    return hipSuccess;
}

size_t errstats_noalloc_bytes() { return ES_NA_BYTES; }

as_status run_error_stats_noalloc(as_ctx *ctx, int W, int H, const double *err, const uint64_t *minmax,
                                  const int32_t *dom, const float *gt, int view, const uint8_t *is_cand,
                                  const as_split_params &p, as_region_buf &rb, int32_t *attr, hipStream_t s) {
    const int64_t P = (int64_t)W * H;
    if (P > (int64_t)AS_NOALLOC_MAX_PIXELS) {
        as_set_error("as_accumulate_error_stats_noalloc: a %dx%d view has %lld pixels, above the static scratch's "
                     "maximum of %lld", W, H, (long long)P, (long long)AS_NOALLOC_MAX_PIXELS);
        return AS_ERR_CAPACITY;
    }
    if (P == 0) return AS_OK;
    unsigned char *base = nullptr;
    if (ctx->device >= 0 && ctx->device < ES_NA_MAX_DEVICES) {
        std::lock_guard<std::mutex> lock(g_na_mutex);
        base = g_na_ptr[ctx->device];
    }
    if (!base) {
        as_set_error("as_accumulate_error_stats_noalloc: no static scratch address for device %d", ctx->device);
        return AS_ERR_STATE;
    }
    const EsScratch sc{base, (int32_t *)(base + ES_NA_OFF_LABEL), (unsigned long long *)(base + ES_NA_OFF_MOM),
                       base + ES_NA_OFF_KEEP, (int64_t *)(base + ES_NA_OFF_KIDX)};
    es_launch(sc, W, H, err, minmax, dom, gt, view, is_cand, p, rb, attr, s);
    return AS_OK;
}

namespace {
void es_launch(const EsScratch &sc, int W, int H, const double *err, const uint64_t *minmax, const int32_t *dom,
               const float *gt, int view, const uint8_t *is_cand, const as_split_params &p, as_region_buf &rb,
               int32_t *attr, hipStream_t s) {
    const int64_t P = (int64_t)W * H;
    uint8_t *B = sc.B;
    uint8_t *keep = sc.keep;
    int32_t *label = sc.label;
    int64_t *kidx = sc.kidx;
    unsigned long long *mom = sc.mom;
    const unsigned grid = (unsigned)((P + 255) / 256);
    const int tiles_x = (W + ET - 1) / ET, tiles = tiles_x * ((H + ET - 1) / ET);

    // element offsets: [-r, r] per axis, or a side of r + 1 (flag)
    const int lo = (p.flags & AS_SPLIT_ERODE_SIDE) ? p.r_erode / 2 : p.r_erode;
    const int hi = (p.flags & AS_SPLIT_ERODE_SIDE) ? p.r_erode - p.r_erode / 2 : p.r_erode;
    // classification, attribution, erosion and the tile-local components in one pass
    hipLaunchKernelGGL(k_erode_ccl_local, dim3(tiles), dim3(ET * ET), 0, s, W, H, tiles_x, p.r_erode, lo, hi, err,
                       reinterpret_cast<const unsigned long long *>(minmax), p.tau_l1, p.L, dom, B, is_cand, attr,
                       label, mom);
    const int64_t nb = ((int64_t)tiles * ES_BORDER + 255) / 256;
    hipLaunchKernelGGL(k_ccl_border, dim3((unsigned)nb), dim3(256), 0, s, W, H, tiles_x, (int64_t)tiles, dom, B,
                       label);
    hipLaunchKernelGGL(k_moments, dim3(grid), dim3(256), 0, s, W, H, label, mom);
    // kept roots, one record slot per block (advancing the buffer's count), records
    hipLaunchKernelGGL(k_region_keep, dim3(grid), dim3(256), 0, s, P, label, mom, p.m_min, keep, kidx);
    hipLaunchKernelGGL(k_region_slots, dim3(1), dim3(1024), 0, s, kidx, (int64_t)grid, rb.count);
    hipLaunchKernelGGL(k_region_emit, dim3(grid), dim3(256), 0, s, W, H, view, mom, keep, kidx, dom, B, gt,
                       rb.records, rb.capacity);
}
}  // namespace

AS_WARM_KERNEL(errstats)
