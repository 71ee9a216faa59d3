// EWA projection, spherical-harmonic colour, depth key and compact box of every
// Gaussian (Sec. 3 of the paper: each Gaussian is projected to the image plane
// and its view-dependent colour decoded from SH along the viewing direction).
//
// One thread per (view, Gaussian) entry, struct-of-arrays reads (coalesced);
// blocks alternate over the views of a batch (view index fastest), so the
// views of one chunk of Gaussians read its parameters while they are still in
// L2.  All arithmetic
// is FP64 and this file is compiled with -ffp-contract=off: the depth key and
// the pixel box decide which (tile, Gaussian) pairs exist, so they are
// computed with a fixed expression order and IEEE-rounded operations.
#include "internal.h"
#include "sh_device.h"

namespace {

__device__ __forceinline__ void quat_to_rot_d(double w, double x, double y, double z, double R[9]) {
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

template <int DEG, bool BUF>
__global__ void __launch_bounds__(256) k_project(const SceneTable sc, const ViewTable vt, BlendRec *__restrict__ rec,
                                                 uint32_t *__restrict__ depth_key, short4 *__restrict__ box,
                                                 uint32_t *__restrict__ ntiles, uint32_t *__restrict__ sort_keys,
                                                 uint32_t *__restrict__ sort_vals, uint32_t *__restrict__ n_ent) {
    const int v = (int)(blockIdx.x % (unsigned)vt.n_views);
    const int64_t i = (int64_t)(blockIdx.x / (unsigned)vt.n_views) * blockDim.x + threadIdx.x;
    const GaussPtrs &g = sc.g[v];
    const DevCam &cam = vt.cam[v];
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_ent = (uint32_t)vt.ent_base[vt.n_views];
    if (i >= g.n) return;
    const int64_t n = g.n;
    const uint32_t bo = (uint32_t)i * 4u;   // the lane's byte offset in every parameter row
    const int64_t e = (int64_t)vt.ent_base[v] + i;
    double mu[3], s[3], q[4];
    for (int k = 0; k < 3; k++) mu[k] = (double)at_row(g.means, k, n, bo);
    for (int k = 0; k < 3; k++) s[k] = exp((double)at_row(g.log_scales, k, n, bo));
    for (int k = 0; k < 4; k++) q[k] = (double)at_row(g.quats, k, n, bo);
    const double ologit = (double)g.opac[i];

    double Rc[9], tc[3];
    for (int k = 0; k < 9; k++) Rc[k] = (double)cam.R[k];
    for (int k = 0; k < 3; k++) tc[k] = (double)cam.t[k];
    const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;

    double tv[3];
    for (int r = 0; r < 3; r++) tv[r] = Rc[r * 3 + 0] * mu[0] + Rc[r * 3 + 1] * mu[1] + Rc[r * 3 + 2] * mu[2] + tc[r];
    const double tx = tv[0], ty = tv[1], tz = tv[2];
    // the depth key, also as the (key, entry) input of the depth sort
    const uint32_t dk = __float_as_uint((float)tz);
    depth_key[e] = dk;
    sort_keys[e] = dk;
    sort_vals[e] = (uint32_t)e;

    BlendRec rr;
    rr.m = make_float4(0.f, 0.f, 0.f, 0.f);
    rr.c = make_float4(0.f, 0.f, 0.f, 0.f);
    rr.rgb = make_float4(0.f, 0.f, 0.f, 0.f);
    short4 bx = make_short4(0, 0, -1, -1);
    uint32_t nt = 0;

    do {
        if (!(tz > AS_NEAR)) break;
        // The SH coefficients are loaded here, so their latency overlaps the
        // covariance and box arithmetic below (an entry culled after this
        // point has read them for nothing; in front of the camera few are).
        // One buffer resource over the array with the row's byte offset a
        // scalar, when every row offset fits 32 bits, else 64-bit row addresses.
        constexpr int nk = (DEG + 1) * (DEG + 1);
        float shv[nk * 3];
        if constexpr (BUF) {
            const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(g.sh), (short)0, -1,
                                                                                AS_BUFFER_RSRC_WORD3);
#pragma unroll
            for (int k = 0; k < nk * 3; k++)
                shv[k] = __uint_as_float(
                    __builtin_amdgcn_raw_buffer_load_b32(r, (int)bo, (int)((uint32_t)k * (uint32_t)n * 4u), 0));
        } else {
#pragma unroll
            for (int k = 0; k < nk * 3; k++) shv[k] = at_row(g.sh, k, n, bo);
        }
        __asm__ __volatile__("" ::: "memory");   // the loads are issued here, not next to their use
        const double qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        const double qnorm = sqrt(qn2);
        double Rg[9];
        quat_to_rot_d(q[0] / qnorm, q[1] / qnorm, q[2] / qnorm, q[3] / qnorm, Rg);
        // perspective Jacobian at the (clamped) centre
        const double limx = 1.3 * ((double)cam.W / (2.0 * fx));
        const double limy = 1.3 * ((double)cam.H / (2.0 * fy));
        const double txtz = tx / tz, tytz = ty / tz;
        const double cx_ = fmin(limx, fmax(-limx, txtz)) * tz;
        const double cy_ = fmin(limy, fmax(-limy, tytz)) * tz;
        const double J[6] = {fx / tz, 0.0, -(fx * cx_) / (tz * tz), 0.0, fy / tz, -(fy * cy_) / (tz * tz)};
        double T[6];
        for (int r = 0; r < 2; r++)
            for (int k = 0; k < 3; k++)
                T[r * 3 + k] = J[r * 3 + 0] * Rc[0 * 3 + k] + J[r * 3 + 1] * Rc[1 * 3 + k] + J[r * 3 + 2] * Rc[2 * 3 + k];
        double S[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0.0;
                for (int k = 0; k < 3; k++) acc += Rg[a * 3 + k] * (s[k] * s[k]) * Rg[b * 3 + k];
                S[a * 3 + b] = acc;
            }
        double C2[4];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                double acc = 0.0;
                for (int k = 0; k < 3; k++)
                    for (int l = 0; l < 3; l++) acc += T[a * 3 + k] * S[k * 3 + l] * T[b * 3 + l];
                C2[a * 2 + b] = acc;
            }
        const double A = C2[0] + AS_LOWPASS, B = C2[1], Cc = C2[3] + AS_LOWPASS;
        const double det = A * Cc - B * B;
        // The culling tests below are taken together after the colour, so
        // the code from the SH loads to the end is one block: the compiler
        // neither sinks the loads to their use nor splits the arithmetic
        // around them (a culled entry computes NaNs or values it discards).
        const double mx = fx * tx / tz + cx;
        const double my = fy * ty / tz + cy;
        const double o = 1.0 / (1.0 + exp(-ologit));
        const double kk = 2.0 * log(255.0 * o);
        const double hx = sqrt(kk * A), hy = sqrt(kk * Cc);
        double x0 = ceil(mx - hx - 0.5), x1 = floor(mx + hx - 0.5);
        double y0 = ceil(my - hy - 0.5), y1 = floor(my + hy - 0.5);
        x0 = fmax(x0, 0.0); y0 = fmax(y0, 0.0);
        x1 = fmin(x1, (double)(cam.W - 1)); y1 = fmin(y1, (double)(cam.H - 1));
        const bool keep = det > 0.0 && o >= (1.0 / 255.0) && x0 <= x1 && y0 <= y1;

        // colour along the unit view direction
        double oc[3];
        for (int j = 0; j < 3; j++) oc[j] = -(Rc[0 * 3 + j] * tc[0] + Rc[1 * 3 + j] * tc[1] + Rc[2 * 3 + j] * tc[2]);
        const double v0 = mu[0] - oc[0], v1 = mu[1] - oc[1], v2 = mu[2] - oc[2];
        const double vn = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
        double Y[16];
        sh_eval_basis(v0 / vn, v1 / vn, v2 / vn, DEG, Y);
        double col[3];
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < nk; k++) acc += Y[k] * (double)shv[k * 3 + ch];
            acc += 0.5;
            col[ch] = acc < 0.0 ? 0.0 : acc;
        }
        // The colour is masked with a lane mask the compiler cannot see
        // through (a select would be turned back into a branch around the
        // colour), so its loads and arithmetic stay in this block; a culled
        // entry keeps exact zeros.
        uint32_t km = keep ? 0xFFFFFFFFu : 0u;
        __asm__ __volatile__("" : "+v"(km));
        rr.rgb = make_float4(__uint_as_float(__float_as_uint((float)col[0]) & km),
                             __uint_as_float(__float_as_uint((float)col[1]) & km),
                             __uint_as_float(__float_as_uint((float)col[2]) & km), 0.f);
        if (!keep) break;

        const float mxh = (float)mx, myh = (float)my;
        rr.m = make_float4(mxh, myh, (float)(mx - (double)mxh), (float)(my - (double)myh));
        rr.c = make_float4((float)(Cc / det), (float)(-B / det), (float)(A / det), (float)o);
        const int ix0 = (int)x0, iy0 = (int)y0, ix1 = (int)x1, iy1 = (int)y1;
        bx = make_short4((short)ix0, (short)iy0, (short)ix1, (short)iy1);
        const int bs = vt.bin_shift;   // bins touched (the box lies in the image: no negative coordinates)
        nt = (uint32_t)(((ix1 >> bs) - (ix0 >> bs) + 1) * ((iy1 >> bs) - (iy0 >> bs) + 1));
    } while (0);

    rec[e] = rr;
    box[e] = bx;
    ntiles[e] = nt;
}

}  // namespace

void launch_project(const SceneTable &sc, const ViewTable &vt, int64_t max_n, int deg, BlendRec *rec,
                    uint32_t *depth_key, int16_t *box, uint32_t *ntiles, uint32_t *sort_keys, uint32_t *sort_vals,
                    uint32_t *n_ent, hipStream_t s, bool force_addr64) {
    if (max_n == 0 || vt.n_views == 0) {
        launch_fill_u32(n_ent, 0u, 1, s);
        return;
    }
    const int64_t blocks = (max_n + 255) / 256 * vt.n_views;
    short4 *b4 = reinterpret_cast<short4 *>(box);
    // buffer addressing of the SH rows when the last row's byte offset fits 32 bits
    const bool buf = !force_addr64 && 3 * (int64_t)(deg + 1) * (deg + 1) * max_n * 4 <= (int64_t)UINT32_MAX;
#define AS_PRJ(D)                                                                                                  \
    do {                                                                                                           \
        if (buf) hipLaunchKernelGGL((k_project<D, true>), dim3((unsigned)blocks), dim3(256), 0, s, sc, vt, rec,    \
                                    depth_key, b4, ntiles, sort_keys, sort_vals, n_ent);                          \
        else hipLaunchKernelGGL((k_project<D, false>), dim3((unsigned)blocks), dim3(256), 0, s, sc, vt, rec,       \
                                depth_key, b4, ntiles, sort_keys, sort_vals, n_ent);                              \
    } while (0)
    switch (deg) {
    case 0: AS_PRJ(0); break;
    case 1: AS_PRJ(1); break;
    case 2: AS_PRJ(2); break;
    default: AS_PRJ(3); break;
    }
#undef AS_PRJ
}

AS_WARM_KERNEL(project)
