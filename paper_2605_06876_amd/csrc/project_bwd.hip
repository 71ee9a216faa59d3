// Reverse pass of the projection (Sec. 3): from the per-entry 2D gradients
// (mean, conic, opacity, colour) accumulated by the blend back to the stored
// parameters (means, log-scales, quaternions, opacity logits, SH).  One thread
// per Gaussian, FP64, struct-of-arrays reads and writes.  A batch of views is
// one launch: each thread walks the views in order and sums their
// contributions (a fixed order, so the sum is deterministic), then writes
// every gradient once; a single view uses a leaner kernel with the same
// arithmetic.
//
// Chain: colour = max(0, sum_k Y_k(d) sh_k + 1/2) with d = (mu - o_v)/|mu - o_v|;
// mean2d = (fx tx/tz + cx, fy ty/tz + cy); conic = inverse(J W Sigma W^T J^T
// + 0.3 I) with J the perspective Jacobian at the clamped centre; Sigma =
// R(q/|q|) diag(exp(2 log s)) R^T; o = sigmoid(logit).  The scale and
// rotation gradients are linear in dL/dSigma, so dL/dSigma is summed over the
// views first and mapped to (log s, q) once.
#include "internal.h"
#include "sh_device.h"

namespace {

// SH rows of the single-view kernel.  With BUF (every row offset of the
// array below 2^32 bytes: 48 rows of fewer than 22M Gaussians) a row is read
// and written through one buffer resource over the array, the row's byte
// offset a scalar and the lane's offset the one vector operand shared by all
// rows; otherwise through at_row.  A 64-bit address per row would be held in
// vector registers otherwise: the 48 rows' reads and writes took the kernel
// to 239 VGPRs, two waves per SIMD.
template <bool BUF>
__device__ __forceinline__ float sh_ld(const float *a, int row, int64_t n, uint32_t bo) {
    if constexpr (BUF) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(a), (short)0, -1,
                                                                            AS_BUFFER_RSRC_WORD3);
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)bo, (int)((uint32_t)row * (uint32_t)n * 4u), 0));
    } else {
        return at_row(a, row, n, bo);
    }
}
template <bool BUF>
__device__ __forceinline__ void sh_st(float *a, int row, int64_t n, uint32_t bo, float v) {
    if constexpr (BUF) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(a, (short)0, -1, AS_BUFFER_RSRC_WORD3);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)bo, (int)((uint32_t)row * (uint32_t)n * 4u), 0);
    } else {
        at_row(a, row, n, bo) = v;
    }
}

// One view: the form that keeps the fewest values live, used when a render
// has one view.
template <int DEG, bool BUF>
__global__ void __launch_bounds__(256) k_project_bwd_view(GaussPtrs g, DevCam cam, const uint32_t *__restrict__ ntiles,
                                                     const float *__restrict__ g2d, GradPtrs out,
                                                     float *__restrict__ g2d_norm, int32_t *__restrict__ vis_count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const int64_t n = g.n, os = out.stride;
    const uint32_t bo = (uint32_t)i * 4u;   // the lane's byte offset in every row (n < 2^30)
    constexpr int nk = (DEG + 1) * (DEG + 1);
    if (ntiles[i] == 0) {
        for (int k = 0; k < 3; k++) { at_row(out.means, k, os, bo) = 0.f; at_row(out.log_scales, k, os, bo) = 0.f; }
        for (int k = 0; k < 4; k++) at_row(out.quats, k, os, bo) = 0.f;
        out.opac[i] = 0.f;
#pragma unroll
        for (int k = 0; k < nk * 3; k++) sh_st<BUF>(out.sh, k, os, bo, 0.f);
        return;
    }
    // The colour part first, from the mean and the colour gradient alone, and
    // a compiler barrier before the rest is loaded: the geometry's inputs and
    // intermediates are not held in registers across the SH loops (together
    // they needed 236 VGPRs, two waves per SIMD).
    double mu[3];
    for (int k = 0; k < 3; k++) mu[k] = (double)at_row(g.means, k, n, bo);
    double Rc[9], tc[3];
    for (int k = 0; k < 9; k++) Rc[k] = (double)cam.R[k];
    for (int k = 0; k < 3; k++) tc[k] = (double)cam.t[k];
    double dmu[3];
    {
        const double grgb[3] = {g2d[i * 9 + 6], g2d[i * 9 + 7], g2d[i * 9 + 8]};
        // colour and view direction
        double oc[3];
        for (int j = 0; j < 3; j++) oc[j] = -(Rc[0 * 3 + j] * tc[0] + Rc[1 * 3 + j] * tc[1] + Rc[2 * 3 + j] * tc[2]);
        const double v[3] = {mu[0] - oc[0], mu[1] - oc[1], mu[2] - oc[2]};
        const double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const double d[3] = {v[0] / vn, v[1] / vn, v[2] / vn};
        double Y[16];
        sh_eval_basis(d[0], d[1], d[2], DEG, Y);
        // One pass over the coefficients: per channel the raw colour
        // sum_k Y_k sh_k (its clamp decides whether the channel's gradient
        // passes) and the gradient of that sum with respect to the direction,
        // G_ch = sum_k sh_k dY_k (the terms of sh_weighted_grad).  The
        // direction gradient is then sum_ch gc_ch G_ch, the same sum as
        // sum_k (sum_ch sh_k gc_ch) dY_k regrouped, so the coefficients are not
        // read a second time (a second read missed L2 and cost about 100 MB of
        // HBM traffic per C2 launch).
        double gc[3], gd[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            double shc[16], raw = 0.0;
#pragma unroll
            for (int k = 0; k < nk; k++) {
                shc[k] = (double)sh_ld<BUF>(g.sh, k * 3 + ch, n, bo);
                raw += Y[k] * shc[k];
            }
            double gch[3];
            sh_weighted_grad(d[0], d[1], d[2], DEG, shc, gch);
            gc[ch] = raw + 0.5 < 0.0 ? 0.0 : grgb[ch];
            for (int a = 0; a < 3; a++) gd[a] += gc[ch] * gch[a];
        }
#pragma unroll
        for (int k = 0; k < nk; k++)
#pragma unroll
            for (int ch = 0; ch < 3; ch++) sh_st<BUF>(out.sh, k * 3 + ch, os, bo, (float)(Y[k] * gc[ch]));
        const double ddot = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
        for (int a = 0; a < 3; a++) dmu[a] = (gd[a] - d[a] * ddot) / vn;
    }
    // the colour part's result is an operand of the barrier, so its arithmetic
    // finishes before the geometry's loads, which the barrier holds after it
    __asm__ __volatile__("" : "+v"(dmu[0]), "+v"(dmu[1]), "+v"(dmu[2]) : : "memory");

    const double gm0 = g2d[i * 9 + 0], gm1 = g2d[i * 9 + 1];
    const double gca = g2d[i * 9 + 2], gcb = g2d[i * 9 + 3], gcc = g2d[i * 9 + 4];
    const double gop = g2d[i * 9 + 5];
    if (g2d_norm) g2d_norm[i] += (float)sqrt(gm0 * gm0 + gm1 * gm1);
    if (vis_count) vis_count[i] += 1;
    double s[3], q[4];
    for (int k = 0; k < 3; k++) s[k] = exp((double)at_row(g.log_scales, k, n, bo));
    for (int k = 0; k < 4; k++) q[k] = (double)at_row(g.quats, k, n, bo);
    const double o = 1.0 / (1.0 + exp(-(double)g.opac[i]));
    const double fx = cam.fx, fy = cam.fy;
    double tv[3];
    for (int r = 0; r < 3; r++) tv[r] = Rc[r * 3 + 0] * mu[0] + Rc[r * 3 + 1] * mu[1] + Rc[r * 3 + 2] * mu[2] + tc[r];
    const double tx = tv[0], ty = tv[1], tz = tv[2];
    const double qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / qnorm, x = q[1] / qnorm, y = q[2] / qnorm, z = q[3] / qnorm;
    const double Rg[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                          2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                          2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
    // opacity
    out.opac[i] = (float)(gop * o * (1.0 - o));

    // mean2d
    double dt[3] = {0.0, 0.0, 0.0};
    dt[0] += gm0 * fx / tz;
    dt[1] += gm1 * fy / tz;
    dt[2] += -gm0 * fx * tx / (tz * tz) - gm1 * fy * ty / (tz * tz);

    // conic = inverse(cov): dL/dcov = -K G K
    const double limx = 1.3 * ((double)cam.W / (2.0 * fx));
    const double limy = 1.3 * ((double)cam.H / (2.0 * fy));
    const double txtz = tx / tz, tytz = ty / tz;
    const bool clx = txtz < -limx || txtz > limx, cly = tytz < -limy || tytz > limy;
    const double cx_ = fmin(limx, fmax(-limx, txtz)) * tz;
    const double cy_ = fmin(limy, fmax(-limy, tytz)) * tz;
    const double J[6] = {fx / tz, 0.0, -(fx * cx_) / (tz * tz), 0.0, fy / tz, -(fy * cy_) / (tz * tz)};
    double T[6];
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++)
            T[r * 3 + k] = J[r * 3 + 0] * Rc[k] + J[r * 3 + 1] * Rc[3 + k] + J[r * 3 + 2] * Rc[6 + k];
    double Sg[9];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += Rg[a * 3 + k] * (s[k] * s[k]) * Rg[b * 3 + k];
            Sg[a * 3 + b] = acc;
        }
    double C2[4];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++)
                for (int l = 0; l < 3; l++) acc += T[a * 3 + k] * Sg[k * 3 + l] * T[b * 3 + l];
            C2[a * 2 + b] = acc;
        }
    const double A = C2[0] + AS_LOWPASS, B = C2[1], Cc = C2[3] + AS_LOWPASS;
    const double det = A * Cc - B * B;
    const double K[4] = {Cc / det, -B / det, -B / det, A / det};
    const double Gk[4] = {gca, 0.5 * gcb, 0.5 * gcb, gcc};
    double KG[4], Gc[4];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) KG[a * 2 + b] = K[a * 2] * Gk[b] + K[a * 2 + 1] * Gk[2 + b];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) Gc[a * 2 + b] = -(KG[a * 2] * K[b] + KG[a * 2 + 1] * K[2 + b]);
    double dS[9], dT[6];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int r = 0; r < 2; r++)
                for (int qq = 0; qq < 2; qq++) acc += T[r * 3 + a] * Gc[r * 2 + qq] * T[qq * 3 + b];
            dS[a * 3 + b] = acc;
        }
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++) {
            double acc = 0.0;
            for (int qq = 0; qq < 2; qq++)
                for (int l = 0; l < 3; l++) acc += Gc[r * 2 + qq] * T[qq * 3 + l] * Sg[l * 3 + k];
            dT[r * 3 + k] = 2.0 * acc;
        }
    double dJ[6];
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++)
            dJ[r * 3 + k] = dT[r * 3 + 0] * Rc[k * 3 + 0] + dT[r * 3 + 1] * Rc[k * 3 + 1] + dT[r * 3 + 2] * Rc[k * 3 + 2];
    dt[2] += dJ[0] * (-fx / (tz * tz)) + dJ[4] * (-fy / (tz * tz));
    if (!clx) {
        dt[0] += dJ[2] * (-fx / (tz * tz));
        dt[2] += dJ[2] * (2.0 * fx * tx / (tz * tz * tz));
    } else {
        dt[2] += dJ[2] * (fx * (cx_ / tz) / (tz * tz));
    }
    if (!cly) {
        dt[1] += dJ[5] * (-fy / (tz * tz));
        dt[2] += dJ[5] * (2.0 * fy * ty / (tz * tz * tz));
    } else {
        dt[2] += dJ[5] * (fy * (cy_ / tz) / (tz * tz));
    }
    for (int a = 0; a < 3; a++) dmu[a] += Rc[0 * 3 + a] * dt[0] + Rc[1 * 3 + a] * dt[1] + Rc[2 * 3 + a] * dt[2];
    for (int a = 0; a < 3; a++) at_row(out.means, a, os, bo) = (float)dmu[a];
    // scales
    for (int k = 0; k < 3; k++) {
        double acc = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) acc += Rg[a * 3 + k] * dS[a * 3 + b] * Rg[b * 3 + k];
        at_row(out.log_scales, k, os, bo) = (float)(2.0 * s[k] * s[k] * acc);
    }
    // rotation -> quaternion
    double dR[9];
    for (int a = 0; a < 3; a++)
        for (int k = 0; k < 3; k++) {
            double acc = 0.0;
            for (int b = 0; b < 3; b++) acc += dS[a * 3 + b] * Rg[b * 3 + k];
            dR[a * 3 + k] = 2.0 * acc * s[k] * s[k];
        }
    double dq[4];
    dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                   2.0 * x * dR[8]);
    dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                   2.0 * y * dR[8]);
    dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] +
                   y * dR[7]);
    const double qn[4] = {w, x, y, z};
    const double qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
    for (int k = 0; k < 4; k++) at_row(out.quats, k, os, bo) = (float)((dq[k] - qn[k] * qd) / qnorm);
}


// All views of a batch in one pass per Gaussian (SH rows addressed as in the
// single-view kernel, BUF).
template <int DEG, bool BUF>
__global__ void __launch_bounds__(256) k_project_bwd(GaussPtrs g, const ViewTable vt, const uint32_t *__restrict__ ntiles,
                                                     const float *__restrict__ g2d, GradPtrs out,
                                                     float *__restrict__ g2d_norm, int32_t *__restrict__ vis_count) {
    constexpr int nk = (DEG + 1) * (DEG + 1);
    // SH gradient accumulators live in LDS (thread-private columns), not registers
    __shared__ float s_dsh[nk * 3][256];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
    if (i >= g.n) return;
    const int64_t n = g.n, os = out.stride;
    const uint32_t bo = (uint32_t)i * 4u;   // the lane's byte offset in every row
#pragma unroll
    for (int k = 0; k < nk * 3; k++) s_dsh[k][tid] = 0.f;

    double mu[3], s[3], q[4];
    for (int k = 0; k < 3; k++) mu[k] = (double)at_row(g.means, k, n, bo);
    for (int k = 0; k < 3; k++) s[k] = exp((double)at_row(g.log_scales, k, n, bo));
    for (int k = 0; k < 4; k++) q[k] = (double)at_row(g.quats, k, n, bo);
    const double o = 1.0 / (1.0 + exp(-(double)g.opac[i]));
    const double qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / qnorm, x = q[1] / qnorm, y = q[2] / qnorm, z = q[3] / qnorm;
    const double Rg[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                          2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                          2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};

    double dmu[3] = {0.0, 0.0, 0.0};
    double dS[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double gop = 0.0;
    float nrm = 0.f;
    int32_t vis = 0;

    for (int v = 0; v < vt.n_views; v++) {
        // keeps the SH coefficients' loads inside the loop (from cache) instead
        // of 48 doubles held in registers across it
        __asm__ __volatile__("" ::: "memory");
        const int64_t e = (int64_t)vt.ent_base[v] + i;
        if (ntiles[e] == 0) continue;
        const DevCam &cam = vt.cam[v];
        const double gm0 = g2d[e * 9 + 0], gm1 = g2d[e * 9 + 1];
        const double gca = g2d[e * 9 + 2], gcb = g2d[e * 9 + 3], gcc = g2d[e * 9 + 4];
        const double grgb[3] = {g2d[e * 9 + 6], g2d[e * 9 + 7], g2d[e * 9 + 8]};
        gop += g2d[e * 9 + 5];
        nrm += (float)sqrt(gm0 * gm0 + gm1 * gm1);
        vis += 1;

        double Rc[9], tc[3];
        for (int k = 0; k < 9; k++) Rc[k] = (double)cam.R[k];
        for (int k = 0; k < 3; k++) tc[k] = (double)cam.t[k];
        const double fx = cam.fx, fy = cam.fy;
        double tv[3];
        for (int r = 0; r < 3; r++) tv[r] = Rc[r * 3 + 0] * mu[0] + Rc[r * 3 + 1] * mu[1] + Rc[r * 3 + 2] * mu[2] + tc[r];
        const double tx = tv[0], ty = tv[1], tz = tv[2];

        // colour and view direction
        double oc[3];
        for (int j = 0; j < 3; j++) oc[j] = -(Rc[0 * 3 + j] * tc[0] + Rc[1 * 3 + j] * tc[1] + Rc[2 * 3 + j] * tc[2]);
        const double vv[3] = {mu[0] - oc[0], mu[1] - oc[1], mu[2] - oc[2]};
        const double vn = sqrt(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
        const double d[3] = {vv[0] / vn, vv[1] / vn, vv[2] / vn};
        double Y[16];
        sh_eval_basis(d[0], d[1], d[2], DEG, Y);
        // as in the single-view kernel: one pass over the coefficients gives
        // each channel's raw colour (its clamp) and direction gradient
        double gc[3], gd[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            double shc[16], raw = 0.0;
#pragma unroll
            for (int k = 0; k < nk; k++) {
                shc[k] = (double)sh_ld<BUF>(g.sh, k * 3 + ch, n, bo);
                raw += Y[k] * shc[k];
            }
            double gch[3];
            sh_weighted_grad(d[0], d[1], d[2], DEG, shc, gch);
            gc[ch] = raw + 0.5 < 0.0 ? 0.0 : grgb[ch];
            for (int a = 0; a < 3; a++) gd[a] += gc[ch] * gch[a];
        }
#pragma unroll
        for (int k = 0; k < nk; k++)
#pragma unroll
            for (int ch = 0; ch < 3; ch++) s_dsh[k * 3 + ch][tid] += (float)(Y[k] * gc[ch]);
        const double ddot = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
        for (int a = 0; a < 3; a++) dmu[a] += (gd[a] - d[a] * ddot) / vn;

        // mean2d
        double dt[3] = {0.0, 0.0, 0.0};
        dt[0] += gm0 * fx / tz;
        dt[1] += gm1 * fy / tz;
        dt[2] += -gm0 * fx * tx / (tz * tz) - gm1 * fy * ty / (tz * tz);

        // conic = inverse(cov): dL/dcov = -K G K
        const double limx = 1.3 * ((double)cam.W / (2.0 * fx));
        const double limy = 1.3 * ((double)cam.H / (2.0 * fy));
        const double txtz = tx / tz, tytz = ty / tz;
        const bool clx = txtz < -limx || txtz > limx, cly = tytz < -limy || tytz > limy;
        const double cx_ = fmin(limx, fmax(-limx, txtz)) * tz;
        const double cy_ = fmin(limy, fmax(-limy, tytz)) * tz;
        const double J[6] = {fx / tz, 0.0, -(fx * cx_) / (tz * tz), 0.0, fy / tz, -(fy * cy_) / (tz * tz)};
        double T[6];
        for (int r = 0; r < 2; r++)
            for (int k = 0; k < 3; k++)
                T[r * 3 + k] = J[r * 3 + 0] * Rc[k] + J[r * 3 + 1] * Rc[3 + k] + J[r * 3 + 2] * Rc[6 + k];
        double Sg[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0.0;
                for (int k = 0; k < 3; k++) acc += Rg[a * 3 + k] * (s[k] * s[k]) * Rg[b * 3 + k];
                Sg[a * 3 + b] = acc;
            }
        double C2[4];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                double acc = 0.0;
                for (int k = 0; k < 3; k++)
                    for (int l = 0; l < 3; l++) acc += T[a * 3 + k] * Sg[k * 3 + l] * T[b * 3 + l];
                C2[a * 2 + b] = acc;
            }
        const double A = C2[0] + AS_LOWPASS, B = C2[1], Cc = C2[3] + AS_LOWPASS;
        const double det = A * Cc - B * B;
        const double K[4] = {Cc / det, -B / det, -B / det, A / det};
        const double Gk[4] = {gca, 0.5 * gcb, 0.5 * gcb, gcc};
        double KG[4], Gc[4];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) KG[a * 2 + b] = K[a * 2] * Gk[b] + K[a * 2 + 1] * Gk[2 + b];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) Gc[a * 2 + b] = -(KG[a * 2] * K[b] + KG[a * 2 + 1] * K[2 + b]);
        double dT[6];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0.0;
                for (int r = 0; r < 2; r++)
                    for (int qq = 0; qq < 2; qq++) acc += T[r * 3 + a] * Gc[r * 2 + qq] * T[qq * 3 + b];
                dS[a * 3 + b] += acc;
            }
        for (int r = 0; r < 2; r++)
            for (int k = 0; k < 3; k++) {
                double acc = 0.0;
                for (int qq = 0; qq < 2; qq++)
                    for (int l = 0; l < 3; l++) acc += Gc[r * 2 + qq] * T[qq * 3 + l] * Sg[l * 3 + k];
                dT[r * 3 + k] = 2.0 * acc;
            }
        double dJ[6];
        for (int r = 0; r < 2; r++)
            for (int k = 0; k < 3; k++)
                dJ[r * 3 + k] =
                    dT[r * 3 + 0] * Rc[k * 3 + 0] + dT[r * 3 + 1] * Rc[k * 3 + 1] + dT[r * 3 + 2] * Rc[k * 3 + 2];
        dt[2] += dJ[0] * (-fx / (tz * tz)) + dJ[4] * (-fy / (tz * tz));
        if (!clx) {
            dt[0] += dJ[2] * (-fx / (tz * tz));
            dt[2] += dJ[2] * (2.0 * fx * tx / (tz * tz * tz));
        } else {
            dt[2] += dJ[2] * (fx * (cx_ / tz) / (tz * tz));
        }
        if (!cly) {
            dt[1] += dJ[5] * (-fy / (tz * tz));
            dt[2] += dJ[5] * (2.0 * fy * ty / (tz * tz * tz));
        } else {
            dt[2] += dJ[5] * (fy * (cy_ / tz) / (tz * tz));
        }
        for (int a = 0; a < 3; a++) dmu[a] += Rc[0 * 3 + a] * dt[0] + Rc[1 * 3 + a] * dt[1] + Rc[2 * 3 + a] * dt[2];
    }

    if (vis && g2d_norm) g2d_norm[i] += nrm;
    if (vis && vis_count) vis_count[i] += vis;
    if (!vis) {   // no view saw it: zero gradients
        for (int k = 0; k < 3; k++) { at_row(out.means, k, os, bo) = 0.f; at_row(out.log_scales, k, os, bo) = 0.f; }
        for (int k = 0; k < 4; k++) at_row(out.quats, k, os, bo) = 0.f;
        out.opac[i] = 0.f;
#pragma unroll
        for (int k = 0; k < nk * 3; k++) sh_st<BUF>(out.sh, k, os, bo, 0.f);
        return;
    }
    out.opac[i] = (float)(gop * o * (1.0 - o));
#pragma unroll
    for (int k = 0; k < nk * 3; k++) sh_st<BUF>(out.sh, k, os, bo, s_dsh[k][tid]);
    for (int a = 0; a < 3; a++) at_row(out.means, a, os, bo) = (float)dmu[a];
    // scales
    for (int k = 0; k < 3; k++) {
        double acc = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) acc += Rg[a * 3 + k] * dS[a * 3 + b] * Rg[b * 3 + k];
        at_row(out.log_scales, k, os, bo) = (float)(2.0 * s[k] * s[k] * acc);
    }
    // rotation -> quaternion
    double dR[9];
    for (int a = 0; a < 3; a++)
        for (int k = 0; k < 3; k++) {
            double acc = 0.0;
            for (int b = 0; b < 3; b++) acc += dS[a * 3 + b] * Rg[b * 3 + k];
            dR[a * 3 + k] = 2.0 * acc * s[k] * s[k];
        }
    double dq[4];
    dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                   2.0 * x * dR[8]);
    dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                   2.0 * y * dR[8]);
    dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] +
                   y * dR[7]);
    const double qn[4] = {w, x, y, z};
    const double qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
    for (int k = 0; k < 4; k++) at_row(out.quats, k, os, bo) = (float)((dq[k] - qn[k] * qd) / qnorm);
}

}  // namespace

void launch_project_bwd(const GaussPtrs &g, const ViewTable &vt, const uint32_t *ntiles, const float *grad2d,
                        GradPtrs out, float *g2d_norm, int32_t *vis_count, hipStream_t s, bool force_addr64) {
    if (g.n == 0) return;
    const dim3 grid((unsigned)((g.n + 255) / 256));
    // buffer addressing when the last SH row's byte offset fits 32 bits
    const int64_t rows = 3 * (int64_t)(g.deg + 1) * (g.deg + 1);
    const bool buf = !force_addr64 && rows * (g.n > out.stride ? g.n : out.stride) * 4 <= (int64_t)UINT32_MAX;
    if (vt.n_views == 1) {
        const DevCam &cam = vt.cam[0];
#define AS_PBV(D)                                                                                                  \
    do {                                                                                                           \
        if (buf) hipLaunchKernelGGL((k_project_bwd_view<D, true>), grid, dim3(256), 0, s, g, cam, ntiles, grad2d,  \
                                    out, g2d_norm, vis_count);                                                     \
        else hipLaunchKernelGGL((k_project_bwd_view<D, false>), grid, dim3(256), 0, s, g, cam, ntiles, grad2d, out, \
                                g2d_norm, vis_count);                                                              \
    } while (0)
        switch (g.deg) {
        case 0: AS_PBV(0); break;
        case 1: AS_PBV(1); break;
        case 2: AS_PBV(2); break;
        default: AS_PBV(3); break;
        }
#undef AS_PBV
        return;
    }
#define AS_PBB(D)                                                                                                  \
    do {                                                                                                           \
        if (buf) hipLaunchKernelGGL((k_project_bwd<D, true>), grid, dim3(256), 0, s, g, vt, ntiles, grad2d, out,   \
                                    g2d_norm, vis_count);                                                          \
        else hipLaunchKernelGGL((k_project_bwd<D, false>), grid, dim3(256), 0, s, g, vt, ntiles, grad2d, out,      \
                                g2d_norm, vis_count);                                                              \
    } while (0)
    switch (g.deg) {
    case 0: AS_PBB(0); break;
    case 1: AS_PBB(1); break;
    case 2: AS_PBB(2); break;
    default: AS_PBB(3); break;
    }
#undef AS_PBB
}

AS_WARM_KERNEL(project_bwd)
