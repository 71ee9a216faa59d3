// Kernels of the optimisation loop around the path: the L1 loss and its
// gradient, the Adam step, and the bookkeeping of 3DGS's adaptive density
// control (selection, row maps of the split, clone + prune, optimiser-state
// carry-over, opacity reset), Sec. 3 and Sec. 5 "Implementation".
//
// A Gaussian set is 11 + 3 (d + 1)^2 rows of floats with one row stride:
// means [3], log scales [3], quaternion [4], opacity logit [1], SH [k][3].
// Reductions go through per-block partials and a one-block pass: device-wide
// atomics on a few words serialise at the memory side.
#include "internal.h"

namespace {

constexpr int TB = 256;
constexpr int PART_MAX = 1024;   // blocks of a reduction launch (partials buffer rows)

struct RowSet {
    float *means, *ls, *q, *op, *sh;
    int64_t stride;
};

__host__ __device__ __forceinline__ int set_rows(int deg) { return 11 + 3 * (deg + 1) * (deg + 1); }

__device__ __forceinline__ float *row_ptr(const RowSet &s, int r) {
    if (r < 3) return s.means + (int64_t)r * s.stride;
    if (r < 6) return s.ls + (int64_t)(r - 3) * s.stride;
    if (r < 10) return s.q + (int64_t)(r - 6) * s.stride;
    if (r == 10) return s.op;
    return s.sh + (int64_t)(r - 11) * s.stride;
}

RowSet rows_of(const as_gaussians_mut &g) { return RowSet{g.means, g.log_scales, g.quats, g.opacity_logits, g.sh, g.n}; }
RowSet rows_of(const as_gaussians &g) {
    return RowSet{const_cast<float *>(g.means), const_cast<float *>(g.log_scales), const_cast<float *>(g.quats),
                  const_cast<float *>(g.opacity_logits), const_cast<float *>(g.sh), g.n};
}

struct AdamLr {
    float means, ls, q, op, dc, rest;
};

// grid.y = row of the set; grid.x strides over the Gaussians
__global__ void __launch_bounds__(TB) k_adam(RowSet p, RowSet g, RowSet m, RowSet v, int64_t n, AdamLr lr, float b1,
                                             float b2, float eps, float step_size, float inv_sqrt_bc2) {
    const int r = blockIdx.y;
    const float l = r < 3 ? lr.means : r < 6 ? lr.ls : r < 10 ? lr.q : r == 10 ? lr.op : r < 14 ? lr.dc : lr.rest;
    float *P = row_ptr(p, r), *M = row_ptr(m, r), *V = row_ptr(v, r);
    const float *G = row_ptr(g, r);
    const float s = l * step_size;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        const float gi = G[i];
        const float mi = b1 * M[i] + (1.0f - b1) * gi;
        const float vi = b2 * V[i] + (1.0f - b2) * (gi * gi);
        M[i] = mi;
        V[i] = vi;
        const float denom = sqrtf(vi) * inv_sqrt_bc2 + eps;
        P[i] = P[i] - s * (mi / denom);
    }
}

__device__ __forceinline__ double wave_sum_d(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// sum |d| and sum d^2 per block into part[block][2]; the gradient of the mean L1
__global__ void __launch_bounds__(TB) k_l1(int64_t n3, const float *__restrict__ img, const float *__restrict__ gt,
                                           float *__restrict__ dL, float inv, double *__restrict__ part) {
    __shared__ double s1[TB / 64], s2[TB / 64];
    double a = 0.0, b = 0.0;
    for (int64_t u = (int64_t)blockIdx.x * TB + threadIdx.x; u < n3; u += (int64_t)gridDim.x * TB) {
        const float d = img[u] - gt[u];
        if (dL) dL[u] = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
        const double dd = (double)d;
        a += fabs(dd);
        b += dd * dd;
    }
    a = wave_sum_d(a);
    b = wave_sum_d(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s1[w] = a;
        s2[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < TB / 64; k++) {
            a += s1[k];
            b += s2[k];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// one block: sum the partials in block order (deterministic)
__global__ void __launch_bounds__(TB) k_sum_partials(const double *__restrict__ part, int nblk, double *__restrict__ out) {
    __shared__ double s1[TB / 64], s2[TB / 64];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblk; k += TB) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    a = wave_sum_d(a);
    b = wave_sum_d(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s1[w] = a;
        s2[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < TB / 64; k++) {
            a += s1[k];
            b += s2[k];
        }
        out[0] = a;
        out[1] = b;
    }
}

__device__ __forceinline__ float max_log_scale(const float *ls, int64_t stride, int64_t i) {
    return fmaxf(fmaxf(ls[i], ls[stride + i]), ls[2 * stride + i]);
}

__global__ void __launch_bounds__(TB) k_select(int64_t n, const float *__restrict__ ls, int64_t stride,
                                               const float *__restrict__ accum, const int32_t *__restrict__ vis,
                                               double thr, double size_thr, uint8_t *__restrict__ clone,
                                               uint8_t *__restrict__ cand_flag) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    const int32_t c = vis[i];
    const double a = (double)accum[i] / (double)(c > 1 ? c : 1);
    const bool sel = a >= thr;
    const bool big = exp((double)max_log_scale(ls, stride, i)) > size_thr;
    clone[i] = sel && !big ? 1 : 0;
    cand_flag[i] = sel && big ? 1 : 0;
}

// ids of the set flags, ascending: out[scan[i]] = i
__global__ void __launch_bounds__(TB) k_compact_ids(int64_t n, const uint8_t *__restrict__ flag,
                                                    const int64_t *__restrict__ scan, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < n && flag[i]) out[scan[i]] = (int32_t)i;
}

// a candidate's parent stays unless its mode is RESET (1)
__global__ void __launch_bounds__(TB) k_mark_kept(const int32_t *__restrict__ cand, int64_t n_cand,
                                                  const int64_t *__restrict__ n_cand_dev,
                                                  const uint8_t *__restrict__ mode, int64_t n, uint8_t *__restrict__ keep) {
    const int64_t c = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (c >= count_in_use(n_cand, n_cand_dev)) return;
    const int32_t id = cand[c];
    if (id >= 0 && id < n && mode[c] != 1) keep[id] = 0;
}

// keep[i] = 1 for the rows in use, 0 for the rest of the capacity
__global__ void __launch_bounds__(TB) k_keep_init(int64_t n, const int64_t *__restrict__ n_dev,
                                                  uint8_t *__restrict__ keep) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < n) keep[i] = i < count_in_use(n, n_dev) ? 1 : 0;
}

__global__ void __launch_bounds__(TB) k_row_map(int64_t n, const uint8_t *__restrict__ keep,
                                                const int64_t *__restrict__ pos, const int32_t *__restrict__ state_in,
                                                int64_t capacity, int32_t *__restrict__ row_src) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < n && keep[i] && pos[i] < capacity) row_src[pos[i]] = state_in ? state_in[i] : (int32_t)i;
}

__global__ void __launch_bounds__(TB) k_prune_flags(int64_t n, const int64_t *__restrict__ n_dev,
                                                    const float *__restrict__ op, const float *__restrict__ ls,
                                                    int64_t stride, const uint8_t *__restrict__ clone_mask,
                                                    double min_op, double max_scale, uint8_t *__restrict__ keep,
                                                    uint8_t *__restrict__ dup) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    if (i >= count_in_use(n, n_dev)) {   // past the rows in use: neither kept nor cloned
        keep[i] = 0;
        dup[i] = 0;
        return;
    }
    const double o = 1.0 / (1.0 + exp(-(double)op[i]));
    bool k = o >= min_op;
    if (max_scale > 0.0) k = k && exp((double)max_log_scale(ls, stride, i)) <= max_scale;
    keep[i] = k ? 1 : 0;
    dup[i] = k && clone_mask && clone_mask[i] ? 1 : 0;
}

// kept rows in order, then the clones; the output has at least 2 n rows
__global__ void __launch_bounds__(TB) k_clone_prune_write(int64_t n, RowSet src, RowSet dst, int nrows,
                                                          const uint8_t *__restrict__ keep,
                                                          const uint8_t *__restrict__ dup,
                                                          const int64_t *__restrict__ kpos,
                                                          const int64_t *__restrict__ dpos,
                                                          const int64_t *__restrict__ n_keep,
                                                          const int32_t *__restrict__ state_in,
                                                          int32_t *__restrict__ state_src) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    if (keep[i]) {
        const int64_t r = kpos[i];
        for (int k = 0; k < nrows; k++) row_ptr(dst, k)[r] = row_ptr(src, k)[i];
        state_src[r] = state_in ? state_in[i] : (int32_t)i;
    }
    if (dup[i]) {
        const int64_t r = *n_keep + dpos[i];
        for (int k = 0; k < nrows; k++) row_ptr(dst, k)[r] = row_ptr(src, k)[i];
        state_src[r] = -1;
    }
}

__global__ void k_add_totals(const int64_t *__restrict__ a, const int64_t *__restrict__ b, int64_t *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = *a + *b;
}

__global__ void __launch_bounds__(TB) k_gather_rows(RowSet src, int64_t src_n, const int32_t *__restrict__ map,
                                                    int64_t n_rows, const int64_t *__restrict__ n_rows_dev,
                                                    RowSet dst) {
    const int r = blockIdx.y;
    const float *S = row_ptr(src, r);
    float *D = row_ptr(dst, r);
    const int64_t m = count_in_use(n_rows, n_rows_dev);
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < m; i += (int64_t)gridDim.x * TB) {
        const int32_t s = map[i];
        D[i] = s >= 0 && s < src_n ? S[s] : 0.0f;
    }
}

__global__ void __launch_bounds__(TB) k_reset_opacity(int64_t n, float *__restrict__ op, float cap,
                                                      float *__restrict__ m, float *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    op[i] = fminf(op[i], cap);
    if (m) m[i] = 0.0f;
    if (v) v[i] = 0.0f;
}

unsigned blocks_for(int64_t n, int64_t cap) {
    int64_t b = (n + TB - 1) / TB;
    if (b > cap) b = cap;
    return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

int train_set_rows(int deg) { return set_rows(deg); }

void launch_adam(const as_gaussians_mut &p, const as_gaussians &g, const as_gaussians_mut &m, const as_gaussians_mut &v,
                 const as_adam_params &hp, int32_t step, hipStream_t s) {
    const int64_t n = p.n;
    if (n == 0) return;
    const double bc1 = 1.0 - pow((double)hp.beta1, (double)step);
    const double bc2 = 1.0 - pow((double)hp.beta2, (double)step);
    const AdamLr lr{hp.lr_means, hp.lr_log_scales, hp.lr_quats, hp.lr_opacity, hp.lr_sh_dc, hp.lr_sh_rest};
    const dim3 grid(blocks_for(n, 1024), (unsigned)set_rows(p.sh_degree));
    hipLaunchKernelGGL(k_adam, grid, dim3(TB), 0, s, rows_of(p), rows_of(g), rows_of(m), rows_of(v), n, lr, hp.beta1,
                       hp.beta2, hp.eps, (float)(1.0 / bc1), (float)(1.0 / sqrt(bc2)));
}

size_t l1_partials_bytes() { return (size_t)PART_MAX * 2 * sizeof(double); }

void launch_l1(int W, int H, const float *img, const float *gt, float *dL, double *sums, double *partials,
               hipStream_t s) {
    const int64_t n3 = 3 * (int64_t)W * H;
    const unsigned g = blocks_for(n3, PART_MAX);
    hipLaunchKernelGGL(k_l1, dim3(g), dim3(TB), 0, s, n3, img, gt, dL, (float)(1.0 / (double)n3), partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(TB), 0, s, partials, (int)g, sums);
}

void launch_select(const as_gaussians &g, const float *accum, const int32_t *vis, double thr, double size_thr,
                   uint8_t *clone, uint8_t *cand_flag, hipStream_t s) {
    if (g.n == 0) return;
    hipLaunchKernelGGL(k_select, dim3(blocks_for(g.n, 1ll << 30)), dim3(TB), 0, s, g.n, g.log_scales, g.n, accum, vis,
                       thr, size_thr, clone, cand_flag);
}

void launch_compact_ids(int64_t n, const uint8_t *flag, const int64_t *scan, int32_t *out, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_compact_ids, dim3(blocks_for(n, 1ll << 30)), dim3(TB), 0, s, n, flag, scan, out);
}

void launch_keep_init(int64_t n, const int64_t *n_dev, uint8_t *keep, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_keep_init, dim3(blocks_for(n, 1ll << 30)), dim3(TB), 0, s, n, n_dev, keep);
}

void launch_mark_kept(const int32_t *cand, int64_t n_cand, const int64_t *n_cand_dev, const uint8_t *mode, int64_t n,
                      uint8_t *keep, hipStream_t s) {
    if (n_cand == 0) return;
    hipLaunchKernelGGL(k_mark_kept, dim3(blocks_for(n_cand, 1ll << 30)), dim3(TB), 0, s, cand, n_cand, n_cand_dev,
                       mode, n, keep);
}

void launch_row_map(int64_t n, const uint8_t *keep, const int64_t *pos, const int32_t *state_in, int64_t capacity,
                    int32_t *row_src, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_row_map, dim3(blocks_for(n, 1ll << 30)), dim3(TB), 0, s, n, keep, pos, state_in, capacity,
                       row_src);
}

void launch_prune_flags(const as_gaussians &g, const uint8_t *clone_mask, double min_op, double max_scale,
                        uint8_t *keep, uint8_t *dup, hipStream_t s) {
    if (g.n == 0) return;
    hipLaunchKernelGGL(k_prune_flags, dim3(blocks_for(g.n, 1ll << 30)), dim3(TB), 0, s, g.n, g.n_dev,
                       g.opacity_logits, g.log_scales, g.n, clone_mask, min_op, max_scale, keep, dup);
}

void launch_clone_prune_write(const as_gaussians &g, const as_gaussians_mut &out, const uint8_t *keep,
                              const uint8_t *dup, const int64_t *kpos, const int64_t *dpos, const int64_t *n_keep,
                              const int64_t *n_dup, const int32_t *state_in, int32_t *state_src, int64_t *n_out,
                              hipStream_t s) {
    if (g.n > 0)
        hipLaunchKernelGGL(k_clone_prune_write, dim3(blocks_for(g.n, 1ll << 30)), dim3(TB), 0, s, g.n, rows_of(g),
                           rows_of(out), set_rows(g.sh_degree), keep, dup, kpos, dpos, n_keep, state_in, state_src);
    hipLaunchKernelGGL(k_add_totals, dim3(1), dim3(64), 0, s, n_keep, n_dup, n_out);
}

void launch_gather_rows(const as_gaussians &src, const int32_t *map, int64_t n_rows, const int64_t *n_rows_dev,
                        const as_gaussians_mut &dst, hipStream_t s) {
    if (n_rows == 0) return;
    const dim3 grid(blocks_for(n_rows, 1024), (unsigned)set_rows(src.sh_degree));
    hipLaunchKernelGGL(k_gather_rows, grid, dim3(TB), 0, s, rows_of(src), src.n, map, n_rows, n_rows_dev,
                       rows_of(dst));
}

void launch_reset_opacity(const as_gaussians_mut &g, float cap, float *m, float *v, hipStream_t s) {
    if (g.n == 0) return;
    hipLaunchKernelGGL(k_reset_opacity, dim3(blocks_for(g.n, 1ll << 30)), dim3(TB), 0, s, g.n, g.opacity_logits, cap,
                       m, v);
}

AS_WARM_KERNEL(train)
