// The AdpSplit adaptive split (Sec. 4.2, 4.3, App. A and the implementation
// details of Sec. 5) and the stream-compacted append.
//
//   1. region records sorted by (candidate, view, label) with the LDS radix
//      sorter, so that each candidate owns a contiguous range;
//   2. one thread per region: child proposal (centre at t* of Eq. (tstar) on
//      the centroid ray, shape from the clipped, unprojected PCA axes,
//      Gram-Schmidt rotation [u1 | u2 | z_v], colour from the target);
//   3. one wave per candidate: transitive merge graph under
//      Eq. (merge_conditions) (lock-free union-find, roots = first member),
//      merged parameters of Eq. (merge_cov), ranking by covariance extent and
//      the N_max cap, then the mode (vanilla / reset / adaptive / random) and
//      count (the ablation variants of Table 2 skip the merge, or the region
//      children altogether);
//   4. scans of the counts and of the removal mask, survivor copy and child
//      write-out.
// All decision arithmetic is FP64 with a fixed expression order; this file is
// compiled with -ffp-contract=off.
#include "internal.h"

namespace {

enum { SP_K0, SP_K1, SP_V0, SP_V1, SP_HIST, SP_N, SP_RS, SP_RE, SP_PROP, SP_UF, SP_ROOT, SP_GRP, SP_KEPT, SP_NKEPT,
       SP_CAMS, SP_REM, SP_REMSCAN, SP_SCAN, SP_TOT, SP_COUNT };

constexpr double C0_SH = 0.28209479177387814;   // degree-0 real SH constant 1/(2 sqrt(pi))

struct Prop {
    double mu[3], R[9], s[3], rgb[3], Sig[9], Sinv[9];
    int32_t ok, view;
};

struct Group {
    double mu[3], R[9], s[3], rgb[3], extent;
};

__device__ __forceinline__ int64_t find_cand(const int32_t *cand, int64_t n_cand, int32_t id) {
    int64_t lo = 0, hi = n_cand;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cand[mid] < id) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n_cand && cand[lo] == id) ? lo : -1;
}

struct Parent {
    double mu[3], s[3], R[9], o;
};

__device__ __forceinline__ void load_parent(const GaussPtrs &g, int64_t i, Parent &p) {
    const int64_t n = g.n;
    for (int k = 0; k < 3; k++) p.mu[k] = (double)g.means[k * n + i];
    for (int k = 0; k < 3; k++) p.s[k] = exp((double)g.log_scales[k * n + i]);
    double q[4];
    for (int k = 0; k < 4; k++) q[k] = (double)g.quats[k * n + i];
    const double qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / qnorm, x = q[1] / qnorm, y = q[2] / qnorm, z = q[3] / qnorm;
    p.R[0] = 1.0 - 2.0 * (y * y + z * z); p.R[1] = 2.0 * (x * y - w * z);       p.R[2] = 2.0 * (x * z + w * y);
    p.R[3] = 2.0 * (x * y + w * z);       p.R[4] = 1.0 - 2.0 * (x * x + z * z); p.R[5] = 2.0 * (y * z - w * x);
    p.R[6] = 2.0 * (x * z - w * y);       p.R[7] = 2.0 * (y * z + w * x);       p.R[8] = 1.0 - 2.0 * (x * x + y * y);
    p.o = 1.0 / (1.0 + exp(-(double)g.opac[i]));
}

__device__ __forceinline__ double clipv(double x, double a) {
    const double m = fabs(x) < a ? fabs(x) : a;
    return x < 0.0 ? -m : m;
}

// Child proposal of one region (App. A).
__device__ void make_proposal(const Parent &par, const as_region &r, const DevCam &cam, double eps, Prop &p) {
    p.ok = 0;
    double Rc[9], tc[3];
    for (int k = 0; k < 9; k++) Rc[k] = (double)cam.R[k];
    for (int k = 0; k < 3; k++) tc[k] = (double)cam.t[k];
    double ov[3];
    for (int j = 0; j < 3; j++) ov[j] = -(Rc[0 * 3 + j] * tc[0] + Rc[1 * 3 + j] * tc[1] + Rc[2 * 3 + j] * tc[2]);
    const double fx = cam.fx, fy = cam.fy;
    const double dc[3] = {(r.cx - (double)cam.cx) / fx, (r.cy - (double)cam.cy) / fy, 1.0};
    double dw[3];
    for (int j = 0; j < 3; j++) dw[j] = Rc[0 * 3 + j] * dc[0] + Rc[1 * 3 + j] * dc[1] + Rc[2 * 3 + j] * dc[2];
    const double dwn = sqrt(dw[0] * dw[0] + dw[1] * dw[1] + dw[2] * dw[2]);
    const double d[3] = {dw[0] / dwn, dw[1] / dwn, dw[2] / dwn};
    double Am[9];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += par.R[a * 3 + k] * (1.0 / (par.s[k] * par.s[k])) * par.R[b * 3 + k];
            Am[a * 3 + b] = acc;
        }
    const double bv[3] = {par.mu[0] - ov[0], par.mu[1] - ov[1], par.mu[2] - ov[2]};
    double Ad[3];
    for (int a = 0; a < 3; a++) Ad[a] = Am[a * 3 + 0] * d[0] + Am[a * 3 + 1] * d[1] + Am[a * 3 + 2] * d[2];
    const double num = bv[0] * Ad[0] + bv[1] * Ad[1] + bv[2] * Ad[2];
    const double den = d[0] * Ad[0] + d[1] * Ad[1] + d[2] * Ad[2];
    const double tstar = num / (den + eps);
    for (int a = 0; a < 3; a++) p.mu[a] = ov[a] + tstar * d[a];
    const double dcn = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
    const double tz = tstar / dcn;
    if (!(tz > AS_NEAR)) return;
    double smax = par.s[0];
    if (par.s[1] > smax) smax = par.s[1];
    if (par.s[2] > smax) smax = par.s[2];
    const double e1x = r.e1[0], e1y = r.e1[1];
    const double e2x = -e1y, e2y = e1x;
    const double w1x = clipv(e1x * r.sigma1 * tz / fx, smax * fabs(e1x));
    const double w1y = clipv(e1y * r.sigma1 * tz / fy, smax * fabs(e1y));
    const double w2x = clipv(e2x * r.sigma2 * tz / fx, smax * fabs(e2x));
    const double w2y = clipv(e2y * r.sigma2 * tz / fy, smax * fabs(e2y));
    double a1[3], a2[3];
    for (int k = 0; k < 3; k++) {
        a1[k] = w1x * Rc[0 * 3 + k] + w1y * Rc[1 * 3 + k];
        a2[k] = w2x * Rc[0 * 3 + k] + w2y * Rc[1 * 3 + k];
    }
    const double n1 = sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
    const double n2 = sqrt(a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]);
    if (!(n1 > 0.0) || !(n2 > 0.0)) return;
    p.s[0] = n1; p.s[1] = n2; p.s[2] = n2;
    const double u1[3] = {a1[0] / n1, a1[1] / n1, a1[2] / n1};
    const double pr = a2[0] * u1[0] + a2[1] * u1[1] + a2[2] * u1[2];
    const double q2[3] = {a2[0] - pr * u1[0], a2[1] - pr * u1[1], a2[2] - pr * u1[2]};
    const double nq = sqrt(q2[0] * q2[0] + q2[1] * q2[1] + q2[2] * q2[2]);
    if (!(nq > 0.0)) return;
    const double u2[3] = {q2[0] / nq, q2[1] / nq, q2[2] / nq};
    for (int k = 0; k < 3; k++) {
        p.R[k * 3 + 0] = u1[k];
        p.R[k * 3 + 1] = u2[k];
        p.R[k * 3 + 2] = Rc[2 * 3 + k];
    }
    for (int ch = 0; ch < 3; ch++) p.rgb[ch] = (double)r.rgb[ch];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0, acci = 0.0;
            for (int k = 0; k < 3; k++) {
                acc += p.R[a * 3 + k] * (p.s[k] * p.s[k]) * p.R[b * 3 + k];
                acci += p.R[a * 3 + k] * (1.0 / (p.s[k] * p.s[k])) * p.R[b * 3 + k];
            }
            p.Sig[a * 3 + b] = acc;
            p.Sinv[a * 3 + b] = acci;
        }
    p.ok = 1;
}

__device__ __forceinline__ double maha(const double *Sinv, const double *dl) {
    double acc = 0.0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) acc += dl[a] * Sinv[a * 3 + b] * dl[b];
    return sqrt(acc);
}

// Cyclic Jacobi on a symmetric 3x3 matrix; columns of V are eigenvectors,
// sorted by descending eigenvalue, last column flipped so det V = +1.
__device__ void jacobi3(const double *Ain, double V[9], double lam[3]) {
    double A[9];
    for (int k = 0; k < 9; k++) A[k] = Ain[k];
    for (int k = 0; k < 9; k++) V[k] = (k % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 32; sweep++) {
        const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        const double dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-30 * dia) break;
        for (int p = 0; p < 2; p++)
            for (int q = p + 1; q < 3; q++) {
                const double apq = A[p * 3 + q];
                if (apq == 0.0) continue;
                const double app = A[p * 3 + p], aqq = A[q * 3 + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; k++) {
                    const double akp = A[k * 3 + p], akq = A[k * 3 + q];
                    A[k * 3 + p] = cs * akp - sn * akq;
                    A[k * 3 + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; k++) {
                    const double apk = A[p * 3 + k], aqk = A[q * 3 + k];
                    A[p * 3 + k] = cs * apk - sn * aqk;
                    A[q * 3 + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < 3; k++) {
                    const double vkp = V[k * 3 + p], vkq = V[k * 3 + q];
                    V[k * 3 + p] = cs * vkp - sn * vkq;
                    V[k * 3 + q] = sn * vkp + cs * vkq;
                }
            }
    }
    for (int k = 0; k < 3; k++) lam[k] = A[k * 4];
    for (int a = 0; a < 2; a++) {
        int best = a;
        for (int b = a + 1; b < 3; b++)
            if (lam[b] > lam[best]) best = b;
        if (best != a) {
            const double tl = lam[a];
            lam[a] = lam[best];
            lam[best] = tl;
            for (int k = 0; k < 3; k++) {
                const double tv = V[k * 3 + a];
                V[k * 3 + a] = V[k * 3 + best];
                V[k * 3 + best] = tv;
            }
        }
    }
    const double det = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
                       V[2] * (V[3] * V[7] - V[4] * V[6]);
    if (det < 0.0)
        for (int k = 0; k < 3; k++) V[k * 3 + 2] = -V[k * 3 + 2];
}

// Unit quaternion (w >= 0) of a rotation matrix (Shepperd's method).
__device__ void rot_to_quat(const double *R, double q[4]) {
    const double tr = R[0] + R[4] + R[8];
    double w, x, y, z;
    if (tr > 0.0) {
        const double s = sqrt(tr + 1.0) * 2.0;
        w = 0.25 * s; x = (R[7] - R[5]) / s; y = (R[2] - R[6]) / s; z = (R[3] - R[1]) / s;
    } else if (R[0] > R[4] && R[0] > R[8]) {
        const double s = sqrt(1.0 + R[0] - R[4] - R[8]) * 2.0;
        w = (R[7] - R[5]) / s; x = 0.25 * s; y = (R[1] + R[3]) / s; z = (R[2] + R[6]) / s;
    } else if (R[4] > R[8]) {
        const double s = sqrt(1.0 + R[4] - R[0] - R[8]) * 2.0;
        w = (R[2] - R[6]) / s; x = (R[1] + R[3]) / s; y = 0.25 * s; z = (R[5] + R[7]) / s;
    } else {
        const double s = sqrt(1.0 + R[8] - R[0] - R[4]) * 2.0;
        w = (R[3] - R[1]) / s; x = (R[2] + R[6]) / s; y = (R[5] + R[7]) / s; z = 0.25 * s;
    }
    double nn = sqrt(w * w + x * x + y * y + z * z);
    if (w < 0.0) nn = -nn;
    q[0] = w / nn; q[1] = x / nn; q[2] = y / nn; q[3] = z / nn;
}

// ---- kernels ----------------------------------------------------------------------------

__global__ void k_reg_prep(const int64_t *__restrict__ count, int64_t cap, uint32_t *__restrict__ n32) {
    const int64_t c = *count;
    *n32 = (uint32_t)(c < cap ? c : cap);
}

__global__ void k_reg_keys(const as_region *__restrict__ recs, const uint32_t *__restrict__ n32, int64_t cap, int lb,
                           int vb, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap || i >= (int64_t)*n32) return;
    const as_region &r = recs[i];
    keys[i] = ((uint64_t)(uint32_t)r.cand << (vb + lb)) | ((uint64_t)(uint32_t)r.view << lb) | (uint64_t)(uint32_t)r.label;
    vals[i] = (uint32_t)i;
}

__global__ void k_cand_ranges(const as_region *__restrict__ recs, const uint32_t *__restrict__ order,
                              const uint32_t *__restrict__ n32, int64_t cap, const int32_t *__restrict__ cand,
                              int64_t n_cand, const int64_t *__restrict__ n_cand_dev, int64_t *__restrict__ rs,
                              int64_t *__restrict__ re) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t R = *n32;
    if (i >= cap || i >= R) return;
    const int32_t c = recs[order[i]].cand;
    const int64_t ci = find_cand(cand, count_in_use(n_cand, n_cand_dev), c);
    if (ci < 0) return;
    if (i == 0 || recs[order[i - 1]].cand != c) rs[ci] = i;
    if (i == R - 1 || recs[order[i + 1]].cand != c) re[ci] = i + 1;
}

__global__ void k_propose(GaussPtrs g, const as_region *__restrict__ recs, const uint32_t *__restrict__ order,
                          const uint32_t *__restrict__ n32, int64_t cap, const int32_t *__restrict__ cand,
                          int64_t n_cand, const int64_t *__restrict__ n_cand_dev, const DevCam *__restrict__ cams,
                          int n_views, double eps, Prop *__restrict__ props) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap || i >= (int64_t)*n32) return;
    const as_region r = recs[order[i]];
    Prop p;
    p.ok = 0;
    p.view = r.view;
    if (find_cand(cand, count_in_use(n_cand, n_cand_dev), r.cand) >= 0 && r.view >= 0 && r.view < n_views &&
        r.cand < rows_in_use(g)) {
        Parent par;
        load_parent(g, r.cand, par);
        make_proposal(par, r, cams[r.view], eps, p);
    }
    props[i] = p;
}

__device__ __forceinline__ int32_t uf_load(const int32_t *L, int64_t x) {
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

// One wave per candidate.
__global__ void __launch_bounds__(256) k_merge(GaussPtrs g, const int32_t *__restrict__ cand, int64_t n_cand,
                                               const int64_t *__restrict__ n_cand_dev,
                                               const int32_t *__restrict__ attr, const int64_t *__restrict__ rs_a,
                                               const int64_t *__restrict__ re_a, const Prop *__restrict__ props,
                                               int32_t *__restrict__ uf_all, int32_t *__restrict__ root_all,
                                               Group *__restrict__ grp_all, int32_t *__restrict__ kept_all,
                                               int32_t *__restrict__ nkept, double gamma_d, double gamma_c,
                                               int n_max, int variant, uint32_t flags, int fixed_n,
                                               uint8_t *__restrict__ mode, int32_t *__restrict__ count) {
    const int lane = threadIdx.x & 63;
    const int64_t ci = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ci >= n_cand) return;
    if (ci >= count_in_use(n_cand, n_cand_dev)) {   // capacity past the candidates in use: no rows
        if (lane == 0) {
            mode[ci] = 0;
            count[ci] = 0;
            nkept[ci] = 0;
        }
        return;
    }
    if (variant == AS_VARIANT_FIXED_N) {   // the random split with a fixed N, whatever the regions say
        if (lane == 0) {
            mode[ci] = 3;
            count[ci] = fixed_n;
            nkept[ci] = 0;
        }
        return;
    }
    const int64_t rs = rs_a[ci], re = re_a[ci];
    const int32_t np = (int32_t)(re - rs);
    const Prop *pp = props + rs;
    int32_t *uf = uf_all + rs;
    int32_t *rootof = root_all + rs;
    Group *grp = grp_all + rs;
    int32_t *kept = kept_all + rs;

    for (int32_t j = lane; j < np; j += 64) uf[j] = pp[j].ok ? j : -1;
    __threadfence();
    __builtin_amdgcn_wave_barrier();
    // Eq. (merge_conditions) over every pair of this parent's proposals (the
    // ablation variants do not merge)
    const bool merge = variant == AS_VARIANT_ADPSPLIT;
    for (int32_t a = 0; merge && a < np; a++) {
        if (!pp[a].ok) continue;
        for (int32_t b = a + 1 + lane; b < np; b += 64) {
            if (!pp[b].ok) continue;
            if ((flags & AS_SPLIT_CROSS_VIEW) && pp[b].view == pp[a].view) continue;
            const double dl[3] = {pp[b].mu[0] - pp[a].mu[0], pp[b].mu[1] - pp[a].mu[1], pp[b].mu[2] - pp[a].mu[2]};
            const double dm = maha(pp[a].Sinv, dl) + maha(pp[b].Sinv, dl);
            double dc = 0.0;
            for (int ch = 0; ch < 3; ch++) {
                const double t = fabs(pp[a].rgb[ch] - pp[b].rgb[ch]);
                if (t > dc) dc = t;
            }
            if (dm <= gamma_d && dc <= gamma_c) uf_unite(uf, a, b);
        }
    }
    __threadfence();
    __builtin_amdgcn_wave_barrier();
    for (int32_t j = lane; j < np; j += 64) rootof[j] = pp[j].ok ? uf_find(uf, j) : -1;
    __threadfence();
    __builtin_amdgcn_wave_barrier();

    // Eq. (merge_cov): one merged child per group, summed in member order
    int32_t nroots = 0;
    for (int32_t j0 = 0; j0 < np; j0 += 64) {
        const int32_t j = j0 + lane;
        const bool isroot = j < np && rootof[j] == j;
        nroots += (int32_t)__popcll(__ballot(isroot));
        if (!isroot) continue;
        Group gr;
        int64_t M = 0;
        double Sbar[9];
        for (int k = 0; k < 3; k++) { gr.mu[k] = 0.0; gr.rgb[k] = 0.0; }
        for (int k = 0; k < 9; k++) Sbar[k] = 0.0;
        for (int32_t m = j; m < np; m++) {
            if (rootof[m] != j) continue;
            M++;
            for (int k = 0; k < 3; k++) { gr.mu[k] += pp[m].mu[k]; gr.rgb[k] += pp[m].rgb[k]; }
            for (int k = 0; k < 9; k++) Sbar[k] += pp[m].Sig[k];
        }
        if (M == 1) {
            for (int k = 0; k < 3; k++) { gr.mu[k] = pp[j].mu[k]; gr.rgb[k] = pp[j].rgb[k]; gr.s[k] = pp[j].s[k]; }
            for (int k = 0; k < 9; k++) gr.R[k] = pp[j].R[k];
        } else {
            for (int k = 0; k < 3; k++) { gr.mu[k] = gr.mu[k] / (double)M; gr.rgb[k] = gr.rgb[k] / (double)M; }
            for (int k = 0; k < 9; k++) Sbar[k] = Sbar[k] / (double)M;
            double E[9], lam[3];
            jacobi3(Sbar, E, lam);
            for (int r = 0; r < 3; r++) {
                const double er[3] = {E[0 * 3 + r], E[1 * 3 + r], E[2 * 3 + r]};
                double best = 0.0;
                for (int32_t m = j; m < np; m++) {
                    if (rootof[m] != j) continue;
                    const double off = fabs(er[0] * (pp[m].mu[0] - gr.mu[0]) + er[1] * (pp[m].mu[1] - gr.mu[1]) +
                                            er[2] * (pp[m].mu[2] - gr.mu[2]));
                    double Se[3];
                    for (int k = 0; k < 3; k++)
                        Se[k] = pp[m].Sig[k * 3 + 0] * er[0] + pp[m].Sig[k * 3 + 1] * er[1] + pp[m].Sig[k * 3 + 2] * er[2];
                    const double sig = sqrt(er[0] * Se[0] + er[1] * Se[1] + er[2] * Se[2]);
                    const double reach = off + sig;
                    if (reach > best) best = reach;
                }
                gr.s[r] = best;
            }
            for (int k = 0; k < 9; k++) gr.R[k] = E[k];
        }
        if (flags & AS_SPLIT_EXTENT_MAX) {
            double m = gr.s[0];
            if (gr.s[1] > m) m = gr.s[1];
            if (gr.s[2] > m) m = gr.s[2];
            gr.extent = m;
        } else {
            gr.extent = gr.s[0] * gr.s[1] * gr.s[2];
        }
        grp[j] = gr;
    }
    __threadfence();
    __builtin_amdgcn_wave_barrier();
    // rank by (extent descending, first member ascending); keep N_max
    for (int32_t j = lane; j < np; j += 64) {
        if (rootof[j] != j) continue;
        const double ej = grp[j].extent;
        int32_t rank = 0;
        for (int32_t h = 0; h < np; h++) {
            if (h == j || rootof[h] != h) continue;
            const double eh = grp[h].extent;
            if (eh > ej || (eh == ej && h < j)) rank++;
        }
        if (rank < n_max) kept[rank] = j;
    }
    if (lane == 0) {
        const int32_t nk = nroots < n_max ? nroots : n_max;
        const int32_t id = cand[ci];
        uint8_t md;
        int32_t cnt;
        if (attr[id] == 0) { md = 0; cnt = 2; }
        else if (nk == 0) { md = 1; cnt = 0; }
        else if (variant == AS_VARIANT_ADAPTIVE_N) { md = 3; cnt = nk; }   // as many random children as proposals
        else { md = 2; cnt = nk + 1; }
        mode[ci] = md;
        count[ci] = cnt;
        nkept[ci] = nk;
    }
}

__global__ void k_mark_removed(const int32_t *__restrict__ cand, int64_t n_cand, const int64_t *__restrict__ n_cand_dev,
                               const uint8_t *__restrict__ mode, uint8_t *__restrict__ removed) {
    const int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ci >= count_in_use(n_cand, n_cand_dev)) return;
    if (mode[ci] != 1) removed[cand[ci]] = 1;
}

__global__ void k_copy_survivors(GaussPtrs g, const uint8_t *__restrict__ removed,
                                 const int64_t *__restrict__ rem_prefix, GradPtrs out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows_in_use(g) || removed[i]) return;
    const int64_t n = g.n, os = out.stride;
    const int64_t d = i - rem_prefix[i];
    const int nk = (g.deg + 1) * (g.deg + 1);
    for (int k = 0; k < 3; k++) out.means[k * os + d] = g.means[k * n + i];
    for (int k = 0; k < 3; k++) out.log_scales[k * os + d] = g.log_scales[k * n + i];
    for (int k = 0; k < 4; k++) out.quats[k * os + d] = g.quats[k * n + i];
    out.opac[d] = g.opac[i];
    for (int k = 0; k < nk * 3; k++) out.sh[(int64_t)k * os + d] = g.sh[(int64_t)k * n + i];
}

__device__ __forceinline__ void copy_row(const GaussPtrs &g, int64_t src, GradPtrs &out, int64_t dst) {
    const int64_t n = g.n, os = out.stride;
    const int nk = (g.deg + 1) * (g.deg + 1);
    for (int k = 0; k < 3; k++) out.means[k * os + dst] = g.means[k * n + src];
    for (int k = 0; k < 3; k++) out.log_scales[k * os + dst] = g.log_scales[k * n + src];
    for (int k = 0; k < 4; k++) out.quats[k * os + dst] = g.quats[k * n + src];
    out.opac[dst] = g.opac[src];
    for (int k = 0; k < nk * 3; k++) out.sh[(int64_t)k * os + dst] = g.sh[(int64_t)k * n + src];
}

__global__ void k_write_children(GaussPtrs g, const int32_t *__restrict__ cand, int64_t n_cand,
                                 const int64_t *__restrict__ n_cand_dev, const uint8_t *__restrict__ mode, const int64_t *__restrict__ offset,
                                 const int64_t *__restrict__ tot, const int64_t *__restrict__ rs_a,
                                 const Group *__restrict__ grp_all, const int32_t *__restrict__ kept_all,
                                 const int32_t *__restrict__ nkept, const int32_t *__restrict__ count,
                                 const float *__restrict__ noise, int noise_n, double eta, uint32_t flags,
                                 GradPtrs out, int64_t *__restrict__ n_out) {
    const int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_surv = rows_in_use(g) - tot[0];
    if (ci == 0) *n_out = n_surv + tot[1];
    if (ci >= count_in_use(n_cand, n_cand_dev)) return;
    const int64_t base = n_surv + offset[ci];
    const int32_t id = cand[ci];
    const uint8_t md = mode[ci];
    const int64_t os = out.stride;
    const int nk = (g.deg + 1) * (g.deg + 1);
    if (md == 0 || md == 3) {
        // Eq. (vanilla_split_sample), Eq. (vanilla_split_scale) with N = count
        // (2 for the VANILLA fallback)
        const int32_t N = count[ci];
        Parent par;
        load_parent(g, id, par);
        for (int c2 = 0; c2 < N; c2++) {
            const int64_t dst = base + c2;
            copy_row(g, id, out, dst);
            double dl[3];
            for (int k = 0; k < 3; k++) dl[k] = par.s[k] * (double)noise[((int64_t)ci * noise_n + c2) * 3 + k];
            for (int k = 0; k < 3; k++) {
                const double m = par.mu[k] + (par.R[k * 3 + 0] * dl[0] + par.R[k * 3 + 1] * dl[1] + par.R[k * 3 + 2] * dl[2]);
                out.means[k * os + dst] = (float)m;
                out.log_scales[k * os + dst] = (float)((double)g.log_scales[k * g.n + id] - log(eta * (double)N));
            }
        }
    } else if (md == 2) {
        const int64_t rs = rs_a[ci];
        const int32_t ng = nkept[ci];
        for (int32_t r = 0; r < ng; r++) {
            const Group gr = grp_all[rs + kept_all[rs + r]];
            const int64_t dst = base + r;
            double q[4];
            rot_to_quat(gr.R, q);
            for (int k = 0; k < 3; k++) out.means[k * os + dst] = (float)gr.mu[k];
            for (int k = 0; k < 3; k++) out.log_scales[k * os + dst] = (float)log(gr.s[k]);
            for (int k = 0; k < 4; k++) out.quats[k * os + dst] = (float)q[k];
            out.opac[dst] = g.opac[id];   // Eq. (child_params): the parent's opacity
            for (int ch = 0; ch < 3; ch++) out.sh[(int64_t)ch * os + dst] = (float)((gr.rgb[ch] - 0.5) / C0_SH);
            for (int k = 3; k < nk * 3; k++) out.sh[(int64_t)k * os + dst] = 0.0f;
        }
        const int64_t dst = base + ng;
        copy_row(g, id, out, dst);
        const double o = 1.0 / (1.0 + exp(-(double)g.opac[id]));
        const double pr = o / (double)(ng + 1);
        const float shared = (float)log(pr / (1.0 - pr));
        out.opac[dst] = shared;
        if (flags & AS_SPLIT_SHARE_OPACITY)   // second reading: every row of the block at o/(N+1)
            for (int32_t r = 0; r < ng; r++) out.opac[base + r] = shared;
    }
}

int bits_for(int64_t v) {   // bits needed to represent 0..v
    int b = 1;
    while ((int64_t(1) << b) <= v && b < 62) b++;
    return b;
}

constexpr int CAM_CHUNK = 16;
struct CamChunk {
    int m;
    DevCam cam[CAM_CHUNK];
};
__global__ void k_store_cams(const CamChunk c, DevCam *__restrict__ dst) {
    if ((int)threadIdx.x < c.m) dst[threadIdx.x] = c.cam[threadIdx.x];
}

}  // namespace

// Bytes of each scratch slot for region capacity `cap`, `nc` candidates, `nv`
// views and `n` Gaussians: the region sort's keys, values and histogram, the
// candidates' region ranges, proposals, union-find, groups and kept lists,
// the camera table, the removal mask and its scan.
static void sp_need(int64_t cap, int64_t nc, int64_t nv, int64_t n, size_t need[SP_COUNT]) {
    cap = cap > 0 ? cap : 1;
    nc = nc > 0 ? nc : 1;
    nv = nv > 0 ? nv : 1;
    n = n > 0 ? n : 1;
    const size_t v[SP_COUNT] = {(size_t)cap * 8, (size_t)cap * 8, (size_t)cap * 4, (size_t)cap * 4, sort_hist_bytes(cap),
                                64, (size_t)nc * 8, (size_t)nc * 8, (size_t)cap * sizeof(Prop), (size_t)cap * 4,
                                (size_t)cap * 4, (size_t)cap * sizeof(Group), (size_t)cap * 4, (size_t)nc * 4,
                                (size_t)nv * sizeof(DevCam), (size_t)n, (size_t)n * 8, scan_tmp_bytes(n > nc ? n : nc),
                                64};
    for (int k = 0; k < SP_COUNT; k++) need[k] = v[k];
}

size_t split_reserve_bytes(const as_reserve &r) {
    size_t need[SP_COUNT], total = 0;
    sp_need(r.max_regions, r.max_candidates, r.max_views, r.max_gaussians, need);
    for (int k = 0; k < SP_COUNT; k++) total += devbuf_size(need[k]);
    return total;
}

hipError_t split_reserve(as_ctx *ctx, const as_reserve &r) {
    size_t need[SP_COUNT];
    sp_need(r.max_regions, r.max_candidates, r.max_views, r.max_gaussians, need);
    hipError_t e = hipSuccess;
    for (int k = 0; k < SP_COUNT && e == hipSuccess; k++) e = devbuf_ensure(ctx->sp[k], need[k]);
    return e;
}

as_status run_adaptive_split(as_ctx *ctx, const GaussPtrs &g, const int32_t *cand, int64_t n_cand,
                             const int64_t *n_cand_dev, const as_region_buf &rb, const as_camera *views, int n_views, const int32_t *attr,
                             const as_split_params &p, const float *noise, GradPtrs out, int64_t out_cap,
                             uint8_t *mode, int32_t *count, int64_t *offset, int64_t *n_out, hipStream_t s) {
    (void)out_cap;
    const int64_t cap = rb.capacity > 0 ? rb.capacity : 1;
    int64_t max_px = 1;
    for (int v = 0; v < n_views; v++) {
        const int64_t px = (int64_t)views[v].width * views[v].height;
        if (px > max_px) max_px = px;
    }
    const int lb = bits_for(max_px), vb = bits_for(n_views > 0 ? n_views : 1), cb = bits_for(g.n);
    if (lb + vb + cb > 64) {
        as_set_error("region sort key needs %d bits (> 64)", lb + vb + cb);
        return AS_ERR_ARG;
    }
    // the scratch sizes of sp_need (every count at least 1) must be reserved
    const int64_t nc1 = n_cand > 0 ? n_cand : 1, nv1 = n_views > 0 ? n_views : 1, n1 = g.n > 0 ? g.n : 1;
    const as_reserve &res = ctx->res;
    if (cap > res.max_regions || nc1 > res.max_candidates || nv1 > res.max_views || n1 > res.max_gaussians) {
        as_set_error("as_adaptive_split: needs max_regions >= %lld, max_candidates >= %lld, max_views >= %lld, "
                     "max_gaussians >= %lld in as_ctx_reserve (reserved %lld, %lld, %d, %lld)", (long long)cap,
                     (long long)nc1, (long long)nv1, (long long)n1, (long long)res.max_regions,
                     (long long)res.max_candidates, res.max_views, (long long)res.max_gaussians);
        return AS_ERR_CAPACITY;
    }
    DevBuf *sp = ctx->sp;
    uint64_t *keys[2] = {(uint64_t *)sp[SP_K0].p, (uint64_t *)sp[SP_K1].p};
    uint32_t *vals[2] = {(uint32_t *)sp[SP_V0].p, (uint32_t *)sp[SP_V1].p};
    uint32_t *n32 = (uint32_t *)sp[SP_N].p;
    int64_t *rs = (int64_t *)sp[SP_RS].p, *re = (int64_t *)sp[SP_RE].p, *tot = (int64_t *)sp[SP_TOT].p;
    Prop *props = (Prop *)sp[SP_PROP].p;
    Group *grp = (Group *)sp[SP_GRP].p;
    int32_t *uf = (int32_t *)sp[SP_UF].p, *rootof = (int32_t *)sp[SP_ROOT].p, *kept = (int32_t *)sp[SP_KEPT].p;
    int32_t *nkept = (int32_t *)sp[SP_NKEPT].p;
    DevCam *dcams = (DevCam *)sp[SP_CAMS].p;
    uint8_t *removed = (uint8_t *)sp[SP_REM].p;
    int64_t *remscan = (int64_t *)sp[SP_REMSCAN].p;

    // cameras travel as kernel arguments (no host copy, no synchronisation)
    for (int v0 = 0; v0 < n_views; v0 += CAM_CHUNK) {
        CamChunk cc;
        cc.m = n_views - v0 < CAM_CHUNK ? n_views - v0 : CAM_CHUNK;
        for (int k = 0; k < cc.m; k++) cc.cam[k] = to_devcam(views[v0 + k]);
        hipLaunchKernelGGL(k_store_cams, dim3(1), dim3(64), 0, s, cc, dcams + v0);
    }
    const unsigned gcap = (unsigned)((cap + 255) / 256);
    hipLaunchKernelGGL(k_reg_prep, dim3(1), dim3(1), 0, s, rb.count, cap, n32);
    hipLaunchKernelGGL(k_reg_keys, dim3(gcap), dim3(256), 0, s, rb.records, n32, cap, lb, vb, keys[0], vals[0]);
    const int sel = radix_sort_u64(keys, vals, n32, cap, cap, 0, lb + vb + cb, 8, sp[SP_HIST].p, s);
    const uint32_t *order = vals[sel];
    launch_fill_i64(rs, 0, nc1, s);
    launch_fill_i64(re, 0, nc1, s);
    hipLaunchKernelGGL(k_cand_ranges, dim3(gcap), dim3(256), 0, s, rb.records, order, n32, cap, cand, n_cand,
                       n_cand_dev, rs, re);
    hipLaunchKernelGGL(k_propose, dim3(gcap), dim3(256), 0, s, g, rb.records, order, n32, cap, cand, n_cand,
                       n_cand_dev, dcams,
                       n_views, p.eps, props);
    if (n_cand > 0)
        hipLaunchKernelGGL(k_merge, dim3((unsigned)((n_cand + 3) / 4)), dim3(256), 0, s, g, cand, n_cand, n_cand_dev,
                           attr, rs,
                           re, props, uf, rootof, grp, kept, nkept, p.gamma_d, p.gamma_c, p.n_max, p.variant, p.flags,
                           p.fixed_n, mode, count);
    scan_i32_to_i64(count, offset, n_cand, tot + 1, sp[SP_SCAN].p, s);
    launch_fill_u8(removed, 0, g.n > 0 ? g.n : 1, s);
    if (n_cand > 0)
        hipLaunchKernelGGL(k_mark_removed, dim3((unsigned)((n_cand + 255) / 256)), dim3(256), 0, s, cand, n_cand,
                           n_cand_dev,
                           mode, removed);
    scan_u8_to_i64(removed, remscan, g.n, tot, sp[SP_SCAN].p, s);
    if (g.n > 0)
        hipLaunchKernelGGL(k_copy_survivors, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s, g, removed,
                           remscan, out);
    hipLaunchKernelGGL(k_write_children, dim3((unsigned)((nc1 + 255) / 256)), dim3(256), 0, s, g, cand, n_cand,
                       n_cand_dev, mode,
                       offset, tot, rs, grp, kept, nkept, count, noise, p.noise_n ? p.noise_n : 2, p.eta, p.flags, out,
                       n_out);
    return AS_OK;
}

AS_WARM_KERNEL(split)
