/*
 * CPU FP64 oracle for the differentiable Gaussian rasterizer and the AdpSplit
 * adaptive split ("AdpSplit: error-driven adaptive splitting", arxiv 2605.06876).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, headers or constant tables with the HIP kernels.
 *
 * Style: plain loops in the order the paper states the method, every float
 * value widened to double on entry, no blocking or reordering beyond the
 * definition.  Built with -ffp-contract=off so that every expression rounds
 * exactly as written.
 *
 * Conventions (readings of points the paper leaves open are marked [Ann]):
 *  - Parameters are stored raw: scale s = exp(log_scale), opacity
 *    o = 1/(1+exp(-logit)), rotation from the normalised quaternion (w,x,y,z)
 *    [A1; Sec. 3 defines s, R, o only].
 *  - Camera: world->camera rotation R (row-major) and translation t; camera
 *    axes x right, y down, z forward, so rows 0,1,2 of R are the camera's
 *    right, down and forward directions in world space [A3; App. A].
 *  - Continuous pixel frame: the centre of pixel (x, y) is (x+1/2, y+1/2) [A2].
 *  - 3DGS rasterizer constants: near plane 0.2, low-pass 0.3, alpha clamp 0.99,
 *    skip alpha < 1/255, stop once transmittance would fall below 1e-4 [A5].
 *  - The per-Gaussian "compact box" is the exact axis-aligned box of the
 *    ellipse where alpha >= 1/255 [A4; Sec. 5 "Implementation" cites the
 *    compact-box method without defining it].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NEAR_PLANE 0.2
#define LOWPASS 0.3
#define ALPHA_MIN (1.0 / 255.0)
#define ALPHA_MAX 0.99
#define T_STOP 1e-4

/* ------------------------------------------------------------------------ */
/* Camera: packed as 21 doubles R[9], t[3], fx, fy, cx, cy, W, H, bg[3].    */
/* ------------------------------------------------------------------------ */
typedef struct {
    double R[9], t[3], fx, fy, cx, cy;
    int W, H;
    double bg[3];
} ocam;

static void cam_unpack(const double *c, ocam *o) {
    for (int k = 0; k < 9; k++) o->R[k] = c[k];
    for (int k = 0; k < 3; k++) o->t[k] = c[9 + k];
    o->fx = c[12]; o->fy = c[13]; o->cx = c[14]; o->cy = c[15];
    o->W = (int)c[16]; o->H = (int)c[17];
    for (int k = 0; k < 3; k++) o->bg[k] = c[18 + k];
}

/* Camera centre in world space: o_v = -R^T t (App. A, ray origin). */
static void cam_centre(const ocam *c, double o[3]) {
    for (int j = 0; j < 3; j++)
        o[j] = -(c->R[0 * 3 + j] * c->t[0] + c->R[1 * 3 + j] * c->t[1] + c->R[2 * 3 + j] * c->t[2]);
}

/* ------------------------------------------------------------------------ */
/* Sec. 3: activations, rotation and 3D covariance Sigma = R S S^T R^T.     */
/* ------------------------------------------------------------------------ */
static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Rotation matrix of the unit quaternion (w, x, y, z), row-major. */
static void quat_to_rot(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Load Gaussian i from the SoA arrays: mean, scale, normalised quaternion,
 * rotation, opacity. */
typedef struct {
    double mu[3], s[3], qn[4], qnorm, R[9], o;
} ogauss;

static void load_gauss(int64_t n, int64_t i, const float *means, const float *log_scales,
                       const float *quats, const float *opac, ogauss *g) {
    for (int k = 0; k < 3; k++) g->mu[k] = (double)means[k * n + i];
    for (int k = 0; k < 3; k++) g->s[k] = exp((double)log_scales[k * n + i]);
    double q[4];
    for (int k = 0; k < 4; k++) q[k] = (double)quats[k * n + i];
    g->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; k++) g->qn[k] = q[k] / g->qnorm;
    quat_to_rot(g->qn, g->R);
    g->o = sigmoid((double)opac[i]);
}

/* Sigma = R diag(s^2) R^T, entry (a, b). */
static void cov3d(const double R[9], const double s[3], double S[9]) {
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += R[a * 3 + k] * (s[k] * s[k]) * R[b * 3 + k];
            S[a * 3 + b] = acc;
        }
}

/* ------------------------------------------------------------------------ */
/* Sec. 3: view-dependent colour c_i(d_v) from real spherical harmonics.    */
/* Real SH with the Condon-Shortley phase, degree <= 3 [A6]; normalisation  */
/* constants are evaluated from their closed forms sqrt((2l+1)/(4 pi) ...). */
/* ------------------------------------------------------------------------ */
static void sh_basis(double x, double y, double z, double Y[16]) {
    const double pi = 3.14159265358979323846;
    double k00 = sqrt(1.0 / (4.0 * pi));
    double k1 = sqrt(3.0 / (4.0 * pi));
    double k2a = sqrt(15.0 / (4.0 * pi));   /* xy, yz, xz */
    double k20 = sqrt(5.0 / (16.0 * pi));   /* 3z^2-1 */
    double k22 = sqrt(15.0 / (16.0 * pi));  /* x^2-y^2 */
    double k33 = sqrt(35.0 / (32.0 * pi));
    double k32 = sqrt(105.0 / (4.0 * pi));
    double k31 = sqrt(21.0 / (32.0 * pi));
    double k30 = sqrt(7.0 / (16.0 * pi));
    double k32b = sqrt(105.0 / (16.0 * pi));
    double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = k00;
    Y[1] = -k1 * y;
    Y[2] = k1 * z;
    Y[3] = -k1 * x;
    Y[4] = k2a * x * y;
    Y[5] = -k2a * y * z;
    Y[6] = k20 * (2.0 * zz - xx - yy);
    Y[7] = -k2a * x * z;
    Y[8] = k22 * (xx - yy);
    Y[9] = -k33 * y * (3.0 * xx - yy);
    Y[10] = k32 * x * y * z;
    Y[11] = -k31 * y * (4.0 * zz - xx - yy);
    Y[12] = k30 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -k31 * x * (4.0 * zz - xx - yy);
    Y[14] = k32b * z * (xx - yy);
    Y[15] = -k33 * x * (xx - 3.0 * yy);
}

/* Partial derivatives dY_k/dx, dY_k/dy, dY_k/dz of the polynomials above,
 * treating (x, y, z) as independent (the unit-norm constraint is applied by
 * the caller through the normalisation Jacobian). */
static void sh_basis_grad(double x, double y, double z, double dY[16][3]) {
    const double pi = 3.14159265358979323846;
    double k1 = sqrt(3.0 / (4.0 * pi));
    double k2a = sqrt(15.0 / (4.0 * pi));
    double k20 = sqrt(5.0 / (16.0 * pi));
    double k22 = sqrt(15.0 / (16.0 * pi));
    double k33 = sqrt(35.0 / (32.0 * pi));
    double k32 = sqrt(105.0 / (4.0 * pi));
    double k31 = sqrt(21.0 / (32.0 * pi));
    double k30 = sqrt(7.0 / (16.0 * pi));
    double k32b = sqrt(105.0 / (16.0 * pi));
    double xx = x * x, yy = y * y, zz = z * z;
    memset(dY, 0, sizeof(double) * 48);
    dY[1][1] = -k1;
    dY[2][2] = k1;
    dY[3][0] = -k1;
    dY[4][0] = k2a * y; dY[4][1] = k2a * x;
    dY[5][1] = -k2a * z; dY[5][2] = -k2a * y;
    dY[6][0] = -2.0 * k20 * x; dY[6][1] = -2.0 * k20 * y; dY[6][2] = 4.0 * k20 * z;
    dY[7][0] = -k2a * z; dY[7][2] = -k2a * x;
    dY[8][0] = 2.0 * k22 * x; dY[8][1] = -2.0 * k22 * y;
    /* Y9 = -k33 (3 x^2 y - y^3) */
    dY[9][0] = -k33 * 6.0 * x * y; dY[9][1] = -k33 * (3.0 * xx - 3.0 * yy);
    /* Y10 = k32 x y z */
    dY[10][0] = k32 * y * z; dY[10][1] = k32 * x * z; dY[10][2] = k32 * x * y;
    /* Y11 = -k31 (4 y z^2 - x^2 y - y^3) */
    dY[11][0] = -k31 * (-2.0 * x * y); dY[11][1] = -k31 * (4.0 * zz - xx - 3.0 * yy); dY[11][2] = -k31 * 8.0 * y * z;
    /* Y12 = k30 (2 z^3 - 3 x^2 z - 3 y^2 z) */
    dY[12][0] = k30 * (-6.0 * x * z); dY[12][1] = k30 * (-6.0 * y * z); dY[12][2] = k30 * (6.0 * zz - 3.0 * xx - 3.0 * yy);
    /* Y13 = -k31 (4 x z^2 - x^3 - x y^2) */
    dY[13][0] = -k31 * (4.0 * zz - 3.0 * xx - yy); dY[13][1] = -k31 * (-2.0 * x * y); dY[13][2] = -k31 * 8.0 * x * z;
    /* Y14 = k32b (x^2 z - y^2 z) */
    dY[14][0] = k32b * 2.0 * x * z; dY[14][1] = -k32b * 2.0 * y * z; dY[14][2] = k32b * (xx - yy);
    /* Y15 = -k33 (x^3 - 3 x y^2) */
    dY[15][0] = -k33 * (3.0 * xx - 3.0 * yy); dY[15][1] = -k33 * (-6.0 * x * y);
}

/* Exported for the orthonormality pin. */
void orc_sh_basis(double x, double y, double z, double *Y) { sh_basis(x, y, z, Y); }

/* ------------------------------------------------------------------------ */
/* Sec. 3 (projection to the image plane): EWA projection, culling, colour, */
/* depth key and compact box for every Gaussian.                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int valid;          /* passes culling and has a non-empty box inside the image */
    double t[3];        /* view-space centre */
    double mean[2];     /* image-plane mean (continuous pixel frame) */
    double cov[3];      /* 2D covariance incl. low-pass: xx, xy, yy */
    double conic[3];    /* inverse 2D covariance: xx, xy, yy */
    double rgb[3];
    int clamped[3];     /* colour channel clamped at 0 */
    double o;
    uint32_t depth_key; /* bits of float(t_z) */
    int box[4];         /* inclusive pixel range x0, y0, x1, y1 */
    int box_flag;       /* a culling or box-edge decision lies within transcendental rounding of its threshold */
} oproj;

/* Box decisions go through exp (scale, opacity) and log (the alpha level); a
 * device's FP64 exp and log may differ from the host's by an ulp, so a value
 * this close (relative) to a threshold can round either way.  The margin is
 * far above an ulp (about 1e6 of them) and still flags almost nothing. */
#define FLAG_BOX_REL 1e-10

/* distance of v to the nearest integer, relative to the magnitudes forming v */
static int near_integer(double v, double scale) {
    return fabs(v - nearbyint(v)) <= FLAG_BOX_REL * (scale + 1.0);
}

static int project_one(int64_t n, int deg, int64_t i, const float *means, const float *log_scales,
                       const float *quats, const float *opac, const float *sh, const ocam *c, oproj *p) {
    memset(p, 0, sizeof(*p));
    ogauss g;
    load_gauss(n, i, means, log_scales, quats, opac, &g);
    p->o = g.o;
    /* view space */
    for (int r = 0; r < 3; r++)
        p->t[r] = c->R[r * 3 + 0] * g.mu[0] + c->R[r * 3 + 1] * g.mu[1] + c->R[r * 3 + 2] * g.mu[2] + c->t[r];
    double tx = p->t[0], ty = p->t[1], tz = p->t[2];
    p->depth_key = 0;
    {
        float fz = (float)tz;
        memcpy(&p->depth_key, &fz, 4);
    }
    if (!(tz > NEAR_PLANE)) return 0;
    /* EWA: J is the Jacobian of the perspective map at the (clamped) centre. */
    double limx = 1.3 * ((double)c->W / (2.0 * c->fx));
    double limy = 1.3 * ((double)c->H / (2.0 * c->fy));
    double txtz = tx / tz, tytz = ty / tz;
    double cx_ = fmin(limx, fmax(-limx, txtz)) * tz;
    double cy_ = fmin(limy, fmax(-limy, tytz)) * tz;
    double J[6] = {c->fx / tz, 0.0, -(c->fx * cx_) / (tz * tz),
                   0.0, c->fy / tz, -(c->fy * cy_) / (tz * tz)};
    double T[6]; /* T = J W, W = camera rotation */
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++)
            T[r * 3 + k] = J[r * 3 + 0] * c->R[0 * 3 + k] + J[r * 3 + 1] * c->R[1 * 3 + k] + J[r * 3 + 2] * c->R[2 * 3 + k];
    double S[9];
    cov3d(g.R, g.s, S);
    double C2[4];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++)
                for (int l = 0; l < 3; l++) acc += T[a * 3 + k] * S[k * 3 + l] * T[b * 3 + l];
            C2[a * 2 + b] = acc;
        }
    double A = C2[0] + LOWPASS, B = C2[1], Cc = C2[3] + LOWPASS;
    p->cov[0] = A; p->cov[1] = B; p->cov[2] = Cc;
    double det = A * Cc - B * B;
    if (!(det > 0.0)) return 0;
    p->conic[0] = Cc / det; p->conic[1] = -B / det; p->conic[2] = A / det;
    p->mean[0] = c->fx * tx / tz + c->cx;
    p->mean[1] = c->fy * ty / tz + c->cy;
    /* colour (Sec. 3): SH evaluated along the unit view direction */
    double oc[3];
    cam_centre(c, oc);
    double v[3] = {g.mu[0] - oc[0], g.mu[1] - oc[1], g.mu[2] - oc[2]};
    double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double Y[16];
    sh_basis(v[0] / vn, v[1] / vn, v[2] / vn, Y);
    int nk = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0.0;
        for (int k = 0; k < nk; k++) acc += Y[k] * (double)sh[((int64_t)k * 3 + ch) * n + i];
        acc += 0.5;
        p->clamped[ch] = acc < 0.0;
        p->rgb[ch] = acc < 0.0 ? 0.0 : acc;
    }
    /* compact box: alpha >= 1/255 <=> d^T conic d <= 2 ln(255 o) */
    if (fabs(255.0 * g.o - 1.0) <= FLAG_BOX_REL) p->box_flag = 1;
    if (!(g.o >= ALPHA_MIN)) return 0;
    double kk = 2.0 * log(255.0 * g.o);
    double hx = sqrt(kk * A), hy = sqrt(kk * Cc);
    {
        double sx = fabs(p->mean[0]) + hx, sy = fabs(p->mean[1]) + hy;
        if (near_integer(p->mean[0] - hx - 0.5, sx) || near_integer(p->mean[0] + hx - 0.5, sx) ||
            near_integer(p->mean[1] - hy - 0.5, sy) || near_integer(p->mean[1] + hy - 0.5, sy))
            p->box_flag = 1;
    }
    double x0 = ceil(p->mean[0] - hx - 0.5), x1 = floor(p->mean[0] + hx - 0.5);
    double y0 = ceil(p->mean[1] - hy - 0.5), y1 = floor(p->mean[1] + hy - 0.5);
    x0 = fmax(x0, 0.0); y0 = fmax(y0, 0.0);
    x1 = fmin(x1, (double)(c->W - 1)); y1 = fmin(y1, (double)(c->H - 1));
    if (!(x0 <= x1 && y0 <= y1)) return 0;
    p->box[0] = (int)x0; p->box[1] = (int)y0; p->box[2] = (int)x1; p->box[3] = (int)y1;
    p->valid = 1;
    return 1;
}

/* Bulk projection; all outputs are per-Gaussian rows. */
void orc_project(int64_t n, int deg, const float *means, const float *log_scales, const float *quats,
                 const float *opac, const float *sh, const double *cam_packed,
                 int32_t *valid, double *mean2d, double *cov2d, double *conic, double *rgb, double *opacity,
                 double *tview, uint32_t *depth_key, int32_t *box, uint8_t *box_flag) {
    ocam c;
    cam_unpack(cam_packed, &c);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        oproj p;
        project_one(n, deg, i, means, log_scales, quats, opac, sh, &c, &p);
        valid[i] = p.valid;
        for (int k = 0; k < 2; k++) mean2d[i * 2 + k] = p.mean[k];
        for (int k = 0; k < 3; k++) cov2d[i * 3 + k] = p.cov[k];
        for (int k = 0; k < 3; k++) conic[i * 3 + k] = p.conic[k];
        for (int k = 0; k < 3; k++) rgb[i * 3 + k] = p.rgb[k];
        for (int k = 0; k < 3; k++) tview[i * 3 + k] = p.t[k];
        opacity[i] = p.o;
        depth_key[i] = p.depth_key;
        for (int k = 0; k < 4; k++) box[i * 4 + k] = p.valid ? p.box[k] : 0;
        if (box_flag) box_flag[i] = (uint8_t)p.box_flag;
    }
}

/* ------------------------------------------------------------------------ */
/* Tile binning by brute force: every (tile, Gaussian) pair whose pixel     */
/* ranges intersect, key = tile << 32 | depth bits, then a stable sort.     */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t key; uint32_t val; int64_t seq; } opair;

static int pair_cmp(const void *a, const void *b) {
    const opair *x = (const opair *)a, *y = (const opair *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->seq < y->seq ? -1 : (x->seq > y->seq);   /* stability: emission order */
}

/* Returns the number of pairs K (or -K-1 if it exceeds cap, nothing written). */
int64_t orc_bin(int64_t n, const int32_t *valid, const int32_t *box, const uint32_t *depth_key,
                int W, int H, int TW, int TH, uint64_t *keys, uint32_t *vals, uint32_t *ranges, int64_t cap) {
    int ntx = (W + TW - 1) / TW, nty = (H + TH - 1) / TH;
    int64_t K = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!valid[i]) continue;
        int tx0 = box[i * 4 + 0] / TW, ty0 = box[i * 4 + 1] / TH;
        int tx1 = box[i * 4 + 2] / TW, ty1 = box[i * 4 + 3] / TH;
        K += (int64_t)(tx1 - tx0 + 1) * (ty1 - ty0 + 1);
    }
    if (K > cap) return -K - 1;
    opair *pairs = (opair *)malloc(sizeof(opair) * (size_t)(K > 0 ? K : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!valid[i]) continue;
        int tx0 = box[i * 4 + 0] / TW, ty0 = box[i * 4 + 1] / TH;
        int tx1 = box[i * 4 + 2] / TW, ty1 = box[i * 4 + 3] / TH;
        for (int ty = ty0; ty <= ty1; ty++)
            for (int tx = tx0; tx <= tx1; tx++) {
                uint64_t tile = (uint64_t)ty * ntx + tx;
                pairs[m].key = (tile << 32) | depth_key[i];
                pairs[m].val = (uint32_t)i;
                pairs[m].seq = m;
                m++;
            }
    }
    qsort(pairs, (size_t)K, sizeof(opair), pair_cmp);
    for (int64_t k = 0; k < K; k++) { keys[k] = pairs[k].key; vals[k] = pairs[k].val; }
    int64_t ntiles = (int64_t)ntx * nty;
    for (int64_t t = 0; t < 2 * ntiles; t++) ranges[t] = 0;
    for (int64_t k = 0; k < K; k++) {
        uint64_t tile = keys[k] >> 32;
        if (k == 0 || (keys[k - 1] >> 32) != tile) ranges[tile * 2] = (uint32_t)k;
        if (k == K - 1 || (keys[k + 1] >> 32) != tile) ranges[tile * 2 + 1] = (uint32_t)(k + 1);
    }
    free(pairs);
    return K;
}

/* ------------------------------------------------------------------------ */
/* Eq. (rendering) and Eq. (dominant-map): per-pixel front-to-back          */
/* compositing over every Gaussian in ascending (depth key, id) order.      */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t key; int64_t id; } odepth;

static int depth_cmp(const void *a, const void *b) {
    const odepth *x = (const odepth *)a, *y = (const odepth *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

static int64_t depth_order(int64_t n, const int32_t *valid, const uint32_t *depth_key, int64_t *order) {
    odepth *d = (odepth *)malloc(sizeof(odepth) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        if (valid[i]) { d[m].key = depth_key[i]; d[m].id = i; m++; }
    qsort(d, (size_t)m, sizeof(odepth), depth_cmp);
    for (int64_t k = 0; k < m; k++) order[k] = d[k].id;
    free(d);
    return m;
}

/* Near-threshold flags (reading B1).  The GPU takes the blend's decisions
 * (alpha vs 1/255, T (1 - alpha) vs 1e-4, the dominant weight's lead, o G vs
 * the 0.99 clamp) in FP32; a pixel is flagged, and left out of the exact
 * comparisons, when the FP64 value of one of them lies within an error bound
 * of the FP32 evaluation from its threshold.
 *
 * Alpha: the kernel forms the exponent from the conic rounded to FP32, the
 * pixel offset from the FP32 mean and a few fused multiply-adds, so the error
 * of the exponent is a few units of roundoff u = 2^-24 times the summed
 * magnitudes of its terms (M below; large for thin, tilted ellipses, where
 * the terms cancel), plus the offset's rounding (at most u (|d| + 16)) times
 * the exponent's gradient, plus the rounding of log2(o) and exp2.  The
 * relative bound of o G is FP32_K u (2 M + |grad| (|dx| + |dy| + 32) + 4)
 * with FP32_K = 16, several times the count of roundings.
 * Transmittance: T's relative error grows by a_k e_k / (1 - a_k) + 2u per
 * contributor (e_k: its alpha bound), or by 1e-6 + 2u for a clamped one.
 * Weights a T carry the sum of the two.  Every decision is compared in units
 * of its bound (plus a floor of FLAG_FLOOR): a margin of at most 1 flags. */
#define U32 5.9604644775390625e-8   /* 2^-24 */
/* The clamp 0.99 in FP32 is 0.99 + 9.5e-9, so a clamped contributor's
 * 1 - alpha is 9.5e-7 smaller, relatively, than in FP64. */
#define CLAMP_ONE_MINUS_REL 1e-6
#define FP32_K 16.0
#define FLAG_FLOOR 1e-6

/* Relative error bound of the blend's FP32 o G at offset (dx, dy) = mean -
 * pixel centre (the exponent's magnitude is at most M, so M enters twice). */
static double alpha_bound(const double *cn, double dx, double dy) {
    const double M = 0.5 * fabs(cn[0]) * dx * dx + fabs(cn[1] * dx * dy) + 0.5 * fabs(cn[2]) * dy * dy;
    const double grad = fabs(cn[0] * dx + cn[1] * dy) + fabs(cn[2] * dy + cn[1] * dx);
    return FP32_K * U32 * (2.0 * M + grad * (fabs(dx) + fabs(dy) + 32.0) + 4.0);
}

/* Margins of one pixel's decisions, each the smallest (relative distance to
 * the threshold) / (its error bound) over the decisions taken; inf when a
 * decision never arises. */
typedef struct {
    double a, t, d, c;      /* alpha, stop, dominant, clamp */
    double errT;            /* relative error bound of T so far */
    double eb, es;          /* error bounds of the best and the second weight */
} omargin;

static void margin_init(omargin *m) {
    m->a = m->t = m->d = m->c = INFINITY;
    m->errT = 0.0; m->eb = m->es = 0.0;
}
static void margin_note(double *mg, double dist, double bound) {
    const double r = dist / (bound + FLAG_FLOOR);
    if (r < *mg) *mg = r;
}
static int margin_flag(const omargin *m) { return m->a <= 1.0 || m->t <= 1.0 || m->d <= 1.0 || m->c <= 1.0; }

typedef struct {
    double color[3], T;
    int ncontrib;
    int64_t dom, last;
    int flag;
    int64_t pairs;    /* Gaussians whose box holds the pixel, up to the stop point */
    double wbest, wsecond;
} opix;

/* Alpha of Gaussian (mean, conic, o) at continuous point (px, py). */
static double alpha_at(const double *mean, const double *conic, double o, double px, double py, double *G_out) {
    double dx = mean[0] - px, dy = mean[1] - py;
    double power = -0.5 * (conic[0] * dx * dx + conic[2] * dy * dy) - conic[1] * dx * dy;
    double G = exp(power);
    if (G_out) *G_out = G;
    double a = o * G;
    return a < ALPHA_MAX ? a : ALPHA_MAX;
}

static void render_pixel(int x, int y, int64_t m, const int64_t *order, const double *mean2d, const double *conic,
                         const double *rgb, const double *opacity, const int32_t *box, const double bg[3], opix *out) {
    double px = x + 0.5, py = y + 0.5;
    double T = 1.0, C[3] = {0, 0, 0}, wbest = -1.0, wsecond = -1.0;
    int64_t dom = -1, last = -1;
    int nc = 0;
    int64_t pairs = 0;
    omargin mg;
    margin_init(&mg);
    for (int64_t k = 0; k < m; k++) {
        int64_t i = order[k];
        const int32_t *b = box + i * 4;
        if (x < b[0] || x > b[2] || y < b[1] || y > b[3]) continue;
        pairs++;
        double araw_G;
        double a = alpha_at(mean2d + i * 2, conic + i * 3, opacity[i], px, py, &araw_G);
        double araw = opacity[i] * araw_G;
        const double dx = mean2d[i * 2] - px, dy = mean2d[i * 2 + 1] - py;
        const double ra = alpha_bound(conic + i * 3, dx, dy);
        margin_note(&mg.a, fabs(araw - ALPHA_MIN) / ALPHA_MIN, ra);
        if (a < ALPHA_MIN) continue;
        const double ea = araw < ALPHA_MAX ? ra : 1e-8;   /* the clamped alpha: 0.99 in FP32 */
        const double eT = mg.errT + (araw < ALPHA_MAX ? a * ea / (1.0 - a) : CLAMP_ONE_MINUS_REL) + 2.0 * U32;
        double testT = T * (1.0 - a);
        margin_note(&mg.t, fabs(testT - T_STOP) / T_STOP, eT);
        if (testT < T_STOP) break;
        margin_note(&mg.c, fabs(araw - ALPHA_MAX) / ALPHA_MAX, ra);
        double w = a * T;
        const double ew = ea + mg.errT + U32;
        for (int ch = 0; ch < 3; ch++) C[ch] += w * rgb[i * 3 + ch];
        if (w > wbest) { wsecond = wbest; mg.es = mg.eb; wbest = w; mg.eb = ew; dom = i; }
        else if (w > wsecond) { wsecond = w; mg.es = ew; }
        mg.errT = eT;
        T = testT;
        nc++;
        last = i;
    }
    if (dom >= 0 && wsecond >= 0.0) margin_note(&mg.d, (wbest - wsecond) / wbest, mg.eb + mg.es);
    for (int ch = 0; ch < 3; ch++) out->color[ch] = C[ch] + T * bg[ch];
    out->T = T; out->ncontrib = nc; out->dom = dom; out->last = last; out->flag = margin_flag(&mg);
    out->pairs = pairs;
    out->wbest = wbest; out->wsecond = wsecond;
}

/* Unclamped alpha o G (FP64) of Gaussian ids[k] at the centre of pixel
 * pix[k] = {x, y}, for measuring how far an FP32 evaluation strays. */
void orc_alpha_pairs(const double *mean2d, const double *conic, const double *opacity, int64_t np,
                     const int32_t *pix, const int64_t *ids, double *out, double *bound) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < np; k++) {
        int64_t i = ids[k];
        double G;
        const double px = pix[k * 2] + 0.5, py = pix[k * 2 + 1] + 0.5;
        alpha_at(mean2d + i * 2, conic + i * 3, opacity[i], px, py, &G);
        out[k] = opacity[i] * G;
        if (bound) bound[k] = alpha_bound(conic + i * 3, mean2d[i * 2] - px, mean2d[i * 2 + 1] - py);
    }
}

/* Render the listed pixels (npix x {x, y}).  Inputs are the per-Gaussian rows
 * of orc_project.  Outputs: colour [npix][3], final transmittance, number of
 * contributors, dominant id (-1 if none), id of the last contributor,
 * near-threshold flag and the per-pixel pair count. */
void orc_render_pixels(int64_t n, const int32_t *valid, const double *mean2d, const double *conic,
                       const double *rgb, const double *opacity, const uint32_t *depth_key, const int32_t *box,
                       const double *bg, int64_t npix, const int32_t *pix,
                       double *color, double *Tfinal, int32_t *ncontrib, int64_t *dom, int64_t *last,
                       uint8_t *flag, int64_t *pairs) {
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t m = depth_order(n, valid, depth_key, order);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; p++) {
        opix o;
        render_pixel(pix[p * 2], pix[p * 2 + 1], m, order, mean2d, conic, rgb, opacity, box, bg, &o);
        for (int ch = 0; ch < 3; ch++) color[p * 3 + ch] = o.color[ch];
        Tfinal[p] = o.T; ncontrib[p] = o.ncontrib; dom[p] = o.dom; last[p] = o.last;
        flag[p] = (uint8_t)o.flag; pairs[p] = o.pairs;
    }
    free(order);
}

/* ------------------------------------------------------------------------ */
/* Analytic reverse pass of Eq. (rendering) for the listed pixels.          */
/* For contributor k with alpha a_k and transmittance T_k in front of it,   */
/*   dC/dc_k = a_k T_k,                                                     */
/*   dC/da_k = T_k c_k - (sum_{j>k} a_j T_j c_j + T_final bg) / (1 - a_k),  */
/* then through a = min(0.99, o G), G = exp(power).  The per-Gaussian 2D    */
/* gradients (mean, conic, opacity, colour) are summed over the pixels.     */
/* ------------------------------------------------------------------------ */
void orc_render_backward_pixels(int64_t n, const int32_t *valid, const double *mean2d, const double *conic,
                                const double *rgb, const double *opacity, const uint32_t *depth_key,
                                const int32_t *box, const double *bg, int64_t npix, const int32_t *pix,
                                const double *dL_dcolor, double *g_mean, double *g_conic, double *g_opac,
                                double *g_rgb) {
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t m = depth_order(n, valid, depth_key, order);
    memset(g_mean, 0, sizeof(double) * 2 * n);
    memset(g_conic, 0, sizeof(double) * 3 * n);
    memset(g_opac, 0, sizeof(double) * n);
    memset(g_rgb, 0, sizeof(double) * 3 * n);
    for (int64_t p = 0; p < npix; p++) {
        int x = pix[p * 2], y = pix[p * 2 + 1];
        double px = x + 0.5, py = y + 0.5;
        const double *gC = dL_dcolor + p * 3;
        /* forward: collect the contributors */
        int cap = 64, nc = 0;
        int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * cap);
        double *al = (double *)malloc(sizeof(double) * cap), *Ts = (double *)malloc(sizeof(double) * cap);
        double *Gs = (double *)malloc(sizeof(double) * cap);
        double T = 1.0;
        for (int64_t k = 0; k < m; k++) {
            int64_t i = order[k];
            const int32_t *b = box + i * 4;
            if (x < b[0] || x > b[2] || y < b[1] || y > b[3]) continue;
            double G;
            double a = alpha_at(mean2d + i * 2, conic + i * 3, opacity[i], px, py, &G);
            if (a < ALPHA_MIN) continue;
            double testT = T * (1.0 - a);
            if (testT < T_STOP) break;
            if (nc == cap) {
                cap *= 2;
                ids = (int64_t *)realloc(ids, sizeof(int64_t) * cap);
                al = (double *)realloc(al, sizeof(double) * cap);
                Ts = (double *)realloc(Ts, sizeof(double) * cap);
                Gs = (double *)realloc(Gs, sizeof(double) * cap);
            }
            ids[nc] = i; al[nc] = a; Ts[nc] = T; Gs[nc] = G; nc++;
            T = testT;
        }
        double Tfin = T;
        /* suffix sums S_k = sum_{j>k} a_j T_j c_j + T_final bg */
        double S[3];
        for (int ch = 0; ch < 3; ch++) S[ch] = Tfin * bg[ch];
        for (int k = nc - 1; k >= 0; k--) {
            int64_t i = ids[k];
            double a = al[k], Tk = Ts[k];
            double dLda = 0.0;
            for (int ch = 0; ch < 3; ch++) {
                g_rgb[i * 3 + ch] += a * Tk * gC[ch];
                dLda += gC[ch] * (Tk * rgb[i * 3 + ch] - S[ch] / (1.0 - a));
            }
            for (int ch = 0; ch < 3; ch++) S[ch] += a * Tk * rgb[i * 3 + ch];
            double o = opacity[i], G = Gs[k];
            if (o * G < ALPHA_MAX) {   /* unclamped branch of min(0.99, o G) */
                g_opac[i] += dLda * G;
                double dLdpow = dLda * o * G;
                double dx = mean2d[i * 2] - px, dy = mean2d[i * 2 + 1] - py;
                const double *cn = conic + i * 3;
                g_mean[i * 2 + 0] += dLdpow * (-(cn[0] * dx + cn[1] * dy));
                g_mean[i * 2 + 1] += dLdpow * (-(cn[2] * dy + cn[1] * dx));
                g_conic[i * 3 + 0] += dLdpow * (-0.5 * dx * dx);
                g_conic[i * 3 + 1] += dLdpow * (-dx * dy);
                g_conic[i * 3 + 2] += dLdpow * (-0.5 * dy * dy);
            }
        }
        free(ids); free(al); free(Ts); free(Gs);
    }
    free(order);
}

/* ------------------------------------------------------------------------ */
/* Chain rule from the 2D quantities back to the stored parameters.         */
/* Gradients are written SoA, in the parameter layout.                      */
/* ------------------------------------------------------------------------ */
void orc_project_backward(int64_t n, int deg, const float *means, const float *log_scales, const float *quats,
                          const float *opac, const float *sh, const double *cam_packed,
                          const double *g_mean, const double *g_conic, const double *g_opac, const double *g_rgb,
                          double *d_means, double *d_log_scales, double *d_quats, double *d_opac, double *d_sh) {
    ocam c;
    cam_unpack(cam_packed, &c);
    int nk = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        for (int k = 0; k < 3; k++) { d_means[k * n + i] = 0.0; d_log_scales[k * n + i] = 0.0; }
        for (int k = 0; k < 4; k++) d_quats[k * n + i] = 0.0;
        d_opac[i] = 0.0;
        for (int k = 0; k < nk * 3; k++) d_sh[(int64_t)k * n + i] = 0.0;
        oproj p;
        if (!project_one(n, deg, i, means, log_scales, quats, opac, sh, &c, &p)) continue;
        ogauss g;
        load_gauss(n, i, means, log_scales, quats, opac, &g);
        double dmu[3] = {0, 0, 0};
        /* opacity: o = sigmoid(logit) */
        d_opac[i] = g_opac[i] * g.o * (1.0 - g.o);
        /* colour: rgb = max(0, sum_k Y_k(d) sh_k + 1/2), d = v/|v| */
        double oc[3];
        cam_centre(&c, oc);
        double v[3] = {g.mu[0] - oc[0], g.mu[1] - oc[1], g.mu[2] - oc[2]};
        double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        double d[3] = {v[0] / vn, v[1] / vn, v[2] / vn};
        double Y[16], dY[16][3];
        sh_basis(d[0], d[1], d[2], Y);
        sh_basis_grad(d[0], d[1], d[2], dY);
        double gd[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ch++) {
            if (p.clamped[ch]) continue;
            double gc = g_rgb[i * 3 + ch];
            for (int k = 0; k < nk; k++) {
                d_sh[((int64_t)k * 3 + ch) * n + i] = Y[k] * gc;
                double shv = (double)sh[((int64_t)k * 3 + ch) * n + i];
                for (int a = 0; a < 3; a++) gd[a] += dY[k][a] * shv * gc;
            }
        }
        double ddot = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
        for (int a = 0; a < 3; a++) dmu[a] += (gd[a] - d[a] * ddot) / vn;
        /* mean2d = (fx tx/tz + cx, fy ty/tz + cy) */
        double tx = p.t[0], ty = p.t[1], tz = p.t[2];
        double dt[3] = {0, 0, 0};
        double gm0 = g_mean[i * 2], gm1 = g_mean[i * 2 + 1];
        dt[0] += gm0 * c.fx / tz;
        dt[1] += gm1 * c.fy / tz;
        dt[2] += -gm0 * c.fx * tx / (tz * tz) - gm1 * c.fy * ty / (tz * tz);
        /* conic = inverse(cov): dL/dcov = -K G K, K the conic matrix, G the
         * symmetric gradient matrix (off-diagonal entry appears twice). */
        double K[4] = {p.conic[0], p.conic[1], p.conic[1], p.conic[2]};
        double Gk[4] = {g_conic[i * 3], 0.5 * g_conic[i * 3 + 1], 0.5 * g_conic[i * 3 + 1], g_conic[i * 3 + 2]};
        double KG[4], Gc[4];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) KG[a * 2 + b] = K[a * 2] * Gk[b] + K[a * 2 + 1] * Gk[2 + b];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) Gc[a * 2 + b] = -(KG[a * 2] * K[b] + KG[a * 2 + 1] * K[2 + b]);
        /* cov (before low-pass) = T Sigma T^T, T = J W */
        double limx = 1.3 * ((double)c.W / (2.0 * c.fx));
        double limy = 1.3 * ((double)c.H / (2.0 * c.fy));
        double txtz = tx / tz, tytz = ty / tz;
        int clx = txtz < -limx || txtz > limx, cly = tytz < -limy || tytz > limy;
        double cx_ = fmin(limx, fmax(-limx, txtz)) * tz;
        double cy_ = fmin(limy, fmax(-limy, tytz)) * tz;
        double J[6] = {c.fx / tz, 0.0, -(c.fx * cx_) / (tz * tz), 0.0, c.fy / tz, -(c.fy * cy_) / (tz * tz)};
        double T[6];
        for (int r = 0; r < 2; r++)
            for (int k = 0; k < 3; k++)
                T[r * 3 + k] = J[r * 3 + 0] * c.R[k] + J[r * 3 + 1] * c.R[3 + k] + J[r * 3 + 2] * c.R[6 + k];
        double Sg[9];
        cov3d(g.R, g.s, Sg);
        /* dL/dSigma = T^T Gc T ; dL/dT = 2 Gc T Sigma */
        double dS[9], dT[6];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0.0;
                for (int r = 0; r < 2; r++)
                    for (int q = 0; q < 2; q++) acc += T[r * 3 + a] * Gc[r * 2 + q] * T[q * 3 + b];
                dS[a * 3 + b] = acc;
            }
        for (int r = 0; r < 2; r++)
            for (int k = 0; k < 3; k++) {
                double acc = 0.0;
                for (int q = 0; q < 2; q++)
                    for (int l = 0; l < 3; l++) acc += Gc[r * 2 + q] * T[q * 3 + l] * Sg[l * 3 + k];
                dT[r * 3 + k] = 2.0 * acc;
            }
        /* dL/dJ = dL/dT W^T */
        double dJ[6];
        for (int r = 0; r < 2; r++)
            for (int k = 0; k < 3; k++)
                dJ[r * 3 + k] = dT[r * 3 + 0] * c.R[k * 3 + 0] + dT[r * 3 + 1] * c.R[k * 3 + 1] + dT[r * 3 + 2] * c.R[k * 3 + 2];
        dt[2] += dJ[0] * (-c.fx / (tz * tz)) + dJ[4] * (-c.fy / (tz * tz));
        if (!clx) { dt[0] += dJ[2] * (-c.fx / (tz * tz)); dt[2] += dJ[2] * (2.0 * c.fx * tx / (tz * tz * tz)); }
        else { dt[2] += dJ[2] * (c.fx * (cx_ / tz) / (tz * tz)); }
        if (!cly) { dt[1] += dJ[5] * (-c.fy / (tz * tz)); dt[2] += dJ[5] * (2.0 * c.fy * ty / (tz * tz * tz)); }
        else { dt[2] += dJ[5] * (c.fy * (cy_ / tz) / (tz * tz)); }
        /* t = W mu + t_w */
        for (int a = 0; a < 3; a++) dmu[a] += c.R[0 * 3 + a] * dt[0] + c.R[1 * 3 + a] * dt[1] + c.R[2 * 3 + a] * dt[2];
        for (int a = 0; a < 3; a++) d_means[a * n + i] = dmu[a];
        /* Sigma = R diag(s^2) R^T: dL/ds_k = 2 s_k (R^T dS R)_kk, s = exp(log s) */
        for (int k = 0; k < 3; k++) {
            double acc = 0.0;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) acc += g.R[a * 3 + k] * dS[a * 3 + b] * g.R[b * 3 + k];
            d_log_scales[k * n + i] = 2.0 * g.s[k] * g.s[k] * acc;
        }
        /* dL/dR = 2 dS R diag(s^2) */
        double dR[9];
        for (int a = 0; a < 3; a++)
            for (int k = 0; k < 3; k++) {
                double acc = 0.0;
                for (int b = 0; b < 3; b++) acc += dS[a * 3 + b] * g.R[b * 3 + k];
                dR[a * 3 + k] = 2.0 * acc * g.s[k] * g.s[k];
            }
        double w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
        double dq[4];
        dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
        dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2.0 * x * dR[8]);
        dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2.0 * y * dR[8]);
        dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
        /* through q / |q| */
        double qd = dq[0] * g.qn[0] + dq[1] * g.qn[1] + dq[2] * g.qn[2] + dq[3] * g.qn[3];
        for (int k = 0; k < 4; k++) d_quats[k * n + i] = (dq[k] - g.qn[k] * qd) / g.qnorm;
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.1 error region partitioning, for one view.                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t cand, view, label, area, band;
    int64_t sx, sy, sxx, sxy, syy;   /* exact moments over integer pixel indices */
    double cx, cy;                   /* centroid, continuous pixel frame */
    double cov[3];                   /* pixel covariance + I/12: xx, xy, yy */
    double e1[2];                    /* dominant PCA direction, canonical sign */
    double sigma1, sigma2;
    double rgb[3];                   /* GT colour of the pixel holding the centroid */
} oregion;

/* Size of the record as seen from Python (numpy structured dtype mirrors it). */
int64_t orc_region_size(void) { return (int64_t)sizeof(oregion); }

/* Exact (A*Sab - Sa*Sb) / A^2 in FP64 from integer moments. */
static double central_moment(int64_t A, int64_t sab, int64_t sa, int64_t sb) {
    __int128 num = (__int128)A * sab - (__int128)sa * sb;
    double dnum;
    if (num >= INT64_MIN && num <= INT64_MAX) dnum = (double)(int64_t)num;
    else dnum = (double)num;
    double dA = (double)A;
    return dnum / (dA * dA);
}

/* Region statistics of Sec. 4.1: centroid, pixel covariance (plus the unit
 * pixel's own 1/12 variance [A13]), PCA directions and standard deviations. */
static void region_stats(oregion *r) {
    double A = (double)r->area;
    r->cx = (double)r->sx / A + 0.5;
    r->cy = (double)r->sy / A + 0.5;
    double cxx = central_moment(r->area, r->sxx, r->sx, r->sx) + 1.0 / 12.0;
    double cxy = central_moment(r->area, r->sxy, r->sx, r->sy);
    double cyy = central_moment(r->area, r->syy, r->sy, r->sy) + 1.0 / 12.0;
    r->cov[0] = cxx; r->cov[1] = cxy; r->cov[2] = cyy;
    /* closed-form symmetric 2x2 eigensystem */
    double half_tr = 0.5 * (cxx + cyy);
    double half_dif = 0.5 * (cxx - cyy);
    double disc = sqrt(half_dif * half_dif + cxy * cxy);
    double l1 = half_tr + disc, l2 = half_tr - disc;
    double ex, ey;
    if (disc == 0.0) { ex = 1.0; ey = 0.0; }
    else if (half_dif >= 0.0) { ex = half_dif + disc; ey = cxy; }
    else { ex = cxy; ey = -half_dif + disc; }
    double en = sqrt(ex * ex + ey * ey);
    ex = ex / en; ey = ey / en;
    if (ex < 0.0 || (ex == 0.0 && ey < 0.0)) { ex = -ex; ey = -ey; }
    r->e1[0] = ex; r->e1[1] = ey;
    r->sigma1 = sqrt(l1);
    r->sigma2 = sqrt(l2 > 0.0 ? l2 : 0.0);
}

/* One sampled view v.  Inputs: rendered image and GT ([3][H][W], FP32), the
 * dominant map D_v ([H][W], -1 where no Gaussian contributes) and the split
 * candidate mask over all n Gaussians.  Outputs: attr[] += number of
 * high-error pixels dominated by each candidate (before erosion [A12]); the
 * retained regions in ascending label order.  Optional per-pixel outputs
 * (any may be NULL): E (normalised error), M, M' (eroded), B (band), label.
 * Returns the number of retained regions, or -(count)-1 if cap was exceeded. */
int64_t orc_error_stats(int W, int H, const float *img, const float *gt, const int32_t *dom,
                        int64_t n, const uint8_t *is_cand, int view, double tau, int r_erode, int m_min,
                        int L, int erode_side, int32_t *attr, oregion *regions, int64_t cap,
                        double *E_out, uint8_t *M_out, uint8_t *Mp_out, uint8_t *B_out, int32_t *label_out) {
    (void)n;
    int64_t P = (int64_t)W * H;
    double *e = (double *)malloc(sizeof(double) * P);
    /* Eq. (l1map): per-pixel L1 error, then min-max normalisation over the view */
    double emin = INFINITY, emax = -INFINITY;
    for (int64_t u = 0; u < P; u++) {
        double d0 = fabs((double)img[0 * P + u] - (double)gt[0 * P + u]);
        double d1 = fabs((double)img[1 * P + u] - (double)gt[1 * P + u]);
        double d2 = fabs((double)img[2 * P + u] - (double)gt[2 * P + u]);
        e[u] = (d0 + d1) + d2;
        if (e[u] < emin) emin = e[u];
        if (e[u] > emax) emax = e[u];
    }
    double *E = (double *)malloc(sizeof(double) * P);
    uint8_t *M = (uint8_t *)malloc(P), *Mp = (uint8_t *)malloc(P), *B = (uint8_t *)malloc(P);
    for (int64_t u = 0; u < P; u++) {
        E[u] = (emax == emin) ? 0.0 : (e[u] - emin) / (emax - emin);   /* [A9] */
        M[u] = E[u] > tau;                                                /* metric map */
        int32_t d = dom[u];
        if (M[u] && d >= 0 && is_cand[d]) attr[d] += 1;
    }
    /* erosion with a (2r+1)^2 square; pixels outside the image count as set [A11].
     * Alternative reading (erode_side): a square of side r+1, offsets -r/2 .. r - r/2. */
    int lo = erode_side ? r_erode / 2 : r_erode, hi = erode_side ? r_erode - r_erode / 2 : r_erode;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int keep = M[(int64_t)y * W + x];
            for (int dy = -lo; dy <= hi && keep; dy++)
                for (int dx = -lo; dx <= hi && keep; dx++) {
                    int xx = x + dx, yy = y + dy;
                    if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
                    if (!M[(int64_t)yy * W + xx]) keep = 0;
                }
            Mp[(int64_t)y * W + x] = (uint8_t)keep;
        }
    /* L uniform error bands over (tau, 1] [A10] */
    for (int64_t u = 0; u < P; u++) {
        B[u] = 0;
        if (Mp[u]) {
            double b = floor(((E[u] - tau) * (double)L) / (1.0 - tau));
            if (b > (double)(L - 1)) b = (double)(L - 1);
            B[u] = (uint8_t)b;
        }
    }
    /* Eq. (error-region): 8-connected components of high-error pixels with the
     * same dominant candidate and band, found by breadth-first search from the
     * first unvisited pixel in raster order, so the label is the component's
     * minimum linear index. */
    int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * P);
    for (int64_t u = 0; u < P; u++) lab[u] = -1;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * P);
    int64_t nreg = 0, total = 0;
    for (int64_t s = 0; s < P; s++) {
        int32_t ds = dom[s];
        if (!Mp[s] || ds < 0 || !is_cand[ds] || lab[s] >= 0) continue;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        lab[s] = (int32_t)s;
        oregion r;
        memset(&r, 0, sizeof(r));
        while (head < tail) {
            int64_t u = queue[head++];
            int64_t x = u % W, y = u / W;
            r.area++; r.sx += x; r.sy += y; r.sxx += x * x; r.sxy += x * y; r.syy += y * y;
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    if (!dx && !dy) continue;
                    int64_t xx = x + dx, yy = y + dy;
                    if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
                    int64_t q = yy * W + xx;
                    if (lab[q] >= 0 || !Mp[q] || dom[q] != ds || B[q] != B[s]) continue;
                    lab[q] = (int32_t)s;
                    queue[tail++] = q;
                }
        }
        /* Eq. (min_region_area) */
        if (r.area < m_min) continue;
        total++;
        if (nreg >= cap) continue;
        r.cand = ds; r.view = view; r.label = (int32_t)s; r.band = B[s];
        region_stats(&r);
        int64_t gx = (int64_t)floor(r.cx), gy = (int64_t)floor(r.cy);   /* [A14] */
        for (int ch = 0; ch < 3; ch++) r.rgb[ch] = (double)gt[ch * P + gy * W + gx];
        regions[nreg++] = r;
    }
    if (E_out) memcpy(E_out, E, sizeof(double) * P);
    if (M_out) memcpy(M_out, M, P);
    if (Mp_out) memcpy(Mp_out, Mp, P);
    if (B_out) memcpy(B_out, B, P);
    if (label_out) memcpy(label_out, lab, sizeof(int32_t) * P);
    free(e); free(E); free(M); free(Mp); free(B); free(lab); free(queue);
    return total > cap ? -total - 1 : nreg;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.2 + App. A: one child proposal per retained region.               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int ok, view;
    double mu[3], R[9], s[3], rgb[3];
    double Sinv[9], Sig[9];
} oprop;

static double clipv(double x, double a) {
    double m = fabs(x) < a ? fabs(x) : a;
    return x < 0.0 ? -m : m;
}

/* Covariance R diag(s^2) R^T of a proposal and its inverse R diag(1/s^2) R^T
 * (Eq. (child_cov); the inverse is the metric of Eq. (merge_conditions)). */
static void prop_cov(oprop *p) {
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0, acci = 0.0;
            for (int k = 0; k < 3; k++) {
                acc += p->R[a * 3 + k] * (p->s[k] * p->s[k]) * p->R[b * 3 + k];
                acci += p->R[a * 3 + k] * (1.0 / (p->s[k] * p->s[k])) * p->R[b * 3 + k];
            }
            p->Sig[a * 3 + b] = acc;
            p->Sinv[a * 3 + b] = acci;
        }
}

static void child_from_region(const ogauss *par, const oregion *r, const ocam *c, double eps, oprop *p) {
    memset(p, 0, sizeof(*p));
    double ov[3];
    cam_centre(c, ov);
    /* ray through the centroid: d_cam, then world direction R_c2w d_cam = R^T d_cam */
    double dc[3] = {(r->cx - c->cx) / c->fx, (r->cy - c->cy) / c->fy, 1.0};
    double dw[3];
    for (int j = 0; j < 3; j++) dw[j] = c->R[0 * 3 + j] * dc[0] + c->R[1 * 3 + j] * dc[1] + c->R[2 * 3 + j] * dc[2];
    double dwn = sqrt(dw[0] * dw[0] + dw[1] * dw[1] + dw[2] * dw[2]);
    double d[3] = {dw[0] / dwn, dw[1] / dwn, dw[2] / dwn};
    /* Eq. (tstar): A = Sigma_i^{-1} = R diag(1/s^2) R^T, b = mu_i - o_v */
    double Am[9];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += par->R[a * 3 + k] * (1.0 / (par->s[k] * par->s[k])) * par->R[b * 3 + k];
            Am[a * 3 + b] = acc;
        }
    double bvec[3] = {par->mu[0] - ov[0], par->mu[1] - ov[1], par->mu[2] - ov[2]};
    double Ad[3];
    for (int a = 0; a < 3; a++) Ad[a] = Am[a * 3 + 0] * d[0] + Am[a * 3 + 1] * d[1] + Am[a * 3 + 2] * d[2];
    double num = bvec[0] * Ad[0] + bvec[1] * Ad[1] + bvec[2] * Ad[2];
    double den = d[0] * Ad[0] + d[1] * Ad[1] + d[2] * Ad[2];
    double tstar = num / (den + eps);
    for (int a = 0; a < 3; a++) p->mu[a] = ov[a] + tstar * d[a];
    /* camera-space depth of the child (App. A) */
    double dcn = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
    double tz = tstar / dcn;
    if (!(tz > NEAR_PLANE)) return;   /* [A16] a child behind the near plane is dropped */
    double smax = par->s[0];
    if (par->s[1] > smax) smax = par->s[1];
    if (par->s[2] > smax) smax = par->s[2];
    double e1x = r->e1[0], e1y = r->e1[1];
    double e2x = -e1y, e2y = e1x;
    double w1x = clipv(e1x * r->sigma1 * tz / c->fx, smax * fabs(e1x));
    double w1y = clipv(e1y * r->sigma1 * tz / c->fy, smax * fabs(e1y));
    double w2x = clipv(e2x * r->sigma2 * tz / c->fx, smax * fabs(e2x));
    double w2y = clipv(e2y * r->sigma2 * tz / c->fy, smax * fabs(e2y));
    /* Eq. (axes_world): u_v, w_v = camera right and down = rows 0 and 1 of R */
    double a1[3], a2[3];
    for (int k = 0; k < 3; k++) {
        a1[k] = w1x * c->R[0 * 3 + k] + w1y * c->R[1 * 3 + k];
        a2[k] = w2x * c->R[0 * 3 + k] + w2y * c->R[1 * 3 + k];
    }
    double n1 = sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
    double n2 = sqrt(a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]);
    if (!(n1 > 0.0) || !(n2 > 0.0)) return;
    /* Eq. (child_scales) and Eq. (gram_schmidt) */
    p->s[0] = n1; p->s[1] = n2; p->s[2] = n2;
    double u1[3] = {a1[0] / n1, a1[1] / n1, a1[2] / n1};
    double pr = a2[0] * u1[0] + a2[1] * u1[1] + a2[2] * u1[2];
    double q2[3] = {a2[0] - pr * u1[0], a2[1] - pr * u1[1], a2[2] - pr * u1[2]};
    double nq = sqrt(q2[0] * q2[0] + q2[1] * q2[1] + q2[2] * q2[2]);
    if (!(nq > 0.0)) return;
    double u2[3] = {q2[0] / nq, q2[1] / nq, q2[2] / nq};
    /* Eq. (child_cov): R = [u1 | u2 | z_v], z_v = camera forward = row 2 of R */
    for (int k = 0; k < 3; k++) {
        p->R[k * 3 + 0] = u1[k];
        p->R[k * 3 + 1] = u2[k];
        p->R[k * 3 + 2] = c->R[2 * 3 + k];
    }
    for (int ch = 0; ch < 3; ch++) p->rgb[ch] = r->rgb[ch];
    prop_cov(p);
    p->ok = 1;
}

/* Mahalanobis length sqrt(delta^T Sinv delta). */
static double maha(const double *Sinv, const double *dl) {
    double acc = 0.0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) acc += dl[a] * Sinv[a * 3 + b] * dl[b];
    return sqrt(acc);
}

/* Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix: V columns are
 * eigenvectors, lam the eigenvalues; sorted by descending eigenvalue with the
 * last column flipped so that det V = +1 [A21]. */
static void jacobi3(const double Ain[9], double V[9], double lam[3]) {
    double A[9];
    memcpy(A, Ain, sizeof(A));
    for (int k = 0; k < 9; k++) V[k] = (k % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 32; sweep++) {
        double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        double dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-30 * dia) break;   /* off-diagonal below 1e-15 relative */
        for (int p = 0; p < 2; p++)
            for (int q = p + 1; q < 3; q++) {
                double apq = A[p * 3 + q];
                if (apq == 0.0) continue;
                double app = A[p * 3 + p], aqq = A[q * 3 + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                /* A <- G^T A G with the rotation G in the (p, q) plane */
                for (int k = 0; k < 3; k++) {
                    double akp = A[k * 3 + p], akq = A[k * 3 + q];
                    A[k * 3 + p] = cs * akp - sn * akq;
                    A[k * 3 + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; k++) {
                    double apk = A[p * 3 + k], aqk = A[q * 3 + k];
                    A[p * 3 + k] = cs * apk - sn * aqk;
                    A[q * 3 + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < 3; k++) {
                    double vkp = V[k * 3 + p], vkq = V[k * 3 + q];
                    V[k * 3 + p] = cs * vkp - sn * vkq;
                    V[k * 3 + q] = sn * vkp + cs * vkq;
                }
            }
    }
    for (int k = 0; k < 3; k++) lam[k] = A[k * 4];
    /* sort descending (stable selection on the diagonal) */
    for (int a = 0; a < 2; a++) {
        int best = a;
        for (int b = a + 1; b < 3; b++)
            if (lam[b] > lam[best]) best = b;
        if (best != a) {
            double tl = lam[a]; lam[a] = lam[best]; lam[best] = tl;
            for (int k = 0; k < 3; k++) {
                double tv = V[k * 3 + a]; V[k * 3 + a] = V[k * 3 + best]; V[k * 3 + best] = tv;
            }
        }
    }
    double det = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) + V[2] * (V[3] * V[7] - V[4] * V[6]);
    if (det < 0.0)
        for (int k = 0; k < 3; k++) V[k * 3 + 2] = -V[k * 3 + 2];
}

void orc_jacobi3(const double *A, double *V, double *lam) { jacobi3(A, V, lam); }

/* Rotation matrix -> unit quaternion (w, x, y, z) with w >= 0, by the largest
 * of the four squared components (Shepperd's method). */
static void rot_to_quat(const double R[9], double q[4]) {
    double tr = R[0] + R[4] + R[8];
    double w, x, y, z;
    if (tr > 0.0) {
        double s = sqrt(tr + 1.0) * 2.0;
        w = 0.25 * s; x = (R[7] - R[5]) / s; y = (R[2] - R[6]) / s; z = (R[3] - R[1]) / s;
    } else if (R[0] > R[4] && R[0] > R[8]) {
        double s = sqrt(1.0 + R[0] - R[4] - R[8]) * 2.0;
        w = (R[7] - R[5]) / s; x = 0.25 * s; y = (R[1] + R[3]) / s; z = (R[2] + R[6]) / s;
    } else if (R[4] > R[8]) {
        double s = sqrt(1.0 + R[4] - R[0] - R[8]) * 2.0;
        w = (R[2] - R[6]) / s; x = (R[1] + R[3]) / s; y = 0.25 * s; z = (R[5] + R[7]) / s;
    } else {
        double s = sqrt(1.0 + R[8] - R[0] - R[4]) * 2.0;
        w = (R[3] - R[1]) / s; x = (R[2] + R[6]) / s; y = (R[5] + R[7]) / s; z = 0.25 * s;
    }
    double nn = sqrt(w * w + x * x + y * y + z * z);
    if (w < 0.0) nn = -nn;
    q[0] = w / nn; q[1] = x / nn; q[2] = y / nn; q[3] = z / nn;
}

/* Split hyper-parameters (Sec. 5 "Implementation"). */
typedef struct {
    double gamma_d, gamma_c, eps, eta;
    int n_max;
    int variant;      /* 0 AdpSplit, 1 fixed N random, 2 adaptive N random, 3 child init without merging (Table 2) */
    int flags;        /* 2 merge across views only [A18 alt], 4 extent = max scale [A22 alt], 8 shared opacity [A23 B] */
    int fixed_n, noise_n;
} osplit;

typedef struct { double mu[3], R[9], s[3], rgb[3], extent; int64_t rep; } ogroup;

static int group_cmp(const void *a, const void *b) {
    const ogroup *x = (const ogroup *)a, *y = (const ogroup *)b;
    if (x->extent != y->extent) return x->extent > y->extent ? -1 : 1;   /* descending extent [A22] */
    return x->rep < y->rep ? -1 : (x->rep > y->rep);                      /* ties: earlier member */
}

typedef struct { int64_t key; int64_t idx; } okey;
static int okey_cmp(const void *a, const void *b) {
    const okey *x = (const okey *)a, *y = (const okey *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

static int64_t uf_find(int64_t *par, int64_t a) {
    while (par[a] != a) a = par[a];
    return a;
}

/* Eq. (merge_cov): the merged child of one group of proposals, given in
 * member order.  Mean and colour are the member averages; the axes E are the
 * eigenvectors of the mean covariance (descending eigenvalues, det +1 [A21]);
 * the scale along axis e_r is the largest member reach along it, the offset
 * |e_r^T (mu_m - mean)| plus the member's 1-sigma extent sqrt(e_r^T Sigma_m
 * e_r) [A20], so lambda_r is that reach squared.  A lone proposal is its own
 * merge result. */
static void merge_members(const oprop *const *mem, int64_t M, ogroup *gr) {
    memset(gr, 0, sizeof(*gr));
    if (M == 1) {
        memcpy(gr->mu, mem[0]->mu, sizeof(gr->mu));
        memcpy(gr->rgb, mem[0]->rgb, sizeof(gr->rgb));
        memcpy(gr->R, mem[0]->R, sizeof(gr->R));
        memcpy(gr->s, mem[0]->s, sizeof(gr->s));
        return;
    }
    double Sbar[9] = {0};
    for (int64_t m = 0; m < M; m++) {
        for (int k = 0; k < 3; k++) { gr->mu[k] += mem[m]->mu[k]; gr->rgb[k] += mem[m]->rgb[k]; }
        for (int k = 0; k < 9; k++) Sbar[k] += mem[m]->Sig[k];
    }
    for (int k = 0; k < 3; k++) { gr->mu[k] = gr->mu[k] / (double)M; gr->rgb[k] = gr->rgb[k] / (double)M; }
    for (int k = 0; k < 9; k++) Sbar[k] = Sbar[k] / (double)M;
    double E[9], lam[3];
    jacobi3(Sbar, E, lam);
    for (int r = 0; r < 3; r++) {
        double er[3] = {E[0 * 3 + r], E[1 * 3 + r], E[2 * 3 + r]};
        double best = 0.0;
        for (int64_t m = 0; m < M; m++) {
            const oprop *p = mem[m];
            double off = fabs(er[0] * (p->mu[0] - gr->mu[0]) + er[1] * (p->mu[1] - gr->mu[1]) +
                              er[2] * (p->mu[2] - gr->mu[2]));
            double Se[3];
            for (int k = 0; k < 3; k++)
                Se[k] = p->Sig[k * 3 + 0] * er[0] + p->Sig[k * 3 + 1] * er[1] + p->Sig[k * 3 + 2] * er[2];
            double sig = sqrt(er[0] * Se[0] + er[1] * Se[1] + er[2] * Se[2]);   /* [A20] */
            double reach = off + sig;
            if (reach > best) best = reach;
        }
        gr->s[r] = best;   /* sqrt(lambda_r) */
    }
    memcpy(gr->R, E, sizeof(gr->R));
}

/* Eq. (merge_cov) for M proposals given directly (mu [M][3], R [M][9]
 * row-major, s [M][3], rgb [M][3]), exported for the closed-form pins; the
 * split calls the same merge_members. */
void orc_merge_group(int64_t M, const double *mu, const double *R, const double *s, const double *rgb,
                     double *mu_out, double *rgb_out, double *R_out, double *s_out) {
    oprop *props = (oprop *)calloc((size_t)(M > 0 ? M : 1), sizeof(oprop));
    const oprop **mem = (const oprop **)malloc(sizeof(oprop *) * (size_t)(M > 0 ? M : 1));
    for (int64_t m = 0; m < M; m++) {
        memcpy(props[m].mu, mu + 3 * m, sizeof(props[m].mu));
        memcpy(props[m].R, R + 9 * m, sizeof(props[m].R));
        memcpy(props[m].s, s + 3 * m, sizeof(props[m].s));
        memcpy(props[m].rgb, rgb + 3 * m, sizeof(props[m].rgb));
        prop_cov(&props[m]);
        props[m].ok = 1;
        mem[m] = &props[m];
    }
    ogroup gr;
    merge_members(mem, M, &gr);
    memcpy(mu_out, gr.mu, sizeof(gr.mu));
    memcpy(rgb_out, gr.rgb, sizeof(gr.rgb));
    memcpy(R_out, gr.R, sizeof(gr.R));
    memcpy(s_out, gr.s, sizeof(gr.s));
    free(props); free(mem);
}

/* Sec. 4.2-4.3 + implementation details: the adaptive split of every
 * candidate.  Inputs: parameters (SoA, n rows), candidate ids (ascending),
 * retained regions of all views (any order), the views' packed cameras, the
 * pre-erosion attribution counts, parameters, and the vanilla-split standard
 * normals [n_cand][2][3].  Outputs: mode (0 vanilla, 1 reset, 2 adaptive),
 * rows added per candidate, their exclusive offsets, and the new parameter
 * set (survivors in order, then one block per candidate).  Returns the new
 * row count, or -needed-1 if out_cap is too small. */
int64_t orc_adaptive_split(int64_t n, int deg, const float *means, const float *log_scales, const float *quats,
                           const float *opac, const float *sh, const int32_t *cand, int64_t n_cand,
                           const oregion *regions, int64_t n_reg, const double *cams_packed, int n_views,
                           const int32_t *attr, const double *params, const float *noise,
                           uint8_t *mode, int32_t *count, int64_t *offset,
                           float *o_means, float *o_log_scales, float *o_quats, float *o_opac, float *o_sh,
                           int64_t out_cap) {
    osplit sp;
    sp.gamma_d = params[0]; sp.gamma_c = params[1]; sp.eps = params[2]; sp.eta = params[3];
    sp.n_max = (int)params[4];
    sp.variant = (int)params[5]; sp.flags = (int)params[6]; sp.fixed_n = (int)params[7];
    sp.noise_n = (int)params[8] > 0 ? (int)params[8] : 2;
    int nk = (deg + 1) * (deg + 1);
    ocam *cams = (ocam *)malloc(sizeof(ocam) * (n_views > 0 ? n_views : 1));
    for (int v = 0; v < n_views; v++) cam_unpack(cams_packed + 21 * v, &cams[v]);
    /* regions grouped by candidate, then view, then label */
    okey *ord = (okey *)malloc(sizeof(okey) * (size_t)(n_reg > 0 ? n_reg : 1));
    for (int64_t k = 0; k < n_reg; k++) {
        ord[k].key = ((int64_t)regions[k].cand << 40) | ((int64_t)regions[k].view << 28) | regions[k].label;
        ord[k].idx = k;
    }
    qsort(ord, (size_t)n_reg, sizeof(okey), okey_cmp);
    /* per-candidate results, kept until the append */
    ogroup **kept = (ogroup **)calloc((size_t)(n_cand > 0 ? n_cand : 1), sizeof(ogroup *));
    int64_t rpos = 0;
    for (int64_t ci = 0; ci < n_cand; ci++) {
        int32_t id = cand[ci];
        while (rpos < n_reg && regions[ord[rpos].idx].cand < id) rpos++;
        int64_t r0 = rpos;
        while (rpos < n_reg && regions[ord[rpos].idx].cand == id) rpos++;
        int64_t nr = rpos - r0;
        ogauss par;
        load_gauss(n, id, means, log_scales, quats, opac, &par);
        /* child proposals, in (view, label) order */
        oprop *props = (oprop *)malloc(sizeof(oprop) * (size_t)(nr > 0 ? nr : 1));
        int64_t np = 0;
        for (int64_t k = 0; k < nr; k++) {
            const oregion *r = &regions[ord[r0 + k].idx];
            if (sp.variant == 1) break;   /* the fixed-N random split ignores the regions */
            child_from_region(&par, r, &cams[r->view], sp.eps, &props[np]);
            props[np].view = r->view;
            if (props[np].ok) np++;
        }
        /* Eq. (merge_conditions) over every pair of this parent's proposals [A17-A19] */
        int64_t *uf = (int64_t *)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
        for (int64_t a = 0; a < np; a++) uf[a] = a;
        for (int64_t a = 0; a < np && sp.variant == 0; a++)   /* the ablation variants do not merge */
            for (int64_t b = a + 1; b < np; b++) {
                if ((sp.flags & 2) && props[a].view == props[b].view) continue;   /* [A18] alternative */
                double dl[3] = {props[b].mu[0] - props[a].mu[0], props[b].mu[1] - props[a].mu[1],
                                props[b].mu[2] - props[a].mu[2]};
                double dm = maha(props[a].Sinv, dl) + maha(props[b].Sinv, dl);
                double dc = 0.0;
                for (int ch = 0; ch < 3; ch++) {
                    double t = fabs(props[a].rgb[ch] - props[b].rgb[ch]);
                    if (t > dc) dc = t;
                }
                if (dm <= sp.gamma_d && dc <= sp.gamma_c) {
                    int64_t ra = uf_find(uf, a), rb = uf_find(uf, b);
                    if (ra != rb) { if (ra < rb) uf[rb] = ra; else uf[ra] = rb; }
                }
            }
        /* Eq. (merge_cov): one merged child per connected group */
        ogroup *groups = (ogroup *)malloc(sizeof(ogroup) * (size_t)(np > 0 ? np : 1));
        const oprop **mem = (const oprop **)malloc(sizeof(oprop *) * (size_t)(np > 0 ? np : 1));
        int64_t ng = 0;
        for (int64_t a = 0; a < np; a++) {
            if (uf_find(uf, a) != a) continue;   /* a is the group's first member */
            ogroup gr;
            int64_t M = 0;
            for (int64_t m = a; m < np; m++)
                if (uf_find(uf, m) == a) mem[M++] = &props[m];
            merge_members(mem, M, &gr);
            gr.rep = a;
            if (sp.flags & 4) gr.extent = fmax(gr.s[0], fmax(gr.s[1], gr.s[2]));   /* [A22] alternative */
            else gr.extent = gr.s[0] * gr.s[1] * gr.s[2];
            groups[ng++] = gr;
        }
        /* keep the N_max largest by covariance extent */
        qsort(groups, (size_t)ng, sizeof(ogroup), group_cmp);
        if (ng > sp.n_max) ng = sp.n_max;
        /* mode selection (Sec. 5 "Implementation") */
        if (sp.variant == 1) { mode[ci] = 3; count[ci] = sp.fixed_n; }          /* fixed-N random split */
        else if (attr[id] == 0) { mode[ci] = 0; count[ci] = 2; }
        else if (ng == 0) { mode[ci] = 1; count[ci] = 0; }
        else if (sp.variant == 2) { mode[ci] = 3; count[ci] = (int32_t)ng; }    /* adaptive N, random placement */
        else { mode[ci] = 2; count[ci] = (int32_t)ng + 1; }
        if (mode[ci] == 2) {
            kept[ci] = (ogroup *)malloc(sizeof(ogroup) * (size_t)ng);
            memcpy(kept[ci], groups, sizeof(ogroup) * (size_t)ng);
        }
        free(props); free(uf); free(groups); free(mem);
    }
    /* append (Sec. 3, end; Sec. 5 "Implementation") */
    uint8_t *removed = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int64_t ci = 0; ci < n_cand; ci++)
        if (mode[ci] != 1) removed[cand[ci]] = 1;
    int64_t nsurv = 0;
    for (int64_t i = 0; i < n; i++) nsurv += !removed[i];
    int64_t acc = 0;
    for (int64_t ci = 0; ci < n_cand; ci++) { offset[ci] = acc; acc += count[ci]; }
    int64_t nout = nsurv + acc;
    if (nout > out_cap) {
        for (int64_t ci = 0; ci < n_cand; ci++) free(kept[ci]);
        free(kept); free(removed); free(ord); free(cams);
        return -nout - 1;
    }
    int64_t w = 0;
#define COPY_ROW(dst, src)                                                                         \
    do {                                                                                           \
        for (int k = 0; k < 3; k++) o_means[k * out_cap + (dst)] = means[k * n + (src)];           \
        for (int k = 0; k < 3; k++) o_log_scales[k * out_cap + (dst)] = log_scales[k * n + (src)]; \
        for (int k = 0; k < 4; k++) o_quats[k * out_cap + (dst)] = quats[k * n + (src)];           \
        o_opac[(dst)] = opac[(src)];                                                               \
        for (int k = 0; k < nk * 3; k++) o_sh[(int64_t)k * out_cap + (dst)] = sh[(int64_t)k * n + (src)]; \
    } while (0)
    for (int64_t i = 0; i < n; i++)
        if (!removed[i]) { COPY_ROW(w, i); w++; }
    const double C0 = sqrt(1.0 / (4.0 * 3.14159265358979323846));
    for (int64_t ci = 0; ci < n_cand; ci++) {
        int32_t id = cand[ci];
        int64_t base = nsurv + offset[ci];
        ogauss par;
        load_gauss(n, id, means, log_scales, quats, opac, &par);
        if (mode[ci] == 0 || mode[ci] == 3) {
            /* Eq. (vanilla_split_sample), Eq. (vanilla_split_scale) with N = count (2 for the fallback) */
            int N = count[ci];
            for (int c2 = 0; c2 < N; c2++) {
                int64_t dst = base + c2;
                COPY_ROW(dst, id);
                double dl[3];
                for (int k = 0; k < 3; k++) dl[k] = par.s[k] * (double)noise[(ci * sp.noise_n + c2) * 3 + k];
                for (int k = 0; k < 3; k++) {
                    double m = par.mu[k] + (par.R[k * 3 + 0] * dl[0] + par.R[k * 3 + 1] * dl[1] + par.R[k * 3 + 2] * dl[2]);
                    o_means[k * out_cap + dst] = (float)m;
                    o_log_scales[k * out_cap + dst] = (float)((double)log_scales[k * n + id] - log(sp.eta * (double)N));
                }
            }
        } else if (mode[ci] == 2) {
            int ng = count[ci] - 1;
            for (int g2 = 0; g2 < ng; g2++) {
                const ogroup *gr = &kept[ci][g2];
                int64_t dst = base + g2;
                double q[4];
                rot_to_quat(gr->R, q);
                for (int k = 0; k < 3; k++) o_means[k * out_cap + dst] = (float)gr->mu[k];
                for (int k = 0; k < 3; k++) o_log_scales[k * out_cap + dst] = (float)log(gr->s[k]);
                for (int k = 0; k < 4; k++) o_quats[k * out_cap + dst] = (float)q[k];
                o_opac[dst] = opac[id];   /* children inherit the parent opacity */
                for (int ch = 0; ch < 3; ch++) o_sh[(int64_t)ch * out_cap + dst] = (float)((gr->rgb[ch] - 0.5) / C0);
                for (int k = 3; k < nk * 3; k++) o_sh[(int64_t)k * out_cap + dst] = 0.0f;
            }
            /* parent copy, opacity reduced by a factor N_i + 1 [A23] */
            int64_t dst = base + ng;
            COPY_ROW(dst, id);
            double pr = par.o / (double)(ng + 1);
            o_opac[dst] = (float)log(pr / (1.0 - pr));
            if (sp.flags & 8)   /* [A23] second reading: the whole block at o/(N_i+1) */
                for (int g2 = 0; g2 < ng; g2++) o_opac[base + g2] = o_opac[dst];
        }
    }
#undef COPY_ROW
    for (int64_t ci = 0; ci < n_cand; ci++) free(kept[ci]);
    free(kept); free(removed); free(ord); free(cams);
    return nout;
}

/* Child proposal of one region, exported for the closed-form pins. */
int orc_child_proposal(const float *means, const float *log_scales, const float *quats, const float *opac,
                       const oregion *r, const double *cam_packed, double eps, double *mu, double *R, double *s) {
    ocam c;
    cam_unpack(cam_packed, &c);
    ogauss par;
    load_gauss(1, 0, means, log_scales, quats, opac, &par);
    oprop p;
    child_from_region(&par, r, &c, eps, &p);
    memcpy(mu, p.mu, sizeof(p.mu));
    memcpy(R, p.R, sizeof(p.R));
    memcpy(s, p.s, sizeof(p.s));
    return p.ok;
}

/* ------------------------------------------------------------------------ */
/* Eq. (rendering) for whole rows: for every pixel of rows [y0, y1), the      */
/* Gaussians whose box holds the pixel, composited in ascending (depth key,   */
/* id) order with exactly the arithmetic of render_pixel.  The set of         */
/* candidates of a row is gathered once per row (Gaussians whose box spans   */
/* it, kept in depth order), which is the same sequence render_pixel walks.   */
/* When dL_dcolor is given, the reverse pass of each pixel follows, as in     */
/* orc_render_backward_pixels, and is added into the 2D gradients.           */
/* ------------------------------------------------------------------------ */
void orc_render_rows(int64_t n, const int32_t *valid, const double *mean2d, const double *conic, const double *rgb,
                     const double *opacity, const uint32_t *depth_key, const int32_t *box, const double *bg, int W,
                     int y0, int y1, double *color, double *Tfinal, int32_t *ncontrib, int64_t *dom, int64_t *last,
                     uint8_t *flag, int64_t *pairs, const double *dL_dcolor, double *g_mean, double *g_conic,
                     double *g_opac, double *g_rgb, double *margins, double *g_abs, double *t_bound) {
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t m = depth_order(n, valid, depth_key, order);
    if (dL_dcolor) {
        memset(g_mean, 0, sizeof(double) * 2 * n);
        memset(g_conic, 0, sizeof(double) * 3 * n);
        memset(g_opac, 0, sizeof(double) * n);
        memset(g_rgb, 0, sizeof(double) * 3 * n);
        if (g_abs) memset(g_abs, 0, sizeof(double) * 9 * n);
    }
#pragma omp parallel
    {
        int64_t *row = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
        /* per-pixel contributor lists for the reverse pass */
        int64_t *cap = (int64_t *)calloc((size_t)W, sizeof(int64_t));
        int64_t **lid = (int64_t **)calloc((size_t)W, sizeof(int64_t *));
        double **lal = (double **)calloc((size_t)W, sizeof(double *));
        double **lT = (double **)calloc((size_t)W, sizeof(double *));
        double **lG = (double **)calloc((size_t)W, sizeof(double *));
#pragma omp for schedule(dynamic, 1)
        for (int y = y0; y < y1; y++) {
            int64_t nr = 0;
            for (int64_t k = 0; k < m; k++) {
                const int32_t *b = box + order[k] * 4;
                if (y >= b[1] && y <= b[3]) row[nr++] = order[k];
            }
            for (int x = 0; x < W; x++) {
                const int64_t p = (int64_t)(y - y0) * W + x;
                double px = x + 0.5, py = y + 0.5;
                double T = 1.0, C[3] = {0, 0, 0}, wbest = -1.0, wsecond = -1.0;
                int64_t dm = -1, ls = -1, pr = 0;
                int nc = 0;
                omargin mg;   /* decision margins in units of their FP32 error bounds */
                margin_init(&mg);
                for (int64_t k = 0; k < nr; k++) {
                    int64_t i = row[k];
                    const int32_t *b = box + i * 4;
                    if (x < b[0] || x > b[2]) continue;
                    pr++;
                    double G;
                    double a = alpha_at(mean2d + i * 2, conic + i * 3, opacity[i], px, py, &G);
                    double araw = opacity[i] * G;
                    const double ra = alpha_bound(conic + i * 3, mean2d[i * 2] - px, mean2d[i * 2 + 1] - py);
                    margin_note(&mg.a, fabs(araw - ALPHA_MIN) / ALPHA_MIN, ra);
                    if (a < ALPHA_MIN) continue;
                    const double ea = araw < ALPHA_MAX ? ra : 1e-8;   /* the clamped alpha: 0.99 in FP32 */
                    const double eT = mg.errT + (araw < ALPHA_MAX ? a * ea / (1.0 - a) : CLAMP_ONE_MINUS_REL) +
                                      2.0 * U32;
                    double testT = T * (1.0 - a);
                    margin_note(&mg.t, fabs(testT - T_STOP) / T_STOP, eT);
                    if (testT < T_STOP) break;
                    margin_note(&mg.c, fabs(araw - ALPHA_MAX) / ALPHA_MAX, ra);
                    double w = a * T;
                    const double ew = ea + mg.errT + U32;
                    for (int ch = 0; ch < 3; ch++) C[ch] += w * rgb[i * 3 + ch];
                    if (w > wbest) { wsecond = wbest; mg.es = mg.eb; wbest = w; mg.eb = ew; dm = i; }
                    else if (w > wsecond) { wsecond = w; mg.es = ew; }
                    mg.errT = eT;
                    if (dL_dcolor) {
                        if (nc == cap[x]) {
                            cap[x] = cap[x] ? 2 * cap[x] : 64;
                            lid[x] = (int64_t *)realloc(lid[x], sizeof(int64_t) * cap[x]);
                            lal[x] = (double *)realloc(lal[x], sizeof(double) * cap[x]);
                            lT[x] = (double *)realloc(lT[x], sizeof(double) * cap[x]);
                            lG[x] = (double *)realloc(lG[x], sizeof(double) * cap[x]);
                        }
                        lid[x][nc] = i; lal[x][nc] = a; lT[x][nc] = T; lG[x][nc] = G;
                    }
                    T = testT;
                    nc++;
                    ls = i;
                }
                if (dm >= 0 && wsecond >= 0.0) margin_note(&mg.d, (wbest - wsecond) / wbest, mg.eb + mg.es);
                for (int ch = 0; ch < 3; ch++) color[p * 3 + ch] = C[ch] + T * bg[ch];
                Tfinal[p] = T; ncontrib[p] = nc; dom[p] = dm; last[p] = ls; flag[p] = (uint8_t)margin_flag(&mg);
                pairs[p] = pr;
                if (margins) {
                    margins[p * 4 + 0] = mg.a;
                    margins[p * 4 + 1] = mg.t;
                    margins[p * 4 + 2] = mg.d;
                    margins[p * 4 + 3] = mg.c;
                }
                if (t_bound) t_bound[p] = mg.errT;
                if (!dL_dcolor) continue;
                const double *gC = dL_dcolor + p * 3;
                double S[3];
                for (int ch = 0; ch < 3; ch++) S[ch] = T * bg[ch];
                for (int k = nc - 1; k >= 0; k--) {
                    int64_t i = lid[x][k];
                    double a = lal[x][k], Tk = lT[x][k], G = lG[x][k];
                    double dLda = 0.0, mag = 0.0;
                    for (int ch = 0; ch < 3; ch++) {
#pragma omp atomic
                        g_rgb[i * 3 + ch] += a * Tk * gC[ch];
                        dLda += gC[ch] * (Tk * rgb[i * 3 + ch] - S[ch] / (1.0 - a));
                        /* every factor but gC is non-negative: the sum of the
                           magnitudes of dLda's terms */
                        mag += fabs(gC[ch]) * (Tk * rgb[i * 3 + ch] + S[ch] / (1.0 - a));
                    }
                    if (g_abs)
                        for (int ch = 0; ch < 3; ch++) {
#pragma omp atomic
                            g_abs[i * 9 + 6 + ch] += a * Tk * fabs(gC[ch]);
                        }
                    for (int ch = 0; ch < 3; ch++) S[ch] += a * Tk * rgb[i * 3 + ch];
                    double o = opacity[i];
                    if (o * G < ALPHA_MAX) {
                        double dLdpow = dLda * o * G;
                        double dx = mean2d[i * 2] - px, dy = mean2d[i * 2 + 1] - py;
                        const double *cn = conic + i * 3;
                        if (g_abs) {
                            /* magnitudes of the products summed into each 2D gradient */
                            double mp = mag * o * G;
                            double t9[6] = {mp * (fabs(cn[0] * dx) + fabs(cn[1] * dy)),
                                            mp * (fabs(cn[2] * dy) + fabs(cn[1] * dx)),
                                            mp * 0.5 * dx * dx, mp * fabs(dx * dy), mp * 0.5 * dy * dy, mag * G};
                            for (int q = 0; q < 6; q++) {
#pragma omp atomic
                                g_abs[i * 9 + q] += t9[q];
                            }
                        }
#pragma omp atomic
                        g_opac[i] += dLda * G;
#pragma omp atomic
                        g_mean[i * 2 + 0] += dLdpow * (-(cn[0] * dx + cn[1] * dy));
#pragma omp atomic
                        g_mean[i * 2 + 1] += dLdpow * (-(cn[2] * dy + cn[1] * dx));
#pragma omp atomic
                        g_conic[i * 3 + 0] += dLdpow * (-0.5 * dx * dx);
#pragma omp atomic
                        g_conic[i * 3 + 1] += dLdpow * (-dx * dy);
#pragma omp atomic
                        g_conic[i * 3 + 2] += dLdpow * (-0.5 * dy * dy);
                    }
                }
            }
        }
        for (int x = 0; x < W; x++) { free(lid[x]); free(lal[x]); free(lT[x]); free(lG[x]); }
        free(lid); free(lal); free(lT); free(lG); free(cap); free(row);
    }
    free(order);
}
