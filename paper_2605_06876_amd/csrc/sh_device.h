// Real spherical harmonics up to degree 3 (Condon-Shortley phase carried by the
// complex harmonics; the real basis is sqrt(2) Re / sqrt(2) Im of Y_l^|m|), in
// FP64, and the partial derivatives of each basis polynomial with respect to
// the (unnormalised-treated) direction components.  Used for the view-dependent
// colour of Sec. 3.
#pragma once

// sqrt((2l+1)/(4 pi) * (l-|m|)!/(l+|m|)!) style normalisations, evaluated once.
#define SH_K00 0.28209479177387814
#define SH_K1 0.48860251190291992
#define SH_K2A 1.0925484305920792
#define SH_K20 0.31539156525252005
#define SH_K22 0.54627421529603959
#define SH_K33 0.59004358992664352
#define SH_K32 2.8906114426405538
#define SH_K31 0.45704579946446577
#define SH_K30 0.3731763325901154
#define SH_K32B 1.4453057213202769

__device__ __forceinline__ void sh_eval_basis(double x, double y, double z, int deg, double Y[16]) {
    Y[0] = SH_K00;
    if (deg < 1) return;
    Y[1] = -SH_K1 * y;
    Y[2] = SH_K1 * z;
    Y[3] = -SH_K1 * x;
    if (deg < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SH_K2A * x * y;
    Y[5] = -SH_K2A * y * z;
    Y[6] = SH_K20 * (2.0 * zz - xx - yy);
    Y[7] = -SH_K2A * x * z;
    Y[8] = SH_K22 * (xx - yy);
    if (deg < 3) return;
    Y[9] = -SH_K33 * y * (3.0 * xx - yy);
    Y[10] = SH_K32 * x * y * z;
    Y[11] = -SH_K31 * y * (4.0 * zz - xx - yy);
    Y[12] = SH_K30 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -SH_K31 * x * (4.0 * zz - xx - yy);
    Y[14] = SH_K32B * z * (xx - yy);
    Y[15] = -SH_K33 * x * (xx - 3.0 * yy);
}

// dY[k][a] = dY_k / d(x, y, z)[a]
__device__ __forceinline__ void sh_eval_basis_grad(double x, double y, double z, int deg, double dY[16][3]) {
    for (int k = 0; k < 16; k++) dY[k][0] = dY[k][1] = dY[k][2] = 0.0;
    if (deg < 1) return;
    dY[1][1] = -SH_K1;
    dY[2][2] = SH_K1;
    dY[3][0] = -SH_K1;
    if (deg < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    dY[4][0] = SH_K2A * y;          dY[4][1] = SH_K2A * x;
    dY[5][1] = -SH_K2A * z;         dY[5][2] = -SH_K2A * y;
    dY[6][0] = -2.0 * SH_K20 * x;   dY[6][1] = -2.0 * SH_K20 * y;   dY[6][2] = 4.0 * SH_K20 * z;
    dY[7][0] = -SH_K2A * z;         dY[7][2] = -SH_K2A * x;
    dY[8][0] = 2.0 * SH_K22 * x;    dY[8][1] = -2.0 * SH_K22 * y;
    if (deg < 3) return;
    dY[9][0] = -SH_K33 * 6.0 * x * y;
    dY[9][1] = -SH_K33 * (3.0 * xx - 3.0 * yy);
    dY[10][0] = SH_K32 * y * z; dY[10][1] = SH_K32 * x * z; dY[10][2] = SH_K32 * x * y;
    dY[11][0] = SH_K31 * 2.0 * x * y;
    dY[11][1] = -SH_K31 * (4.0 * zz - xx - 3.0 * yy);
    dY[11][2] = -SH_K31 * 8.0 * y * z;
    dY[12][0] = -SH_K30 * 6.0 * x * z;
    dY[12][1] = -SH_K30 * 6.0 * y * z;
    dY[12][2] = SH_K30 * (6.0 * zz - 3.0 * xx - 3.0 * yy);
    dY[13][0] = -SH_K31 * (4.0 * zz - 3.0 * xx - yy);
    dY[13][1] = SH_K31 * 2.0 * x * y;
    dY[13][2] = -SH_K31 * 8.0 * x * z;
    dY[14][0] = SH_K32B * 2.0 * x * z; dY[14][1] = -SH_K32B * 2.0 * y * z; dY[14][2] = SH_K32B * (xx - yy);
    dY[15][0] = -SH_K33 * (3.0 * xx - 3.0 * yy);
    dY[15][1] = SH_K33 * 6.0 * x * y;
}

// g[a] = sum_k w[k] dY_k / d(x, y, z)[a], the gradient of sum_k w_k Y_k
// accumulated term by term (the terms of sh_eval_basis_grad), so no table of
// the 48 partial derivatives is held.
__device__ __forceinline__ void sh_weighted_grad(double x, double y, double z, int deg, const double w[16],
                                                 double g[3]) {
    g[0] = g[1] = g[2] = 0.0;
    if (deg < 1) return;
    g[1] += -SH_K1 * w[1];
    g[2] += SH_K1 * w[2];
    g[0] += -SH_K1 * w[3];
    if (deg < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    g[0] += SH_K2A * y * w[4];        g[1] += SH_K2A * x * w[4];
    g[1] += -SH_K2A * z * w[5];       g[2] += -SH_K2A * y * w[5];
    g[0] += -2.0 * SH_K20 * x * w[6]; g[1] += -2.0 * SH_K20 * y * w[6]; g[2] += 4.0 * SH_K20 * z * w[6];
    g[0] += -SH_K2A * z * w[7];       g[2] += -SH_K2A * x * w[7];
    g[0] += 2.0 * SH_K22 * x * w[8];  g[1] += -2.0 * SH_K22 * y * w[8];
    if (deg < 3) return;
    g[0] += -SH_K33 * 6.0 * x * y * w[9];
    g[1] += -SH_K33 * (3.0 * xx - 3.0 * yy) * w[9];
    g[0] += SH_K32 * y * z * w[10]; g[1] += SH_K32 * x * z * w[10]; g[2] += SH_K32 * x * y * w[10];
    g[0] += SH_K31 * 2.0 * x * y * w[11];
    g[1] += -SH_K31 * (4.0 * zz - xx - 3.0 * yy) * w[11];
    g[2] += -SH_K31 * 8.0 * y * z * w[11];
    g[0] += -SH_K30 * 6.0 * x * z * w[12];
    g[1] += -SH_K30 * 6.0 * y * z * w[12];
    g[2] += SH_K30 * (6.0 * zz - 3.0 * xx - 3.0 * yy) * w[12];
    g[0] += -SH_K31 * (4.0 * zz - 3.0 * xx - yy) * w[13];
    g[1] += SH_K31 * 2.0 * x * y * w[13];
    g[2] += -SH_K31 * 8.0 * x * z * w[13];
    g[0] += SH_K32B * 2.0 * x * z * w[14]; g[1] += -SH_K32B * 2.0 * y * z * w[14]; g[2] += SH_K32B * (xx - yy) * w[14];
    g[0] += -SH_K33 * (3.0 * xx - 3.0 * yy) * w[15];
    g[1] += SH_K33 * 6.0 * x * y * w[15];
}

