// Diffusion synthetic acceleration on the device (eq. (diffusion_correction)).
//
// 1D: the consistent DSA of Appendix B.  With the P1 ansatz delta f = delta rho + 3 v delta J and
//     the moment equations eq. (dsa_rho), eq. (dsa_J), the unknowns (delta rho, delta J) of a
//     cell couple only to the two neighbouring cells through D_C = (D^+ + D^-)/2 and
//     D_J = D^+ - D^-, so the system is block tridiagonal with 4x4 blocks and is solved directly
//     (block Thomas, one thread per instance, FP64).  In the orthonormal P1 basis on a cell of
//     width h, with traces P(+1) = (1, s3), P(-1) = (1, -s3):
//       diag(D_C) = [[0, s3/h], [-s3/h, 0]],      diag(D_J) = [[-2/h, 0], [0, -6/h]],
//       upper D_J(c,c+1) = P(+1) P(-1)^T / sqrt(h_c h_c+1),  D_C upper = D_J upper / 2,
//       lower D_J(c,c-1) = P(-1) P(+1)^T / sqrt(h_c h_c-1),  D_C lower = -D_J lower / 2.
//
// 2D: the symmetric interior-penalty (MIP) diffusion form on the Q1 DG space with
//     D = (sum_j w_j v_x^2) / sigma_t, penalty kappa_e = max(kappa_min, kappa_IP),
//     kappa_IP = 2 (D^- + D^+) / h (interior), 4 D / h (boundary), kappa_min = sum_{v.n>0} w v.n,
//     applied matrix-free and solved by block-Jacobi preconditioned CG in FP64.  The face terms
//     reduce, in the orthonormal basis, to 2x2 blocks acting on the Legendre index normal to the
//     face (identity in the tangential index):
//       own '+' face:  kappa/h [[1, s3],[s3, 3]]  - D s3/h^2 [[0, 1],[1, 2 s3]]
//       own '-' face:  kappa/h [[1,-s3],[-s3, 3]] + D s3/h^2 [[0, 1],[1, -2 s3]]
//       to the '+' neighbour: -kappa/h [[1,-s3],[s3,-3]] - D+ s3/h^2 [[0,1],[0,s3]] + D- s3/h^2 [[0,0],[1,-s3]]
//     and the volume term 12 D/h^2 on the dofs of degree 1 in that direction, plus sigma_a.
//     Per-instance scalars are re-derived by every block from fixed-order partial sums, so no
//     grid-wide synchronization is needed and the result does not depend on block scheduling.
#include <type_traits>
#include <algorithm>

#include "rte_internal.h"

namespace rte {
namespace {

constexpr double kS3 = 1.7320508075688772935;
constexpr double kMipC = 4.0;
constexpr int kCgBlock = 256;
constexpr double kOmegaDG = 0.7;      // damping of the block-Jacobi smoother of the multigrid

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ----------------------------------------------------------------------------------- 1D
__device__ void inv4(const double *A, double *Ai) {
    double M[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) { M[i][j] = A[4 * i + j]; M[i][4 + j] = (i == j) ? 1.0 : 0.0; }
    for (int k = 0; k < 4; ++k) {
        int pv = k;
        for (int i = k + 1; i < 4; ++i)
            if (fabs(M[i][k]) > fabs(M[pv][k])) pv = i;
        if (pv != k)
            for (int j = 0; j < 8; ++j) { double t = M[k][j]; M[k][j] = M[pv][j]; M[pv][j] = t; }
        const double d = 1.0 / M[k][k];
        for (int j = 0; j < 8; ++j) M[k][j] *= d;
        for (int i = 0; i < 4; ++i) {
            if (i == k) continue;
            const double f = M[i][k];
            for (int j = 0; j < 8; ++j) M[i][j] -= f * M[k][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) Ai[4 * i + j] = M[i][4 + j];
}

// 4x4 block of the (delta rho, delta J) system built from 2x2 blocks of D_C and D_J
__device__ void dsa1d_block(double dc[4], double dj[4], double sa, double st, double c1,
                            double c2, double c3, bool diag, double out[16]) {
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            out[4 * i + j] = -c1 * dj[2 * i + j] + ((diag && i == j) ? sa : 0.0);
            out[4 * i + 2 + j] = dc[2 * i + j];
            out[4 * (2 + i) + j] = c2 * dc[2 * i + j];
            out[4 * (2 + i) + 2 + j] = -3.0 * c3 * dj[2 * i + j] + ((diag && i == j) ? st : 0.0);
        }
}

__device__ void dsa1d_blocks_at(int c, int nc, const double *h, double sa, double st, double c1,
                                double c2, double c3, double Lo[16], double Dg[16],
                                double Up[16]) {
    const double s3 = kS3;
    const double hc = h[c];
    double dc[4] = {0.0, s3 / hc, -s3 / hc, 0.0};
    double dj[4] = {-2.0 / hc, 0.0, 0.0, -6.0 / hc};
    dsa1d_block(dc, dj, sa, st, c1, c2, c3, true, Dg);
    if (c + 1 < nc) {   // P(+1) P(-1)^T / sqrt(h_c h_c+1) = [[1,-s3],[s3,-3]] / sq
        const double sq = sqrt(hc * h[c + 1]);
        double uj[4] = {1.0 / sq, -s3 / sq, s3 / sq, -3.0 / sq};
        double uc[4] = {0.5 * uj[0], 0.5 * uj[1], 0.5 * uj[2], 0.5 * uj[3]};
        dsa1d_block(uc, uj, 0.0, 0.0, c1, c2, c3, false, Up);
    } else {
        for (int i = 0; i < 16; ++i) Up[i] = 0.0;
    }
    if (c > 0) {        // P(-1) P(+1)^T / sqrt(h_c h_c-1) = [[1,s3],[-s3,-3]] / sq
        const double sq = sqrt(hc * h[c - 1]);
        double lj[4] = {1.0 / sq, s3 / sq, -s3 / sq, -3.0 / sq};
        double lc[4] = {-0.5 * lj[0], -0.5 * lj[1], -0.5 * lj[2], -0.5 * lj[3]};
        dsa1d_block(lc, lj, 0.0, 0.0, c1, c2, c3, false, Lo);
    } else {
        for (int i = 0; i < 16; ++i) Lo[i] = 0.0;
    }
}

// scratch per instance: [nc][16] (D'^-1 U) and [nc][4] (D'^-1 r')
__global__ void dsa1d_kernel(int nc, int B, const double *h, const double *sigma_t,
                             const double *sigma_s, double c1, double c2, double c3,
                             const double *rho_star, const double *rho_prev, double *delta,
                             const int *kind, int want, double *scratch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    if (kind && kind[b] != want) return;
    double *G = scratch + (size_t)b * nc * 20;     // G[c] = D'_c^-1 U_c (16), g[c] = D'_c^-1 r'_c (4)
    double Lo[16], Dg[16], Up[16], Dp[16], Di[16];
    for (int c = 0; c < nc; ++c) {
        const double st = sigma_t[(size_t)b * nc + c], ss = sigma_s[(size_t)b * nc + c];
        dsa1d_blocks_at(c, nc, h, st - ss, st, c1, c2, c3, Lo, Dg, Up);
        double r[4];
        for (int k = 0; k < 2; ++k) {
            const size_t i = ((size_t)b * nc + c) * 2 + k;
            r[k] = ss * (rho_star[i] - (rho_prev ? rho_prev[i] : 0.0));
            r[2 + k] = 0.0;
        }
        for (int i = 0; i < 16; ++i) Dp[i] = Dg[i];
        if (c > 0) {
            const double *Gm = G + (size_t)(c - 1) * 20;
            for (int i = 0; i < 4; ++i) {
                for (int j = 0; j < 4; ++j) {
                    double s = 0.0;
                    for (int k = 0; k < 4; ++k) s += Lo[4 * i + k] * Gm[4 * k + j];
                    Dp[4 * i + j] -= s;
                }
                double s = 0.0;
                for (int k = 0; k < 4; ++k) s += Lo[4 * i + k] * Gm[16 + k];
                r[i] -= s;
            }
        }
        inv4(Dp, Di);
        double *Gc = G + (size_t)c * 20;
        for (int i = 0; i < 4; ++i) {
            for (int j = 0; j < 4; ++j) {
                double s = 0.0;
                for (int k = 0; k < 4; ++k) s += Di[4 * i + k] * Up[4 * k + j];
                Gc[4 * i + j] = s;
            }
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += Di[4 * i + k] * r[k];
            Gc[16 + i] = s;
        }
    }
    double xn[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = nc - 1; c >= 0; --c) {
        const double *Gc = G + (size_t)c * 20;
        double x[4];
        for (int i = 0; i < 4; ++i) {
            double s = Gc[16 + i];
            for (int k = 0; k < 4; ++k) s -= Gc[4 * i + k] * xn[k];
            x[i] = s;
        }
        for (int i = 0; i < 4; ++i) xn[i] = x[i];
        delta[((size_t)b * nc + c) * 2 + 0] = x[0];
        delta[((size_t)b * nc + c) * 2 + 1] = x[1];
    }
}

// ----------------------------------------------------------------------------------- 2D
struct MipArgs {
    int nx, ny, B, nblk;
    long long ncell;
    double hx, hy, cxx, cyy, kx, ky;
    double ihx, ihy;                  // 1/h
    double th_x, th_y;                // s3/h^2
    double vol_x, vol_y;              // 12/h^2
    const double *sigma_t, *sigma_s;
    // per-cell data of the operator, computed once per solve by mip_prepare_kernel:
    //   cf   [B][5][ncell]  sigma_a, Dx, Dy, kappa of the right face, kappa of the top face
    //   binv [B][10][ncell] inverse of the diagonal 4x4 block (upper triangle, row-major), FP32:
    //        it is the block-Jacobi smoother of the preconditioner; one stored entry serves both
    //        halves, so the rounded smoother stays exactly symmetric
    const double *cf;
    const float *binv;
    // cf rounded to FP32 (mixed precision): read by the preconditioner's operator applications
    const float *cf32;
};
constexpr int kCf = 5;
constexpr int kBinv = 10;

__device__ __forceinline__ double kap_int(double Dm, double Dp, double h, double kmin) {
    return fmax(kmin, 0.5 * kMipC * (Dm + Dp) / h);
}
__device__ __forceinline__ double kap_bnd(double D, double h, double kmin) {
    return fmax(kmin, kMipC * D / h);
}

// 2x2 face blocks (row-major [a][a']) in terms of k = kappa/h and t = D s3/h^2
__device__ __forceinline__ void face_plus(double k, double t, double M[4]) {
    const double s3 = kS3;
    M[0] = k; M[1] = k * s3 - t; M[2] = k * s3 - t; M[3] = 3.0 * k - 2.0 * s3 * t;
}
__device__ __forceinline__ void face_minus(double k, double t, double M[4]) {
    const double s3 = kS3;
    M[0] = k; M[1] = -k * s3 + t; M[2] = -k * s3 + t; M[3] = 3.0 * k - 2.0 * s3 * t;
}
// row = '-' cell, column = '+' cell (tm, tp: t of the '-' and '+' cells)
__device__ __forceinline__ void couple_mp(double k, double tm, double tp, double M[4]) {
    const double s3 = kS3;
    M[0] = -k; M[1] = k * s3 - tp; M[2] = -k * s3 + tm; M[3] = 3.0 * k - s3 * tp - s3 * tm;
}
// row = '+' cell, column = '-' cell: transpose of couple_mp
__device__ __forceinline__ void couple_pm(double k, double tm, double tp, double M[4]) {
    double T[4];
    couple_mp(k, tm, tp, T);
    M[0] = T[0]; M[1] = T[2]; M[2] = T[1]; M[3] = T[3];
}

// y += M (x) applied along x (acts on a for each b): dofs (0,1) and (2,3)
__device__ __forceinline__ void addx(const double M[4], const double x[4], double y[4]) {
    y[0] += M[0] * x[0] + M[1] * x[1];
    y[1] += M[2] * x[0] + M[3] * x[1];
    y[2] += M[0] * x[2] + M[1] * x[3];
    y[3] += M[2] * x[2] + M[3] * x[3];
}
// along y (acts on b for each a): dofs (0,2) and (1,3)
__device__ __forceinline__ void addy(const double M[4], const double x[4], double y[4]) {
    y[0] += M[0] * x[0] + M[1] * x[2];
    y[2] += M[2] * x[0] + M[3] * x[2];
    y[1] += M[0] * x[1] + M[1] * x[3];
    y[3] += M[2] * x[1] + M[3] * x[3];
}
__device__ __forceinline__ void addx_mat(const double M[4], double A[16]) {
    // A[k][l] for k,l in {(0,1)} and {(2,3)}
    A[0 * 4 + 0] += M[0]; A[0 * 4 + 1] += M[1]; A[1 * 4 + 0] += M[2]; A[1 * 4 + 1] += M[3];
    A[2 * 4 + 2] += M[0]; A[2 * 4 + 3] += M[1]; A[3 * 4 + 2] += M[2]; A[3 * 4 + 3] += M[3];
}
__device__ __forceinline__ void addy_mat(const double M[4], double A[16]) {
    A[0 * 4 + 0] += M[0]; A[0 * 4 + 2] += M[1]; A[2 * 4 + 0] += M[2]; A[2 * 4 + 2] += M[3];
    A[1 * 4 + 1] += M[0]; A[1 * 4 + 3] += M[1]; A[3 * 4 + 1] += M[2]; A[3 * 4 + 3] += M[3];
}

struct CellCoef {
    double Dx, Dy, sa;
};
__device__ __forceinline__ CellCoef coef_at(const MipArgs &a, int b, long long cell) {
    const double st = a.sigma_t[(size_t)b * a.ncell + cell];
    const double ss = a.sigma_s[(size_t)b * a.ncell + cell];
    CellCoef c;
    c.Dx = a.cxx / st;
    c.Dy = a.cyy / st;
    c.sa = st - ss;
    return c;
}

// Diagonal 4x4 block of the MIP operator at cell (i, j), from the material data (prepare only).
__device__ void mip_diag(const MipArgs &a, int b, int i, int j, double A[16]) {
    const long long cell = (long long)j * a.nx + i;
    const CellCoef cc = coef_at(a, b, cell);
    for (int k = 0; k < 16; ++k) A[k] = 0.0;
    const double vx = a.vol_x * cc.Dx, vy = a.vol_y * cc.Dy;
    A[0] = cc.sa;
    A[5] = cc.sa + vx;
    A[10] = cc.sa + vy;
    A[15] = cc.sa + vx + vy;
    double M[4];
    const double kl = i > 0 ? kap_int(coef_at(a, b, cell - 1).Dx, cc.Dx, a.hx, a.kx) : kap_bnd(cc.Dx, a.hx, a.kx);
    const double kr = i + 1 < a.nx ? kap_int(cc.Dx, coef_at(a, b, cell + 1).Dx, a.hx, a.kx) : kap_bnd(cc.Dx, a.hx, a.kx);
    const double kb = j > 0 ? kap_int(coef_at(a, b, cell - a.nx).Dy, cc.Dy, a.hy, a.ky) : kap_bnd(cc.Dy, a.hy, a.ky);
    const double kt = j + 1 < a.ny ? kap_int(cc.Dy, coef_at(a, b, cell + a.nx).Dy, a.hy, a.ky) : kap_bnd(cc.Dy, a.hy, a.ky);
    const double tx = a.th_x * cc.Dx, ty = a.th_y * cc.Dy;
    face_minus(kl * a.ihx, tx, M); addx_mat(M, A);
    face_plus(kr * a.ihx, tx, M);  addx_mat(M, A);
    face_minus(kb * a.ihy, ty, M); addy_mat(M, A);
    face_plus(kt * a.ihy, ty, M);  addy_mat(M, A);
}

// solve the SPD 4x4 system A z = r (Cholesky)
__device__ void spd4_solve(const double A[16], const double r[4], double z[4]) {
    double L[16];
    for (int k = 0; k < 16; ++k) L[k] = 0.0;
    for (int j = 0; j < 4; ++j) {
        double s = A[5 * j];
        for (int k = 0; k < j; ++k) s -= L[4 * j + k] * L[4 * j + k];
        const double d = sqrt(s);
        L[5 * j] = d;
        for (int i = j + 1; i < 4; ++i) {
            double t = A[4 * i + j];
            for (int k = 0; k < j; ++k) t -= L[4 * i + k] * L[4 * j + k];
            L[4 * i + j] = t / d;
        }
    }
    double y[4];
    for (int i = 0; i < 4; ++i) {
        double s = r[i];
        for (int k = 0; k < i; ++k) s -= L[4 * i + k] * y[k];
        y[i] = s / L[5 * i];
    }
    for (int i = 3; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 4; ++k) s -= L[4 * k + i] * z[k];
        z[i] = s / L[5 * i];
    }
}

__device__ __forceinline__ void load4(const double *v, long long idx, double x[4]) {
    const double4 t = *reinterpret_cast<const double4 *>(v + idx * 4);
    x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
}
__device__ __forceinline__ void store4(double *v, long long idx, const double x[4]) {
    double4 t;
    t.x = x[0]; t.y = x[1]; t.z = x[2]; t.w = x[3];
    *reinterpret_cast<double4 *>(v + idx * 4) = t;
}

// FP32 storage of the preconditioner's vectors (values widened to FP64 on load)
__device__ __forceinline__ void load4(const float *v, long long idx, double x[4]) {
    const float4 t = *reinterpret_cast<const float4 *>(v + idx * 4);
    x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
}
__device__ __forceinline__ void store4(float *v, long long idx, const double x[4]) {
    float4 t;
    t.x = (float)x[0]; t.y = (float)x[1]; t.z = (float)x[2]; t.w = (float)x[3];
    *reinterpret_cast<float4 *>(v + idx * 4) = t;
}

template <typename TC>
__device__ __forceinline__ const TC *cf_of(const MipArgs &a);
template <>
__device__ __forceinline__ const double *cf_of<double>(const MipArgs &a) { return a.cf; }
template <>
__device__ __forceinline__ const float *cf_of<float>(const MipArgs &a) { return a.cf32; }

template <typename TC = double>
__device__ __forceinline__ double cfv(const MipArgs &a, int b, int k, long long cell) {
    return (double)cf_of<TC>(a)[((size_t)b * kCf + k) * a.ncell + cell];
}

// z = B^-1 r with the stored inverse of the diagonal block (symmetric by construction)
__device__ __forceinline__ void binv_apply(const MipArgs &a, int b, long long cell, const double r[4],
                                           double z[4]) {
    const float *q = a.binv + (size_t)b * kBinv * a.ncell + cell;
    const long long n = a.ncell;
    const double m00 = q[0], m01 = q[n], m02 = q[2 * n], m03 = q[3 * n], m11 = q[4 * n],
                 m12 = q[5 * n], m13 = q[6 * n], m22 = q[7 * n], m23 = q[8 * n], m33 = q[9 * n];
    z[0] = m00 * r[0] + m01 * r[1] + m02 * r[2] + m03 * r[3];
    z[1] = m01 * r[0] + m11 * r[1] + m12 * r[2] + m13 * r[3];
    z[2] = m02 * r[0] + m12 * r[1] + m22 * r[2] + m23 * r[3];
    z[3] = m03 * r[0] + m13 * r[1] + m23 * r[2] + m33 * r[3];
}

// y = A x at cell (i,j) with every load (the five cells' x and the coefficients) issued before
// the arithmetic: a missing neighbour reads the cell itself, and its coupling is applied to zero
// (its coefficients are the cell's own, finite, so the term vanishes).  No load waits behind a
// boundary branch, at the price of registers: used where the register count stays within the
// occupancy the kernel had (the mixed-precision DG residual of the multigrid).
template <typename TC, typename F>
__device__ void mip_apply_hoisted(const MipArgs &a, int b, int i, int j, F xat, double y[4]) {
    const long long cell = (long long)j * a.nx + i;
    const bool hl = i > 0, hr = i + 1 < a.nx, hd = j > 0, hu = j + 1 < a.ny;
    const long long cl = hl ? cell - 1 : cell, cr = hr ? cell + 1 : cell;
    const long long cd = hd ? cell - a.nx : cell, cu = hu ? cell + a.nx : cell;
    const double sa = cfv<TC>(a, b, 0, cell), Dx = cfv<TC>(a, b, 1, cell), Dy = cfv<TC>(a, b, 2, cell);
    const double Dxl = cfv<TC>(a, b, 1, cl), kal = cfv<TC>(a, b, 3, cl);
    const double Dxr = cfv<TC>(a, b, 1, cr), kar = cfv<TC>(a, b, 3, cell);
    const double Dyd = cfv<TC>(a, b, 2, cd), kad = cfv<TC>(a, b, 4, cd);
    const double Dyu = cfv<TC>(a, b, 2, cu), kau = cfv<TC>(a, b, 4, cell);
    double xc[4], xl[4], xr[4], xd[4], xu[4], xn[4], M[4];
    xat(cell, xc);
    xat(cl, xl);
    xat(cr, xr);
    xat(cd, xd);
    xat(cu, xu);
    const double vx = a.vol_x * Dx, vy = a.vol_y * Dy;
    const double tx = a.th_x * Dx, ty = a.th_y * Dy;
    y[0] = sa * xc[0];
    y[1] = (sa + vx) * xc[1];
    y[2] = (sa + vy) * xc[2];
    y[3] = (sa + vx + vy) * xc[3];
    {
        const double k = hl ? kal * a.ihx : fmax(a.kx, kMipC * Dx * a.ihx) * a.ihx;
        face_minus(k, tx, M); addx(M, xc, y);
        for (int q = 0; q < 4; ++q) xn[q] = hl ? xl[q] : 0.0;
        couple_pm(k, a.th_x * Dxl, tx, M); addx(M, xn, y);
    }
    {
        const double k = hr ? kar * a.ihx : fmax(a.kx, kMipC * Dx * a.ihx) * a.ihx;
        face_plus(k, tx, M); addx(M, xc, y);
        for (int q = 0; q < 4; ++q) xn[q] = hr ? xr[q] : 0.0;
        couple_mp(k, tx, a.th_x * Dxr, M); addx(M, xn, y);
    }
    {
        const double k = hd ? kad * a.ihy : fmax(a.ky, kMipC * Dy * a.ihy) * a.ihy;
        face_minus(k, ty, M); addy(M, xc, y);
        for (int q = 0; q < 4; ++q) xn[q] = hd ? xd[q] : 0.0;
        couple_pm(k, a.th_y * Dyd, ty, M); addy(M, xn, y);
    }
    {
        const double k = hu ? kau * a.ihy : fmax(a.ky, kMipC * Dy * a.ihy) * a.ihy;
        face_plus(k, ty, M); addy(M, xc, y);
        for (int q = 0; q < 4; ++q) xn[q] = hu ? xu[q] : 0.0;
        couple_mp(k, ty, a.th_y * Dyu, M); addy(M, xn, y);
    }
}

// y = A x at cell (i,j), with x read through a functor (to form p = z + beta p_old on the fly);
// the operator's coefficients come from the per-cell planes (no divisions here), FP64 or (TC =
// float, inside the mixed-precision preconditioner) their FP32 copy
template <typename TC = double, typename F>
__device__ void mip_apply(const MipArgs &a, int b, int i, int j, F xat, double y[4]) {
    const long long cell = (long long)j * a.nx + i;
    const double sa = cfv<TC>(a, b, 0, cell), Dx = cfv<TC>(a, b, 1, cell), Dy = cfv<TC>(a, b, 2, cell);
    double xc[4], xn[4], M[4];
    xat(cell, xc);
    const double vx = a.vol_x * Dx, vy = a.vol_y * Dy;
    const double tx = a.th_x * Dx, ty = a.th_y * Dy;
    y[0] = sa * xc[0];
    y[1] = (sa + vx) * xc[1];
    y[2] = (sa + vy) * xc[2];
    y[3] = (sa + vx + vy) * xc[3];
    if (i > 0) {
        const double tl = a.th_x * cfv<TC>(a, b, 1, cell - 1);
        const double k = cfv<TC>(a, b, 3, cell - 1) * a.ihx;
        face_minus(k, tx, M); addx(M, xc, y);
        xat(cell - 1, xn);
        couple_pm(k, tl, tx, M); addx(M, xn, y);
    } else {
        face_minus(fmax(a.kx, kMipC * Dx * a.ihx) * a.ihx, tx, M); addx(M, xc, y);
    }
    if (i + 1 < a.nx) {
        const double tr = a.th_x * cfv<TC>(a, b, 1, cell + 1);
        const double k = cfv<TC>(a, b, 3, cell) * a.ihx;
        face_plus(k, tx, M); addx(M, xc, y);
        xat(cell + 1, xn);
        couple_mp(k, tx, tr, M); addx(M, xn, y);
    } else {
        face_plus(fmax(a.kx, kMipC * Dx * a.ihx) * a.ihx, tx, M); addx(M, xc, y);
    }
    if (j > 0) {
        const double tb = a.th_y * cfv<TC>(a, b, 2, cell - a.nx);
        const double k = cfv<TC>(a, b, 4, cell - a.nx) * a.ihy;
        face_minus(k, ty, M); addy(M, xc, y);
        xat(cell - a.nx, xn);
        couple_pm(k, tb, ty, M); addy(M, xn, y);
    } else {
        face_minus(fmax(a.ky, kMipC * Dy * a.ihy) * a.ihy, ty, M); addy(M, xc, y);
    }
    if (j + 1 < a.ny) {
        const double tt = a.th_y * cfv<TC>(a, b, 2, cell + a.nx);
        const double k = cfv<TC>(a, b, 4, cell) * a.ihy;
        face_plus(k, ty, M); addy(M, xc, y);
        xat(cell + a.nx, xn);
        couple_mp(k, ty, tt, M); addy(M, xn, y);
    } else {
        face_plus(fmax(a.ky, kMipC * Dy * a.ihy) * a.ihy, ty, M); addy(M, xc, y);
    }
}

// per-cell operator data and the inverse of the diagonal block, once per solve
__global__ void mip_prepare_kernel(MipArgs a, const int *mask, double *cf, float *binv,
                                   float *cf32) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (mask && mask[b] != 1) return;
    const long long cell = (long long)blk.x * blockDim.x + threadIdx.x;
    if (cell >= a.ncell) return;
    const int i = (int)(cell % a.nx), j = (int)(cell / a.nx);
    const CellCoef cc = coef_at(a, b, cell);
    const double kr = i + 1 < a.nx ? kap_int(cc.Dx, coef_at(a, b, cell + 1).Dx, a.hx, a.kx) : 0.0;
    const double kt = j + 1 < a.ny ? kap_int(cc.Dy, coef_at(a, b, cell + a.nx).Dy, a.hy, a.ky) : 0.0;
    double *c = cf + (size_t)b * kCf * a.ncell + cell;
    c[0] = cc.sa;
    c[1 * a.ncell] = cc.Dx;
    c[2 * a.ncell] = cc.Dy;
    c[3 * a.ncell] = kr;
    c[4 * a.ncell] = kt;
    if (cf32) {
        float *c32 = cf32 + (size_t)b * kCf * a.ncell + cell;
        c32[0] = (float)cc.sa;
        c32[1 * a.ncell] = (float)cc.Dx;
        c32[2 * a.ncell] = (float)cc.Dy;
        c32[3 * a.ncell] = (float)kr;
        c32[4 * a.ncell] = (float)kt;
    }
    double A[16], col[4][4];
    mip_diag(a, b, i, j, A);
    for (int k = 0; k < 4; ++k) {
        double e[4] = {0.0, 0.0, 0.0, 0.0};
        e[k] = 1.0;
        spd4_solve(A, e, col[k]);        // column k of A^-1
    }
    float *q = binv + (size_t)b * kBinv * a.ncell + cell;
    int idx = 0;
    for (int r = 0; r < 4; ++r)
        for (int k = r; k < 4; ++k) q[(idx++) * a.ncell] = (float)col[k][r];
}

// fixed-order block sum of two values; thread 0 returns the totals
__device__ void block_sum2(double &v0, double &v1) {
    __shared__ double sh[2][kCgBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        v0 += __shfl_xor(v0, off, 64);
        v1 += __shfl_xor(v1, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sh[0][w] = v0; sh[1][w] = v1; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int k = 0; k < kCgBlock / 64; ++k) { a += sh[0][k]; c += sh[1][k]; }
        v0 = a; v1 = c;
    }
}

// Sum of an instance's n block partials, computed by a whole wave (all 64 lanes must be active):
// lane l adds p[l], p[l + 64], ... in order, then a butterfly over the wave.  Partner lanes add
// the same two values in opposite order, and IEEE addition is commutative, so every lane ends
// with the same bits; the order depends on n only, so every block and wave that needs the sum
// gets the same value.  (One memory round trip per wave: a lane-serial loop over the partials
// waits on n dependent loads, and every block of every CG kernel repeats it.)
__device__ double sum_parts(const double *p, int n) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int k = lane; k < n; k += 64) s += p[k];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// partial-sum layout: part[b][slot][nblk], slots: 0,1 = rz (parity), 2 = pq, 3 = rr, 4 = bb
__device__ __forceinline__ double *slot(double *part, int b, int s, int nblk) {
    return part + ((size_t)b * 5 + s) * nblk;
}

// Warm start, first pass: with d the instance's previous correction, b = Sigma_s (rho* - rho_prev)
// is stored in r and A d in q, and the partials of (d, b) and (d, A d) go to slots 2 and 1.
__global__ void __launch_bounds__(kCgBlock) cg_warm_kernel(MipArgs a, const double *rho_star,
                                                           const double *rho_prev, const int *kind,
                                                           int want, const double *d, double *r,
                                                           double *q, double *part) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (kind && kind[b] != want) return;
    const long long cell = (long long)blk.x * kCgBlock + threadIdx.x;
    double db = 0.0, dad = 0.0;
    if (cell < a.ncell) {
        const size_t base = (size_t)b * a.ncell;
        const long long gi = (long long)base + cell;
        const double ss = a.sigma_s[gi];
        double rs[4], rp[4], bv[4], dc[4], y[4];
        load4(rho_star, gi, rs);
        if (rho_prev) load4(rho_prev, gi, rp);
        else rp[0] = rp[1] = rp[2] = rp[3] = 0.0;
        for (int k = 0; k < 4; ++k) bv[k] = ss * (rs[k] - rp[k]);
        auto dat = [&](long long c, double v[4]) { load4(d, base + c, v); };
        mip_apply(a, b, (int)(cell % a.nx), (int)(cell / a.nx), dat, y);
        load4(d, gi, dc);
        store4(r, gi, bv);
        store4(q, gi, y);
        for (int k = 0; k < 4; ++k) { db += dc[k] * bv[k]; dad += dc[k] * y[k]; }
    }
    block_sum2(db, dad);
    if (threadIdx.x == 0) {
        slot(part, b, 2, a.nblk)[blk.x] = db;
        slot(part, b, 1, a.nblk)[blk.x] = dad;
    }
}

// CG start.  Cold (d == nullptr): x = 0, r = b.  Warm: x = alpha d, r = b - alpha A d with
// alpha = (d, b) / (d, A d), the multiple of d closest to the solution in the energy norm
// (alpha = 0 when d = 0 or the quotient is not a positive finite number); r and A d come from
// cg_warm_kernel.  The stopping test stays relative to ||b||: slot 3 starts as the partials of
// (b, b), so the test before the first iteration stops only a zero (or NaN) right-hand side.
template <typename TZ>
__global__ void __launch_bounds__(kCgBlock) cg_setup_kernel(MipArgs a, const double *rho_star,
                                                            const double *rho_prev, const int *kind,
                                                            int want, const double *d,
                                                            const double *q, double *x, double *r,
                                                            TZ *z, double *part, int *state,
                                                            int *iters, int *n_running, int bj) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    const bool mine = !kind || kind[b] == want;
    if (!mine) {
        if (blk.x == 0 && threadIdx.x == 0) state[b] = 0;
        return;
    }
    double alpha = 0.0;
    if (d) {
        const double db = sum_parts(slot(part, b, 2, a.nblk), a.nblk);
        const double dad = sum_parts(slot(part, b, 1, a.nblk), a.nblk);
        alpha = dad > 0.0 ? db / dad : 0.0;
        if (!(fabs(alpha) < INFINITY)) alpha = 0.0;
    }
    // slots 1 and 2 are only read here and slots 0, 3 and 4 only written, so blocks need no order
    const long long cell = (long long)blk.x * kCgBlock + threadIdx.x;
    double rz = 0.0, bb = 0.0;
    if (cell < a.ncell) {
        const long long gi = (long long)b * a.ncell + cell;
        double bv[4], rv[4], xv[4], zv[4];
        if (d) {
            double dv[4], qv[4];
            load4(r, gi, bv);
            load4(d, gi, dv);
            load4(q, gi, qv);
            for (int k = 0; k < 4; ++k) { xv[k] = alpha * dv[k]; rv[k] = bv[k] - alpha * qv[k]; }
        } else {
            const double ss = a.sigma_s[gi];
            double rs[4], rp[4];
            load4(rho_star, gi, rs);
            if (rho_prev) load4(rho_prev, gi, rp);
        else rp[0] = rp[1] = rp[2] = rp[3] = 0.0;
            for (int k = 0; k < 4; ++k) { bv[k] = ss * (rs[k] - rp[k]); xv[k] = 0.0; rv[k] = bv[k]; }
        }
        store4(x, gi, xv);
        store4(r, gi, rv);
        if (bj) {
            binv_apply(a, b, cell, rv, zv);
            for (int k = 0; k < 4; ++k) zv[k] = (double)(TZ)(bj == 2 ? kOmegaDG * zv[k] : zv[k]);
            store4(z, gi, zv);
            for (int k = 0; k < 4; ++k) rz += rv[k] * zv[k];
        }
        for (int k = 0; k < 4; ++k) bb += bv[k] * bv[k];
    }
    block_sum2(rz, bb);
    if (threadIdx.x == 0) {
        slot(part, b, 0, a.nblk)[blk.x] = rz;
        slot(part, b, 3, a.nblk)[blk.x] = bb;
        slot(part, b, 4, a.nblk)[blk.x] = bb;
        if (blk.x == 0) {
            state[b] = 1;
            iters[b] = 0;
            atomicAdd(n_running, 1);
        }
    }
}

// iteration it >= 1: convergence test on the previous residual, p = z + beta p_old, q = A p
template <typename TZ>
__global__ void __launch_bounds__(kCgBlock) cg_matvec_kernel(MipArgs a, int it, double rtol2,
                                                             int maxit, const TZ *z,
                                                             const double *p_old, double *p_new,
                                                             double *q, double *part, int *state,
                                                             int *iters, int *n_running) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state[b] != 1) return;
    const int nb = a.nblk;
    const double bb = sum_parts(slot(part, b, 4, nb), nb);
    const double rr = it == 1 ? bb : sum_parts(slot(part, b, 3, nb), nb);
    const bool done = !(rr > rtol2 * bb);     // also stops on NaN
    if (done || it > maxit) {
        if (blk.x == 0 && threadIdx.x == 0) {
            const int st = done && rr == rr ? 2 : 3;
            state[b] = st;
            iters[b] = it - 1;
            atomicSub(n_running, 1);
            if (st == 3) atomicAdd(n_running + 1, 1);
        }
        return;
    }
    double beta = 0.0;
    if (it > 1) {
        const double rz_cur = sum_parts(slot(part, b, (it - 1) & 1, nb), nb);
        const double rz_prev = sum_parts(slot(part, b, it & 1, nb), nb);
        beta = rz_cur / rz_prev;
    }
    const long long cell = (long long)blk.x * kCgBlock + threadIdx.x;
    double pq = 0.0, dummy = 0.0;
    if (cell < a.ncell) {
        const size_t base = (size_t)b * a.ncell;
        auto pat = [&](long long c, double v[4]) {
            double zz[4];
            load4(z, base + c, zz);
            if (it > 1) {
                double po[4];
                load4(p_old, base + c, po);
                for (int k = 0; k < 4; ++k) v[k] = zz[k] + beta * po[k];
            } else {
                for (int k = 0; k < 4; ++k) v[k] = zz[k];
            }
        };
        const int i = (int)(cell % a.nx), j = (int)(cell / a.nx);
        double y[4], pc[4];
        mip_apply(a, b, i, j, pat, y);
        pat(cell, pc);
        store4(p_new, base + cell, pc);
        store4(q, base + cell, y);
        for (int k = 0; k < 4; ++k) pq += pc[k] * y[k];
    }
    block_sum2(pq, dummy);
    if (threadIdx.x == 0) slot(part, b, 2, nb)[blk.x] = pq;
}

// Tiled operator applications.  A block of kCgBlock threads owns a 16 x 16 tile of cells (tile
// index = block index, row-major over the mesh's tiles), so these kernels need the per-instance
// block count to equal the tile count.  The value the operator acts on is formed once per cell of
// the tile and of its one-cell halo into LDS, and the five-cell stencil reads it from there; the
// one-cell-per-thread kernels form it again for each of a cell's four neighbours, from global
// memory.
constexpr int kTile = 16;
constexpr int kTileW = kTile + 2;
static_assert(kTile * kTile == kCgBlock, "one thread per cell of a tile");

struct TileCell {
    int i, j, me;          // mesh coordinates, LDS position
    bool in;               // inside the mesh
    long long cell;
};

__device__ __forceinline__ TileCell tile_cell(const MipArgs &a, int ntx, int tile) {
    const int tx = tile % ntx, ty = tile / ntx;
    const int li = threadIdx.x % kTile, lj = threadIdx.x / kTile;
    TileCell t;
    t.i = tx * kTile + li;
    t.j = ty * kTile + lj;
    t.in = t.i < a.nx && t.j < a.ny;
    t.cell = (long long)t.j * a.nx + t.i;
    t.me = (lj + 1) * kTileW + li + 1;
    return t;
}

// sp[] <- val(cell) for every in-mesh cell of the tile and of its halo; own[] <- the thread's own
// cell's value.  Ends with a barrier; every thread of the block must call it.
template <typename F>
__device__ void tile_fill(const MipArgs &a, int ntx, int tile, const TileCell &tc, F val,
                          double4 *sp, double own[4]) {
    if (tc.in) {
        val(tc.cell, own);
        sp[tc.me] = make_double4(own[0], own[1], own[2], own[3]);
    }
    // the halo: left, right, bottom and top edges, one per wavefront (16 lanes each), so that no
    // wavefront carries all the extra loads
    static_assert(kCgBlock == 4 * 64, "four wavefronts, one halo side each");
    if ((threadIdx.x & 63) < kTile) {
        const int tx = tile % ntx, ty = tile / ntx;
        const int side = threadIdx.x >> 6, t = threadIdx.x & 63;
        const int hi = side == 0 ? tx * kTile - 1 : side == 1 ? tx * kTile + kTile : tx * kTile + t;
        const int hj = side == 2 ? ty * kTile - 1 : side == 3 ? ty * kTile + kTile : ty * kTile + t;
        const int at = side == 0 ? (t + 1) * kTileW
                     : side == 1 ? (t + 1) * kTileW + kTile + 1
                     : side == 2 ? t + 1 : (kTile + 1) * kTileW + t + 1;
        if (hi >= 0 && hi < a.nx && hj >= 0 && hj < a.ny) {
            double v[4];
            val((long long)hj * a.nx + hi, v);
            sp[at] = make_double4(v[0], v[1], v[2], v[3]);
        }
    }
    __syncthreads();
}

// reader of the tile's values for the operator: a neighbour's linear offset from the cell is
// -1, +1, -nx or +nx (0: the cell itself, read for a missing neighbour and weighted by zero)
struct TileReader {
    const double4 *sp;
    long long cell, nx;
    int me;
    __device__ void operator()(long long c, double v[4]) const {
        const long long d = c - cell;
        int o = (int)d;
        if (d == nx) o = kTileW;
        else if (d == -nx) o = -kTileW;
        const double4 t = sp[me + o];
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
};

template <typename TZ>
__global__ void __launch_bounds__(kCgBlock) cg_matvec_tile_kernel(MipArgs a, int ntx, int it,
                                                                  double rtol2, int maxit,
                                                                  const TZ *z,
                                                                  const double *p_old,
                                                                  double *p_new, double *q,
                                                                  double *part, int *state,
                                                                  int *iters, int *n_running) {
    __shared__ double4 sp[kTileW * kTileW];
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state[b] != 1) return;
    const int nb = a.nblk;
    const double bb = sum_parts(slot(part, b, 4, nb), nb);
    const double rr = it == 1 ? bb : sum_parts(slot(part, b, 3, nb), nb);
    const bool done = !(rr > rtol2 * bb);     // also stops on NaN
    if (done || it > maxit) {
        if (blk.x == 0 && threadIdx.x == 0) {
            const int st = done && rr == rr ? 2 : 3;
            state[b] = st;
            iters[b] = it - 1;
            atomicSub(n_running, 1);
            if (st == 3) atomicAdd(n_running + 1, 1);
        }
        return;
    }
    double beta = 0.0;
    if (it > 1) {
        const double rz_cur = sum_parts(slot(part, b, (it - 1) & 1, nb), nb);
        const double rz_prev = sum_parts(slot(part, b, it & 1, nb), nb);
        beta = rz_cur / rz_prev;
    }
    const size_t base = (size_t)b * a.ncell;
    auto pat = [&](long long c, double v[4]) {
        double zz[4];
        load4(z, base + c, zz);
        if (it > 1) {
            double po[4];
            load4(p_old, base + c, po);
            for (int k = 0; k < 4; ++k) v[k] = zz[k] + beta * po[k];
        } else {
            for (int k = 0; k < 4; ++k) v[k] = zz[k];
        }
    };
    const TileCell tc = tile_cell(a, ntx, blk.x);
    double pc[4] = {0.0, 0.0, 0.0, 0.0};
    tile_fill(a, ntx, blk.x, tc, pat, sp, pc);
    double pq = 0.0, dummy = 0.0;
    if (tc.in) {
        double y[4];
        mip_apply_hoisted<double>(a, b, tc.i, tc.j, TileReader{sp, tc.cell, a.nx, tc.me}, y);
        store4(p_new, base + tc.cell, pc);
        store4(q, base + tc.cell, y);
        for (int k = 0; k < 4; ++k) pq += pc[k] * y[k];
    }
    block_sum2(pq, dummy);
    if (threadIdx.x == 0) slot(part, b, 2, nb)[blk.x] = pq;
}

template <typename TZ>
__global__ void __launch_bounds__(kCgBlock) cg_update_kernel(MipArgs a, int it, const double *p,
                                                             const double *q, double *x, double *r,
                                                             TZ *z, double *part,
                                                             const int *state, int *iters, int bj) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state[b] != 1) return;
    const int nb = a.nblk;
    const double pq = sum_parts(slot(part, b, 2, nb), nb);
    const double rz = sum_parts(slot(part, b, (it - 1) & 1, nb), nb);
    const double alpha = rz / pq;
    const long long cell = (long long)blk.x * kCgBlock + threadIdx.x;
    double rz_new = 0.0, rr = 0.0;
    if (cell < a.ncell) {
        const long long gi = (long long)b * a.ncell + cell;
        double pv[4], qv[4], xv[4], rv[4], zv[4];
        load4(p, gi, pv);
        load4(q, gi, qv);
        load4(x, gi, xv);
        load4(r, gi, rv);
        for (int k = 0; k < 4; ++k) { xv[k] += alpha * pv[k]; rv[k] -= alpha * qv[k]; }
        store4(x, gi, xv);
        store4(r, gi, rv);
        if (bj) {
            binv_apply(a, b, cell, rv, zv);
            for (int k = 0; k < 4; ++k) zv[k] = (double)(TZ)(bj == 2 ? kOmegaDG * zv[k] : zv[k]);
            store4(z, gi, zv);
            for (int k = 0; k < 4; ++k) rz_new += rv[k] * zv[k];
        }
        for (int k = 0; k < 4; ++k) rr += rv[k] * rv[k];
    }
    block_sum2(rz_new, rr);
    if (threadIdx.x == 0) {
        if (bj == 1) slot(part, b, it & 1, nb)[blk.x] = rz_new;
        slot(part, b, 3, nb)[blk.x] = rr;
        if (blk.x == 0) iters[b] = it;   // updates done; final once the instance stops
    }
}

__global__ void cg_finish_kernel(long long ndof, const double *x, double *delta, const int *state,
                                 const int *iters, int *iters_out, unsigned long long *total,
                                 int *fails, int B) {
    const Blk blk = xcd_block();
    const long long t = (long long)blk.x * blockDim.x + threadIdx.x;
    const int b = blk.y;
    const int st = state[b];
    if (st == 0) return;
    if (x && t < ndof) delta[(size_t)b * ndof + t] = x[(size_t)b * ndof + t];
    if (t == 0 && iters_out) iters_out[b] = iters[b];
    if (t == 0 && total) atomicAdd(total, (unsigned long long)iters[b]);
    if (t == 0 && fails && st == 3) atomicAdd(fails, 1);
}

// a CG call's start: no instance running or failed yet, and the call's squared relative tolerance
__global__ void cg_begin_kernel(int *n_running, double *tol2, double rtol2) {
    if (threadIdx.x == 0) {
        n_running[0] = 0;
        n_running[1] = 0;
        *tol2 = rtol2;
    }
}

// ------------------------------------------------------------------------- multigrid
// Two-level preconditioner for the MIP system: damped block-Jacobi smoothing on the DG space and
// a coarse correction on continuous Q1 functions (vertex values, interpolated into every cell:
// the embedding P), whose operator P^T A P and the operators of coarser vertex grids
// (bilinear interpolation, Galerkin R A P with R = P^T) are computed by probing with nine
// colourings of the vertices; the vertex-grid problem is solved approximately by one V-cycle
// with damped point-Jacobi smoothing.  Every smoother is symmetric, so the preconditioner is.
constexpr double kOmegaV = 2.0 / 3.0;

struct VG {
    int nvx, nvy;
    long long nv;
};

// DG coefficients of the bilinear interpolant of the vertex values around cell (i, j)
__device__ __forceinline__ void p_cell(const double *xv, int nvx, int i, int j, double sqa,
                                       double c[4]) {
    const double u00 = xv[(long long)j * nvx + i], u10 = xv[(long long)j * nvx + i + 1];
    const double u01 = xv[(long long)(j + 1) * nvx + i], u11 = xv[(long long)(j + 1) * nvx + i + 1];
    c[0] = sqa * 0.25 * (u00 + u10 + u01 + u11);
    c[1] = sqa * 0.25 * ((u10 + u11) - (u00 + u01)) / kS3;
    c[2] = sqa * 0.25 * ((u01 + u11) - (u00 + u10)) / kS3;
    c[3] = sqa * 0.25 * (u11 - u10 - u01 + u00) / 3.0;
}

// P^T: vertex (x, y) gathers from the (up to four) cells having it as a corner
template <typename TZ>
__device__ __forceinline__ double pt_vertex(const TZ *rdg, int nx, int ny, int x, int y,
                                            double sqa) {
    // the (up to four) cells' values are loaded before the sum: a missing cell reads cell (0, 0)
    // and a select leaves it out; the sum keeps its order and its terms
    double rv[4][4];
    bool ok[4];
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
            const int i = x - 1 + cx, j = y - 1 + cy;     // cell; the vertex is its corner (1-cx, 1-cy)
            const int k = cy * 2 + cx;
            ok[k] = i >= 0 && j >= 0 && i < nx && j < ny;
            load4(rdg, ok[k] ? (long long)j * nx + i : 0LL, rv[k]);
        }
    double s = 0.0;
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
            const int k = cy * 2 + cx;
            const double sx = cx == 0 ? 1.0 : -1.0;       // corner a = 1 - cx: sign +1 if a == 1
            const double sy = cy == 0 ? 1.0 : -1.0;
            const double *r = rv[k];
            s = ok[k] ? s + sqa * (0.25 * r[0] + sx * r[1] / (4.0 * kS3) + sy * r[2] / (4.0 * kS3) + sx * sy * r[3] / 12.0) : s;
        }
    return s;
}

// t = r - A z.  First the CG's convergence test on the (r, r) partials of the update just done
// (the matvec kernel's test, on the same fixed-order sums): an instance that passes it stops
// here, so it skips the rest of the preconditioner and the next iteration.  Every block reaches
// the same decision; block 0 records it.
template <typename TZ>
__global__ void mg_resid_dg_kernel(MipArgs a, int *state, const double *r, const TZ *z,
                                   TZ *t, const double *part, const double *tol2,
                                   int *n_running) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state[b] != 1) return;
    {
        const double bb = sum_parts(part + ((size_t)b * 5 + 4) * a.nblk, a.nblk);
        const double rr = sum_parts(part + ((size_t)b * 5 + 3) * a.nblk, a.nblk);
        if (!(rr > tol2[0] * bb)) {
            if (blk.x == 0 && threadIdx.x == 0) {
                const int st = rr == rr ? 2 : 3;
                state[b] = st;
                atomicSub(n_running, 1);
                if (st == 3) atomicAdd(n_running + 1, 1);
            }
            return;
        }
    }
    const long long cell = (long long)blk.x * blockDim.x + threadIdx.x;
    if (cell >= a.ncell) return;
    const size_t base = (size_t)b * a.ncell;
    auto zat = [&](long long c, double v[4]) { load4(z, base + c, v); };
    double y[4], rv[4];
    if constexpr (std::is_same<TZ, float>::value)
        mip_apply_hoisted<TZ>(a, b, (int)(cell % a.nx), (int)(cell / a.nx), zat, y);
    else
        mip_apply<TZ>(a, b, (int)(cell % a.nx), (int)(cell / a.nx), zat, y);
    load4(r, base + cell, rv);
    for (int k = 0; k < 4; ++k) y[k] = rv[k] - y[k];
    store4(t, base + cell, y);
}

// b0 = P^T t (level-0 vertex grid); with x0 non-null also level 0's first smoothing step from
// zero, x0 = omega b0 / diag (the tenth plane of S0)
template <typename TZ>
__global__ void mg_restrict_dg_kernel(MipArgs a, const int *state, const TZ *t, VG g,
                                      double *b0, const float *S0, double *x0) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state && state[b] != 1) return;
    const long long v = (long long)blk.x * blockDim.x + threadIdx.x;
    if (v >= g.nv) return;
    const int x = (int)(v % g.nvx), y = (int)(v / g.nvx);
    const double bv = pt_vertex(t + (size_t)b * a.ncell * 4, a.nx, a.ny, x, y, sqrt(a.hx * a.hy));
    b0[(size_t)b * g.nv + v] = bv;
    if (x0) {
        const double wd = S0[((size_t)b * kStencilPlanes + 9) * g.nv + v];
        x0[(size_t)b * g.nv + v] = wd * bv;
    }
}

// ---- vertex grids: 9-point stencils in planes, S[b][(dy+1)*3 + dx+1][v], and a tenth plane
// S[b][9][v] = omega / diagonal (kStencilPlanes planes of nv values per instance)
template <typename TS>
__device__ __forceinline__ const TS *st_of(const TS *S, int b, long long nv) {
    return S + (size_t)b * kStencilPlanes * nv;
}
template <typename TS>
__device__ __forceinline__ TS *st_of(TS *S, int b, long long nv) {
    return S + (size_t)b * kStencilPlanes * nv;
}
// The FP32 copy of a Galerkin operator is read as the symmetric operator it is in exact
// arithmetic: the coupling of v to its neighbour v + d for the four offsets d before it in
// plane order (k < 4) is taken from that neighbour's plane 8 - k (its coupling back to v).  A
// V-cycle thus reads planes 4..9 only, and its operator is exactly symmetric.
template <typename TS>
__device__ __forceinline__ TS stencil_coef(const TS *Sb, int k, long long nv, long long v,
                                           long long w) {
    if constexpr (std::is_same<TS, float>::value)
        return k < 4 ? Sb[(8 - k) * nv + w] : Sb[k * nv + v];
    else
        return Sb[k * nv + v];
}

template <typename TS>
__device__ __forceinline__ double stencil_apply(const TS *Sb, const double *x, VG g, int vx,
                                                int vy) {
    // the nine (coefficient, value) pairs are loaded before the sum: a neighbour outside the
    // grid reads the vertex itself and a select leaves it out, so no load waits behind a branch;
    // the sum keeps its order and its terms
    const long long v = (long long)vy * g.nvx + vx;
    double cv[9], xv[9];
    bool ok[9];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int k = (dy + 1) * 3 + dx + 1;
            const int yy = vy + dy, xx = vx + dx;
            ok[k] = yy >= 0 && yy < g.nvy && xx >= 0 && xx < g.nvx;
            const long long w = ok[k] ? (long long)yy * g.nvx + xx : v;
            cv[k] = (double)stencil_coef(Sb, k, g.nv, v, w);
            xv[k] = x[w];
        }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) s = ok[k] ? s + cv[k] * xv[k] : s;
    return s;
}

// mode 0: x_out = omega b / diag; 1: x_out = x_in + omega (b - S x_in)/diag; 2: out = b - S x_in;
// 3: out = S x_in
template <typename TS>
__global__ void mg_vertex_kernel(const int *state, VG g, const TS *S, const double *x_in,
                                 const double *bv, double *out, int mode) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state && state[b] != 1) return;
    const long long v = (long long)blk.x * blockDim.x + threadIdx.x;
    if (v >= g.nv) return;
    const size_t o = (size_t)b * g.nv;
    const TS *Sb = st_of(S, b, g.nv);
    const double wd = Sb[9 * g.nv + v];
    const int vx = (int)(v % g.nvx), vy = (int)(v / g.nvx);
    double res;
    if (mode == 0) res = wd * bv[o + v];
    else if (mode == 1) res = x_in[o + v] + wd * (bv[o + v] - stencil_apply(Sb, x_in + o, g, vx, vy));
    else if (mode == 2) res = bv[o + v] - stencil_apply(Sb, x_in + o, g, vx, vy);
    else res = stencil_apply(Sb, x_in + o, g, vx, vy);
    out[o + v] = res;
}

// coarse b_c = R r_f (R = transpose of bilinear interpolation); with xc non-null also the coarse
// level's first smoothing step from zero, x_c = omega b_c / diag (the tenth plane of Sc)
__global__ void mg_vrestrict_kernel(const int *state, VG gf, const double *rf, VG gc, double *bc,
                                    const float *Sc, double *xc) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state && state[b] != 1) return;
    const long long v = (long long)blk.x * blockDim.x + threadIdx.x;
    if (v >= gc.nv) return;
    const int X = (int)(v % gc.nvx), Y = (int)(v / gc.nvx);
    const double *r = rf + (size_t)b * gf.nv;
    // the nine fine values are loaded before the sum (a point outside the grid reads the centre
    // and a select leaves it out); the sum keeps its order and its terms
    double rv[9];
    bool ok[9];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int k = (dy + 1) * 3 + dx + 1;
            const int y = 2 * Y + dy, x = 2 * X + dx;
            ok[k] = y >= 0 && y < gf.nvy && x >= 0 && x < gf.nvx;
            rv[k] = r[ok[k] ? (long long)y * gf.nvx + x : (long long)(2 * Y) * gf.nvx + 2 * X];
        }
    double s = 0.0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int k = (dy + 1) * 3 + dx + 1;
            s = ok[k] ? s + (dx == 0 ? 1.0 : 0.5) * (dy == 0 ? 1.0 : 0.5) * rv[k] : s;
        }
    bc[(size_t)b * gc.nv + v] = s;
    if (xc) {
        const double wd = st_of(Sc, b, gc.nv)[9 * gc.nv + v];
        xc[(size_t)b * gc.nv + v] = wd * s;
    }
}

// probing: e = indicator of the vertices of colour (cx, cy) (coordinates mod 3)
__global__ void mg_colour_kernel(const int *state, VG g, int cx, int cy, double *e) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state && state[b] != 1) return;
    const long long v = (long long)blk.x * blockDim.x + threadIdx.x;
    if (v >= g.nv) return;
    const int x = (int)(v % g.nvx), y = (int)(v / g.nvx);
    e[(size_t)b * g.nv + v] = (x % 3 == cx && y % 3 == cy) ? 1.0 : 0.0;
}

// t = A (P e) on the DG space
__global__ void mg_probe_dg_kernel(MipArgs a, const int *state, const double *e, VG g, double *t) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state && state[b] != 1) return;
    const long long cell = (long long)blk.x * blockDim.x + threadIdx.x;
    if (cell >= a.ncell) return;
    const double sqa = sqrt(a.hx * a.hy);
    const double *eb = e + (size_t)b * g.nv;
    auto pat = [&](long long c, double v[4]) { p_cell(eb, g.nvx, (int)(c % a.nx), (int)(c / a.nx), sqa, v); };
    double y[4];
    mip_apply(a, b, (int)(cell % a.nx), (int)(cell / a.nx), pat, y);
    store4(t, (size_t)b * a.ncell + cell, y);
}

// S[v][offset to the colour-(cx,cy) vertex of v's 3x3 neighbourhood] = z[v]
__global__ void mg_scatter_kernel(const int *state, VG g, int cx, int cy, const double *z,
                                  double *S) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state && state[b] != 1) return;
    const long long v = (long long)blk.x * blockDim.x + threadIdx.x;
    if (v >= g.nv) return;
    const int x = (int)(v % g.nvx), y = (int)(v / g.nvx);
    const int mx = ((cx - x) % 3 + 3) % 3, my = ((cy - y) % 3 + 3) % 3;
    const int dx = mx == 2 ? -1 : mx, dy = my == 2 ? -1 : my;
    if (x + dx < 0 || x + dx >= g.nvx || y + dy < 0 || y + dy >= g.nvy) return;
    st_of(S, b, g.nv)[((dy + 1) * 3 + dx + 1) * g.nv + v] = z[(size_t)b * g.nv + v];
}

// Galerkin operator of a coarse vertex level, S_c = R S_f P with the bilinear prolongation P
// (weight 1 at the coincident fine vertex, 1/2 per axis at odd fine coordinates) and R = P^T.
// One thread per coarse vertex I: the fine vertices i of R's row, their stencil entries
// S_f[i][j], and the coarse parents J of every j, all within one coarse neighbour of I.
__device__ __forceinline__ double p_weight(int fine, int coarse) {
    const int d = fine - 2 * coarse;
    return d == 0 ? 1.0 : ((d == 1 || d == -1) ? 0.5 : 0.0);
}

__global__ void mg_galerkin_kernel(const int *state, VG gf, const double *Sf, VG gc, double *Sc) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state && state[b] != 1) return;
    const long long v = (long long)blk.x * blockDim.x + threadIdx.x;
    if (v >= gc.nv) return;
    const int X = (int)(v % gc.nvx), Y = (int)(v / gc.nvx);
    const double *Sb = st_of(Sf, b, gf.nv);
    double acc[9];
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
    for (int dy = -1; dy <= 1; ++dy) {
        const int iy = 2 * Y + dy;
        if (iy < 0 || iy >= gf.nvy) continue;
        for (int dx = -1; dx <= 1; ++dx) {
            const int ix = 2 * X + dx;
            if (ix < 0 || ix >= gf.nvx) continue;
            const double r = p_weight(ix, X) * p_weight(iy, Y);
            const long long i = (long long)iy * gf.nvx + ix;
            for (int ey = -1; ey <= 1; ++ey) {
                const int jy = iy + ey;
                if (jy < 0 || jy >= gf.nvy) continue;
                for (int ex = -1; ex <= 1; ++ex) {
                    const int jx = ix + ex;
                    if (jx < 0 || jx >= gf.nvx) continue;
                    const double rs = r * Sb[((ey + 1) * 3 + ex + 1) * gf.nv + i];
                    // coarse parents of j: jx / 2 (and jx / 2 + 1 when jx is odd), the same in y
                    const int jx0 = jx >> 1, jy0 = jy >> 1;
                    for (int py = 0; py <= (jy & 1); ++py)
                        for (int px = 0; px <= (jx & 1); ++px) {
                            const int JX = jx0 + px, JY = jy0 + py;
                            acc[(JY - Y + 1) * 3 + (JX - X + 1)] +=
                                rs * p_weight(jx, JX) * p_weight(jy, JY);
                        }
                }
            }
        }
    }
    double *Cb = st_of(Sc, b, gc.nv);
    for (int k = 0; k < 9; ++k) Cb[(long long)k * gc.nv + v] = acc[k];
}

// omega / diagonal plane of the smoother
__global__ void mg_wdiag_kernel(const int *state, VG g, double *S) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state && state[b] != 1) return;
    const long long v = (long long)blk.x * blockDim.x + threadIdx.x;
    if (v >= g.nv) return;
    double *Sb = st_of(S, b, g.nv);
    Sb[9 * g.nv + v] = kOmegaV / Sb[4 * g.nv + v];
}

// FP32 copy of an instance's stencil planes (the V-cycle's copy)
__global__ void mg_round_kernel(const int *state, long long n, const double *x, float *y) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state && state[b] != 1) return;
    const long long t = (long long)blk.x * blockDim.x + threadIdx.x;
    if (t < n) y[(size_t)b * n + t] = (float)x[(size_t)b * n + t];
}

__global__ void mg_zero_kernel(const int *state, long long n, double *x) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state && state[b] != 1) return;
    const long long t = (long long)blk.x * blockDim.x + threadIdx.x;
    if (t < n) x[(size_t)b * n + t] = 0.0;
}

// Inverse of the coarsest operator of the instances with mask[b] == 1 (all if null), one
// workgroup per instance: the dense matrix from the 9-point stencils, Gauss-Jordan elimination in
// LDS (the operator is SPD: no pivoting), inverse to cinv [B][nc][nc].
__global__ void __launch_bounds__(256) mg_coarse_invert_kernel(const int *mask, VG g,
                                                               const double *S, double *cinv) {
    extern __shared__ double sh[];
    const int b = blockIdx.x;
    if (mask && mask[b] != 1) return;
    const int n = (int)g.nv, nn = n * n;
    double *A = sh, *X = sh + nn, *f = sh + 2 * nn;
    const double *Sb = st_of(S, b, g.nv);
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
        const int v = e / n, w = e - v * n;
        const int vx = v % g.nvx, vy = v / g.nvx, wx = w % g.nvx, wy = w / g.nvx;
        const int dx = wx - vx, dy = wy - vy;
        const bool nb = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1;
        A[e] = nb ? Sb[((dy + 1) * 3 + dx + 1) * g.nv + v] : 0.0;
        X[e] = v == w ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double piv = 1.0 / A[k * n + k];
        for (int i = threadIdx.x; i < n; i += blockDim.x) f[i] = A[i * n + k];
        __syncthreads();
        // row k scaled by 1/pivot, every other row i minus f_i times the scaled row k
        for (int e = threadIdx.x; e < nn; e += blockDim.x) {
            const int i = e / n, j = e - i * n;
            const double rk = A[k * n + j] * piv, xk = X[k * n + j] * piv;
            if (i == k) continue;
            A[e] -= f[i] * rk;
            X[e] -= f[i] * xk;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            A[k * n + j] *= piv;
            X[k * n + j] *= piv;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < nn; e += blockDim.x) cinv[(size_t)b * nn + e] = X[e];
}

// coarsest grid from zero: x = cinv b when the inverse exists, else nsweep damped Jacobi sweeps;
// one workgroup per instance, vectors in LDS
__global__ void __launch_bounds__(256) mg_coarse_kernel(const int *state, VG g, const float *S,
                                                        const double *bv, double *x, int nsweep,
                                                        const double *cinv) {
    extern __shared__ double sh[];
    const int b = blockIdx.x;
    if (state[b] != 1) return;
    double *xa = sh, *xb = sh + g.nv;
    const size_t o = (size_t)b * g.nv;
    if (cinv) {
        const int n = (int)g.nv;
        const double *Ci = cinv + (size_t)b * n * n;
        for (int v = threadIdx.x; v < n; v += blockDim.x) {
            double acc = 0.0;
            for (int w = 0; w < n; ++w) acc += Ci[v * n + w] * bv[o + w];
            x[o + v] = acc;
        }
        return;
    }
    const float *Sb = st_of(S, b, g.nv);
    const float *wd = Sb + 9 * g.nv;
    for (long long v = threadIdx.x; v < g.nv; v += blockDim.x) xa[v] = wd[v] * bv[o + v];
    __syncthreads();
    for (int k = 1; k < nsweep; ++k) {
        for (long long v = threadIdx.x; v < g.nv; v += blockDim.x) {
            const int vx = (int)(v % g.nvx), vy = (int)(v / g.nvx);
            xb[v] = xa[v] + wd[v] * (bv[o + v] - stencil_apply(Sb, xa, g, vx, vy));
        }
        __syncthreads();
        double *t = xa; xa = xb; xb = t;
    }
    for (long long v = threadIdx.x; v < g.nv; v += blockDim.x) x[o + v] = xa[v];
}


// ---- fused multigrid steps (fewer launches, no intermediate vectors)
// coarse correction, post-smoothing and (r, z) in one pass:
//   z' = z + P x0,  z_out = z' + omega D^-1 (r - A z'),  partial of (r, z_out) into slot s.
// z' of the neighbour cells is formed on the fly; z_out must not alias z (other workgroups read z).
template <typename TZ>
__global__ void __launch_bounds__(kCgBlock) mg_post_dg_kernel(MipArgs a, const int *state,
                                                              const double *r, const double *x0,
                                                              VG g, const TZ *z, TZ *z_out,
                                                              double *part, int s) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state[b] != 1) return;
    const long long cell = (long long)blk.x * kCgBlock + threadIdx.x;
    double rz = 0.0, dummy = 0.0;
    const size_t base = (size_t)b * a.ncell;
    if (cell < a.ncell) {
        const double sqa = sqrt(a.hx * a.hy);
        const double *xb = x0 + (size_t)b * g.nv;
        auto zat = [&](long long c, double v[4]) {
            double pc[4];
            load4(z, base + c, v);
            p_cell(xb, g.nvx, (int)(c % a.nx), (int)(c / a.nx), sqa, pc);
            for (int k = 0; k < 4; ++k) v[k] += pc[k];
        };
        double y[4], zc[4], rv[4], dz[4], zn[4];
        const int i = (int)(cell % a.nx), j = (int)(cell / a.nx);
        mip_apply<TZ>(a, b, i, j, zat, y);
        zat(cell, zc);
        load4(r, base + cell, rv);
        for (int k = 0; k < 4; ++k) y[k] = rv[k] - y[k];
        binv_apply(a, b, cell, y, dz);
        // (r, z) of the value as stored, so that the CG's beta matches the z it reads
        for (int k = 0; k < 4; ++k) {
            zn[k] = (double)(TZ)(zc[k] + kOmegaDG * dz[k]);
            rz += rv[k] * zn[k];
        }
        store4(z_out, base + cell, zn);
    }
    block_sum2(rz, dummy);
    if (threadIdx.x == 0) slot(part, b, s, a.nblk)[blk.x] = rz;
}

// mg_resid_dg_kernel on 16 x 16 tiles (t = r - A z with z read through LDS)
template <typename TZ>
__global__ void __launch_bounds__(kCgBlock) mg_resid_dg_tile_kernel(MipArgs a, int ntx, int *state,
                                                                    const double *r, const TZ *z,
                                                                    TZ *t, const double *part,
                                                                    const double *tol2,
                                                                    int *n_running) {
    __shared__ double4 sp[kTileW * kTileW];
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state[b] != 1) return;
    {
        const double bb = sum_parts(part + ((size_t)b * 5 + 4) * a.nblk, a.nblk);
        const double rr = sum_parts(part + ((size_t)b * 5 + 3) * a.nblk, a.nblk);
        if (!(rr > tol2[0] * bb)) {
            if (blk.x == 0 && threadIdx.x == 0) {
                const int st = rr == rr ? 2 : 3;
                state[b] = st;
                atomicSub(n_running, 1);
                if (st == 3) atomicAdd(n_running + 1, 1);
            }
            return;
        }
    }
    const size_t base = (size_t)b * a.ncell;
    auto zat = [&](long long c, double v[4]) { load4(z, base + c, v); };
    const TileCell tc = tile_cell(a, ntx, blk.x);
    double zc[4];
    tile_fill(a, ntx, blk.x, tc, zat, sp, zc);
    if (!tc.in) return;
    double y[4], rv[4];
    mip_apply_hoisted<TZ>(a, b, tc.i, tc.j, TileReader{sp, tc.cell, a.nx, tc.me}, y);
    load4(r, base + tc.cell, rv);
    for (int k = 0; k < 4; ++k) y[k] = rv[k] - y[k];
    store4(t, base + tc.cell, y);
}

// mg_post_dg_kernel on 16 x 16 tiles (z + P x0 formed once per cell into LDS)
template <typename TZ>
__global__ void __launch_bounds__(kCgBlock) mg_post_dg_tile_kernel(MipArgs a, int ntx,
                                                                   const int *state,
                                                                   const double *r,
                                                                   const double *x0, VG g,
                                                                   const TZ *z, TZ *z_out,
                                                                   double *part, int s) {
    __shared__ double4 sp[kTileW * kTileW];
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state[b] != 1) return;
    const size_t base = (size_t)b * a.ncell;
    const double sqa = sqrt(a.hx * a.hy);
    const double *xb = x0 + (size_t)b * g.nv;
    auto zat = [&](long long c, double v[4]) {
        double pc[4];
        load4(z, base + c, v);
        p_cell(xb, g.nvx, (int)(c % a.nx), (int)(c / a.nx), sqa, pc);
        for (int k = 0; k < 4; ++k) v[k] += pc[k];
    };
    const TileCell tc = tile_cell(a, ntx, blk.x);
    double zc[4] = {0.0, 0.0, 0.0, 0.0};
    tile_fill(a, ntx, blk.x, tc, zat, sp, zc);
    double rz = 0.0, dummy = 0.0;
    if (tc.in) {
        double y[4], rv[4], dz[4], zn[4];
        mip_apply_hoisted<TZ>(a, b, tc.i, tc.j, TileReader{sp, tc.cell, a.nx, tc.me}, y);
        load4(r, base + tc.cell, rv);
        for (int k = 0; k < 4; ++k) y[k] = rv[k] - y[k];
        binv_apply(a, b, tc.cell, y, dz);
        // (r, z) of the value as stored, so that the CG's beta matches the z it reads
        for (int k = 0; k < 4; ++k) {
            zn[k] = (double)(TZ)(zc[k] + kOmegaDG * dz[k]);
            rz += rv[k] * zn[k];
        }
        store4(z_out, base + tc.cell, zn);
    }
    block_sum2(rz, dummy);
    if (threadIdx.x == 0) slot(part, b, s, a.nblk)[blk.x] = rz;
}

// two damped Jacobi sweeps from zero: x1 = w D^-1 b, x2 = x1 + w D^-1 (b - S x1)
__global__ void mg_vpre_kernel(const int *state, VG g, const float *S, const double *bv, double *x2) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state[b] != 1) return;
    const long long v = (long long)blk.x * blockDim.x + threadIdx.x;
    if (v >= g.nv) return;
    const size_t o = (size_t)b * g.nv;
    const float *Sb = st_of(S, b, g.nv);
    const float *wd = Sb + 9 * g.nv;
    const double *bb = bv + o;
    const int vx = (int)(v % g.nvx), vy = (int)(v / g.nvx);
    double sx1 = 0.0;
    for (int dy = -1; dy <= 1; ++dy) {
        const int yy = vy + dy;
        if (yy < 0 || yy >= g.nvy) continue;
        for (int dx = -1; dx <= 1; ++dx) {
            const int xx = vx + dx;
            if (xx < 0 || xx >= g.nvx) continue;
            const long long w = (long long)yy * g.nvx + xx;
            sx1 += stencil_coef(Sb, (dy + 1) * 3 + dx + 1, g.nv, v, w) * (wd[w] * bb[w]);
        }
    }
    const double x1 = wd[v] * bb[v];
    x2[o + v] = x1 + wd[v] * (bb[v] - sx1);
}

__device__ __forceinline__ double prolong_at(const double *c, VG gc, int x, int y) {
    const int X0 = x / 2, Y0 = y / 2;
    const int X1 = (x & 1) ? X0 + 1 : X0, Y1 = (y & 1) ? Y0 + 1 : Y0;
    return 0.25 * (c[(long long)Y0 * gc.nvx + X0] + c[(long long)Y0 * gc.nvx + X1] +
                   c[(long long)Y1 * gc.nvx + X0] + c[(long long)Y1 * gc.nvx + X1]);
}

// x3 = x2 + P x_c, x4 = x3 + w D^-1 (b - S x3)
__global__ void mg_vpost1_kernel(const int *state, VG g, const float *S, const double *bv,
                                 const double *x2, VG gc, const double *xc, double *x4) {
    const Blk blk = xcd_block();
    const int b = blk.y;
    if (state[b] != 1) return;
    const long long v = (long long)blk.x * blockDim.x + threadIdx.x;
    if (v >= g.nv) return;
    const size_t o = (size_t)b * g.nv;
    const float *Sb = st_of(S, b, g.nv);
    const double *cb = xc + (size_t)b * gc.nv;
    const int vx = (int)(v % g.nvx), vy = (int)(v / g.nvx);
    // Every load is issued before the arithmetic.  The coarse values that the prolongation at
    // the nine neighbours reads all lie in the 3 x 3 coarse patch from (PX, PY) = ((vx - 1) >> 1,
    // (vy - 1) >> 1): for a fine offset d the two coarse columns (X0, X1) are patch columns
    // kP0/kP1[d + 1] of an even vx and kQ0/kQ1[d + 1] of an odd one (rows likewise).  Patch
    // entries outside the coarse grid are clamped in and used only by neighbours outside the
    // fine grid, which a select leaves out of the sum; such a neighbour's x2 reads the centre.
    constexpr int kP0[3] = {0, 1, 1}, kP1[3] = {1, 1, 2}, kQ0[3] = {0, 0, 1}, kQ1[3] = {0, 1, 1};
    const int PX = (vx - 1) >> 1, PY = (vy - 1) >> 1;
    const bool ex = (vx & 1) == 0, ey = (vy & 1) == 0;
    double cp[3][3], xn[9];
    float cv[9];
    bool ok[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int Y = min(max(PY + r, 0), gc.nvy - 1), X = min(max(PX + q, 0), gc.nvx - 1);
            cp[r][q] = cb[(long long)Y * gc.nvx + X];
        }
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int k = (dy + 1) * 3 + dx + 1;
            const int yy = vy + dy, xx = vx + dx;
            ok[k] = yy >= 0 && yy < g.nvy && xx >= 0 && xx < g.nvx;
            const long long w = ok[k] ? (long long)yy * g.nvx + xx : v;
            cv[k] = stencil_coef(Sb, k, g.nv, v, w);
            xn[k] = x2[o + w];
        }
    auto pick = [&](int re, int ro, int ce, int co) -> double {
        const double e = ex ? cp[re][ce] : cp[re][co];
        const double d = ex ? cp[ro][ce] : cp[ro][co];
        return ey ? e : d;
    };
    double sx3 = 0.0, x3 = 0.0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int k = (dy + 1) * 3 + dx + 1;
            const int a = dx + 1, c = dy + 1;
            // prolong_at's sum (Y0 X0, Y0 X1, Y1 X0, Y1 X1) on the patch values
            const double pv = 0.25 * (pick(kP0[c], kQ0[c], kP0[a], kQ0[a]) +
                                       pick(kP0[c], kQ0[c], kP1[a], kQ1[a]) +
                                       pick(kP1[c], kQ1[c], kP0[a], kQ0[a]) +
                                       pick(kP1[c], kQ1[c], kP1[a], kQ1[a]));
            const double xv = xn[k] + pv;
            if (k == 4) x3 = xv;
            sx3 = ok[k] ? sx3 + cv[k] * xv : sx3;
        }
    x4[o + v] = x3 + Sb[9 * g.nv + v] * (bv[o + v] - sx3);
}


// V-cycle over the small coarse levels ls..L-1 of one instance in one workgroup, all vectors and
// the FP32 stencils in LDS (the stencils are copied in once, so no sweep waits on global
// memory): same smoothing, restriction, prolongation and coarsest sweeps as the per-level kernels.
struct SmallLevels {
    int n;
    int nvx[kMaxLevels], nvy[kMaxLevels];
    long long nv[kMaxLevels];
    const float *S[kMaxLevels];
};

// n values from global memory into LDS, U loads in flight per thread before their stores
template <typename T, int U>
__device__ __forceinline__ void copy_to_lds(const T *src, T *dst, long long n, int t, int nt) {
    for (long long v0 = t; v0 < n; v0 += (long long)U * nt) {
        T tmp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long v = v0 + (long long)u * nt;
            tmp[u] = v < n ? src[v] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long v = v0 + (long long)u * nt;
            if (v < n) dst[v] = tmp[u];
        }
    }
}

// LDS layout: per level l, four vectors of nv doubles (xa, xb, bv, rv) at sh + o[l] + k nv, then
// every level's FP32 stencil planes at (float *)sh + os[l].  The shapes and offsets sit in LDS
// and every address is sh plus an integer, so the compiler keeps LDS accesses as ds_ operations:
// arrays of pointers or kernel-argument arrays indexed by the runtime level would go through
// private memory and turn each LDS access into a flat one.
struct SmallDesc {
    int nvx[kMaxLevels], nvy[kMaxLevels], nv[kMaxLevels], o[kMaxLevels], os[kMaxLevels];
};

__global__ void __launch_bounds__(1024) mg_small_vcycle_kernel(const int *state, SmallLevels sl,
                                                               const double *b_top, double *x_top,
                                                               int nsweep, const double *cinv) {
    extern __shared__ double sh[];
    __shared__ SmallDesc d;
    const int b = blockIdx.x;
    if (state[b] != 1) return;
    const int t = threadIdx.x, nt = blockDim.x;
    float *shf = reinterpret_cast<float *>(sh);
    {
        int o = 0;
#pragma unroll
        for (int l = 0; l < kMaxLevels; ++l)
            if (l < sl.n) o += 4 * (int)sl.nv[l];
        int os = 2 * o;
#pragma unroll
        for (int l = 0; l < kMaxLevels; ++l) {
            if (l < sl.n) {
                const long long nv = sl.nv[l];
                // planes 0..3 are never read (stencil_coef takes them from the neighbours'
                // planes 8..5), so only planes 4..9 are copied
                copy_to_lds<float, 12>(st_of(sl.S[l], b, nv) + 4 * nv, shf + os + 4 * nv,
                                       (kStencilPlanes - 4) * nv, t, nt);
                if (t == 0) {
                    d.nvx[l] = sl.nvx[l];
                    d.nvy[l] = sl.nvy[l];
                    d.nv[l] = (int)nv;
                    d.os[l] = os;
                }
                os += kStencilPlanes * (int)nv;
            }
        }
        if (t == 0) {
            int oo = 0;
#pragma unroll
            for (int l = 0; l < kMaxLevels; ++l)
                if (l < sl.n) { d.o[l] = oo; oo += 4 * (int)sl.nv[l]; }
        }
        // level 0's right-hand side (bv of level 0 sits at 2 nv[0])
        copy_to_lds<double, 4>(b_top + (size_t)b * sl.nv[0], sh + 2 * sl.nv[0], sl.nv[0], t, nt);
    }
    __syncthreads();
    const int n_lev = sl.n;
    auto grid_of = [&](int l) { VG g; g.nvx = d.nvx[l]; g.nvy = d.nvy[l]; g.nv = d.nv[l]; return g; };
    auto vec = [&](int l, int k) { return sh + d.o[l] + k * d.nv[l]; };   // 0 xa, 1 xb, 2 bv, 3 rv
    auto S_of = [&](int l) { return static_cast<const float *>(shf + d.os[l]); };
    // down: two pre-smoothing sweeps, residual, restriction
    for (int l = 0; l < n_lev - 1; ++l) {
        const VG g = grid_of(l);
        const float *S = S_of(l);
        const float *wd = S + 9 * g.nv;
        double *xa = vec(l, 0), *xb = vec(l, 1), *bv = vec(l, 2), *rv = vec(l, 3);
        for (long long v = t; v < g.nv; v += nt) xa[v] = wd[v] * bv[v];
        __syncthreads();
        for (long long v = t; v < g.nv; v += nt) {
            const int vx = (int)(v % g.nvx), vy = (int)(v / g.nvx);
            xb[v] = xa[v] + wd[v] * (bv[v] - stencil_apply(S, xa, g, vx, vy));
        }
        __syncthreads();
        for (long long v = t; v < g.nv; v += nt) {
            const int vx = (int)(v % g.nvx), vy = (int)(v / g.nvx);
            rv[v] = bv[v] - stencil_apply(S, xb, g, vx, vy);
        }
        __syncthreads();
        const VG gc = grid_of(l + 1);
        double *bc = vec(l + 1, 2);
        for (long long v = t; v < gc.nv; v += nt) {
            const int X = (int)(v % gc.nvx), Y = (int)(v / gc.nvx);
            double acc = 0.0;
            for (int dy = -1; dy <= 1; ++dy) {
                const int y = 2 * Y + dy;
                if (y < 0 || y >= g.nvy) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int x = 2 * X + dx;
                    if (x < 0 || x >= g.nvx) continue;
                    acc += (dx == 0 ? 1.0 : 0.5) * (dy == 0 ? 1.0 : 0.5) * rv[(long long)y * g.nvx + x];
                }
            }
            bc[v] = acc;
        }
        __syncthreads();
    }
    // coarsest from zero: the exact solve when the inverse exists, else damped Jacobi sweeps;
    // the result ends in xb
    {
        const int l = n_lev - 1;
        double *xa = vec(l, 0), *xb = vec(l, 1), *bv = vec(l, 2);
        if (cinv) {
            const int n = d.nv[l];
            const double *Ci = cinv + (size_t)b * n * n;
            for (int v = t; v < n; v += nt) {
                double acc = 0.0;
#pragma unroll 8
                for (int w = 0; w < n; ++w) acc += Ci[v * n + w] * bv[w];
                xb[v] = acc;
            }
            __syncthreads();
        } else {
            const VG g = grid_of(l);
            const float *S = S_of(l);
            const float *wd = S + 9 * g.nv;
            for (long long v = t; v < g.nv; v += nt) xb[v] = wd[v] * bv[v];
            __syncthreads();
            for (int k = 1; k < nsweep; ++k) {
                for (long long v = t; v < g.nv; v += nt) {
                    const int vx = (int)(v % g.nvx), vy = (int)(v / g.nvx);
                    xa[v] = xb[v] + wd[v] * (bv[v] - stencil_apply(S, xb, g, vx, vy));
                }
                __syncthreads();
                for (long long v = t; v < g.nv; v += nt) xb[v] = xa[v];
                __syncthreads();
            }
        }
    }
    // up: prolongation-correction, two post-smoothing sweeps (result in xb)
    for (int l = n_lev - 2; l >= 0; --l) {
        const VG g = grid_of(l), gc = grid_of(l + 1);
        const float *S = S_of(l);
        const float *wd = S + 9 * g.nv;
        double *xa = vec(l, 0), *xb = vec(l, 1), *bv = vec(l, 2);
        const double *c = vec(l + 1, 1);
        for (long long v = t; v < g.nv; v += nt) {
            const int x = (int)(v % g.nvx), y = (int)(v / g.nvx);
            const int X0 = x / 2, Y0 = y / 2;
            const int X1 = (x & 1) ? X0 + 1 : X0, Y1 = (y & 1) ? Y0 + 1 : Y0;
            xb[v] += 0.25 * (c[(long long)Y0 * gc.nvx + X0] + c[(long long)Y0 * gc.nvx + X1] +
                             c[(long long)Y1 * gc.nvx + X0] + c[(long long)Y1 * gc.nvx + X1]);
        }
        __syncthreads();
        for (long long v = t; v < g.nv; v += nt) {
            const int vx = (int)(v % g.nvx), vy = (int)(v / g.nvx);
            xa[v] = xb[v] + wd[v] * (bv[v] - stencil_apply(S, xb, g, vx, vy));
        }
        __syncthreads();
        for (long long v = t; v < g.nv; v += nt) {
            const int vx = (int)(v % g.nvx), vy = (int)(v / g.nvx);
            xb[v] = xa[v] + wd[v] * (bv[v] - stencil_apply(S, xa, g, vx, vy));
        }
        __syncthreads();
    }
    const double *x0 = vec(0, 1);
    for (long long v = t; v < sl.nv[0]; v += nt) x_top[(size_t)b * sl.nv[0] + v] = x0[v];
}

MipArgs mip_args(const rte_problem *p, int nblk) {
    MipArgs a;
    a.nx = p->nx;
    a.ny = p->ny;
    a.B = p->B;
    a.nblk = nblk;
    a.ncell = p->ncell;
    a.hx = p->hx;
    a.hy = p->hy;
    a.cxx = p->cxx;
    a.cyy = p->cyy;
    a.kx = p->kmin_x;
    a.ky = p->kmin_y;
    a.ihx = 1.0 / p->hx;
    a.ihy = 1.0 / p->hy;
    a.th_x = kS3 / (p->hx * p->hx);
    a.th_y = kS3 / (p->hy * p->hy);
    a.vol_x = 12.0 / (p->hx * p->hx);
    a.vol_y = 12.0 / (p->hy * p->hy);
    a.sigma_t = p->sigma_t;
    a.sigma_s = p->sigma_s;
    a.cf = nullptr;
    a.binv = nullptr;
    a.cf32 = nullptr;
    return a;
}
MipArgs mip_args(const rte_problem *p, const CGSpace &c) {
    MipArgs a = mip_args(p, c.nblk);
    a.cf = c.cf;
    a.binv = c.binv;
    a.cf32 = c.cf32;
    return a;
}

}  // namespace

int mg_levels(int nx, int ny, int *nvx, int *nvy) {
    // coarsen by two while both cell counts are even and the coarser grid keeps >= 2 cells
    if (nx < 2 || ny < 2) return 0;
    int L = 0, cx = nx, cy = ny;
    while (L < kMaxLevels) {
        if (nvx) nvx[L] = cx + 1;
        if (nvy) nvy[L] = cy + 1;
        ++L;
        if ((cx & 1) || (cy & 1) || cx < 4 || cy < 4) break;
        cx /= 2;
        cy /= 2;
    }
    return L;
}

namespace {
VG vg_of(const MGLevel &l) {
    VG g;
    g.nvx = l.nvx;
    g.nvy = l.nvy;
    g.nv = l.nv;
    return g;
}
constexpr int kCoarseSweeps = 30;
// damped Jacobi sweeps before and after the coarse correction on the vertex levels that run as
// separate launches (the LDS-resident small levels always use two)
constexpr int kVertexSweeps = 1;

// LDS bytes per vertex of a level held by the small-level kernel: 4 FP64 vectors and the
// FP32 stencil planes
constexpr long long kSmallBytesPerVertex = 4 * 8 + kStencilPlanes * 4;
constexpr long long kSmallLdsMax = 128 * 1024;

// first level whose V-cycle tail (it and all coarser levels) fits in the workgroup's LDS
int small_start(const rte_problem *p, const CGSpace &c) {
    const long long budget = std::min<long long>(kSmallLdsMax, p->lds_per_cu);
    long long tail = 0;
    int ls = c.mg.L;
    for (int l = c.mg.L - 1; l >= 0; --l) {
        tail += kSmallBytesPerVertex * c.mg.lv[l].nv;
        if (tail > budget) break;
        ls = l;
    }
    return ls;
}

// true when vcycle treats level l with the grid-wide kernels (neither the LDS small-level kernel
// nor the coarsest solve): such a level starts from x = omega b / diag in xb
bool vertex_grid_level(const rte_problem *p, const CGSpace &c, int l) {
    const int ls = small_start(p, c);
    if (l == ls && ls < c.mg.L) return false;
    return l != c.mg.L - 1;
}

// one V-cycle on level l for the right-hand side lv[l].bv; returns the buffer holding x_l
double *vcycle(const rte_problem *p, const CGSpace &c, int l, hipStream_t s) {
    const MGLevel &L = c.mg.lv[l];
    const VG g = vg_of(L);
    const dim3 grid(blocks_for(L.nv, 256), p->B);
    const int ls = small_start(p, c);
    if (l == ls && ls < c.mg.L) {
        SmallLevels sl;
        sl.n = c.mg.L - ls;
        long long lds = 0;
        for (int k = 0; k < sl.n; ++k) {
            const MGLevel &M = c.mg.lv[ls + k];
            sl.nvx[k] = M.nvx;
            sl.nvy[k] = M.nvy;
            sl.nv[k] = M.nv;
            sl.S[k] = M.S32;
            lds += kSmallBytesPerVertex * M.nv;
        }

        hipLaunchKernelGGL(mg_small_vcycle_kernel, dim3(p->B), dim3(1024), (size_t)lds, s, c.state,
                           sl, L.bv, L.xb, kCoarseSweeps, c.mg.cinv);
        return L.xb;
    }
    if (l == c.mg.L - 1) {
        if (L.nv <= 4096) {
            hipLaunchKernelGGL(mg_coarse_kernel, dim3(p->B), dim3(256), 2 * L.nv * sizeof(double), s,
                               c.state, g, L.S32, L.bv, L.xa, kCoarseSweeps, c.mg.cinv);
            return L.xa;
        }
        hipLaunchKernelGGL(mg_vertex_kernel<float>, grid, dim3(256), 0, s, c.state, g, L.S32, L.xa, L.bv, L.xa, 0);
        double *cur = L.xa, *nxt = L.xb;
        for (int k = 1; k < kCoarseSweeps; ++k) {
            hipLaunchKernelGGL(mg_vertex_kernel<float>, grid, dim3(256), 0, s, c.state, g, L.S32, cur, L.bv, nxt, 1);
            double *t = cur; cur = nxt; nxt = t;
        }
        return cur;
    }
    const MGLevel &C = c.mg.lv[l + 1];
    const VG gcv = vg_of(C);
    // pre-smoothing from zero (the first step, x = omega b / diag, was written into xb by the
    // kernel that formed b), residual, restriction
    if (kVertexSweeps == 2)
        hipLaunchKernelGGL(mg_vpre_kernel, grid, dim3(256), 0, s, c.state, g, L.S32, L.bv, L.xb);
    hipLaunchKernelGGL(mg_vertex_kernel<float>, grid, dim3(256), 0, s, c.state, g, L.S32, L.xb, L.bv, L.rv, 2);
    const bool x_first = vertex_grid_level(p, c, l + 1);
    hipLaunchKernelGGL(mg_vrestrict_kernel, dim3(blocks_for(C.nv, 256), p->B), dim3(256), 0, s,
                       c.state, g, L.rv, gcv, C.bv, C.S32, x_first ? C.xb : nullptr);
    double *xc = vcycle(p, c, l + 1, s);
    // coarse correction with the first post-smoothing sweep, then the second sweep
    hipLaunchKernelGGL(mg_vpost1_kernel, grid, dim3(256), 0, s, c.state, g, L.S32, L.bv, L.xb, gcv, xc, L.xa);
    if (kVertexSweeps == 1) return L.xa;
    hipLaunchKernelGGL(mg_vertex_kernel<float>, grid, dim3(256), 0, s, c.state, g, L.S32, L.xa, L.bv, L.xb, 1);
    return L.xb;
}
}  // namespace

hipError_t launch_dsa_build(const rte_problem *p, const CGSpace &c, const int *mask,
                            hipStream_t s) {
    const MipArgs a = mip_args(p, c);
    const int *all = mask;        // the selected instances (every instance if null)
    const dim3 gc(blocks_for(p->ncell, 256), p->B);
    hipLaunchKernelGGL(mip_prepare_kernel, gc, dim3(256), 0, s, a, mask, c.cf, c.binv, c.cf32);
    for (int l = 0; l < c.mg.L; ++l) {
        const MGLevel &L = c.mg.lv[l];
        const VG g = vg_of(L);
        const dim3 gv(blocks_for(L.nv, 256), p->B);
        if (l == 0) {
            // the DG operator seen through P: probed with the 9 vertex colours (coordinates
            // mod 3), whose 3 x 3 neighbourhoods hold one vertex of each colour
            hipLaunchKernelGGL(mg_zero_kernel, dim3(blocks_for(L.nv * kStencilPlanes, 256), p->B),
                               dim3(256), 0, s, all, L.nv * kStencilPlanes, L.S);
            for (int cy = 0; cy < 3; ++cy)
                for (int cx = 0; cx < 3; ++cx) {
                    hipLaunchKernelGGL(mg_colour_kernel, gv, dim3(256), 0, s, all, g, cx, cy, c.mg.e);
                    hipLaunchKernelGGL(mg_probe_dg_kernel, gc, dim3(256), 0, s, a, all, c.mg.e, g, c.mg.t);
                    hipLaunchKernelGGL(mg_restrict_dg_kernel<double>, gv, dim3(256), 0, s, a, all, c.mg.t, g, L.rv,
                                       nullptr, nullptr);
                    hipLaunchKernelGGL(mg_scatter_kernel, gv, dim3(256), 0, s, all, g, cx, cy, L.rv, L.S);
                }
        } else {
            const MGLevel &F = c.mg.lv[l - 1];
            hipLaunchKernelGGL(mg_galerkin_kernel, gv, dim3(256), 0, s, all, vg_of(F), F.S, g, L.S);
        }
        hipLaunchKernelGGL(mg_wdiag_kernel, gv, dim3(256), 0, s, all, g, L.S);
        hipLaunchKernelGGL(mg_round_kernel, dim3(blocks_for(L.nv * kStencilPlanes, 256), p->B),
                           dim3(256), 0, s, all, L.nv * kStencilPlanes, L.S, L.S32);
    }
    // LDS beyond 64 KiB for the small-level V-cycle (set here, outside any stream capture)
    if (c.mg.L > 0)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(mg_small_vcycle_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)std::min<long long>(kSmallLdsMax, p->lds_per_cu));
    if (c.mg.cinv) {
        const MGLevel &C = c.mg.lv[c.mg.L - 1];
        const size_t lds = (2 * (size_t)C.nv * C.nv + C.nv) * sizeof(double);
        hipLaunchKernelGGL(mg_coarse_invert_kernel, dim3(p->B), dim3(256), lds, s, all, vg_of(C),
                           C.S, c.mg.cinv);
    }
    return hipGetLastError();
}

namespace {
template <typename TZ>
hipError_t mg_precond_t(const rte_problem *p, const CGSpace &c, int slot_id, hipStream_t s) {
    const MipArgs a = mip_args(p, c);
    const dim3 gc(blocks_for(p->ncell, 256), p->B);
    const MGLevel &L0 = c.mg.lv[0];
    const VG g0 = vg_of(L0);
    TZ *z = reinterpret_cast<TZ *>(c.z);
    TZ *t = reinterpret_cast<TZ *>(c.mg.t);
    // z holds the pre-smoothed z = omega D^-1 r (written with r by the CG kernels);
    // residual t = r - A z and the coarse right-hand side P^T t
    const int ntx = (p->nx + kTile - 1) / kTile, nty = (p->ny + kTile - 1) / kTile;
    const bool tiled = (long long)ntx * nty == c.nblk && (long long)c.nblk == (long long)gc.x;
    if (tiled)
        hipLaunchKernelGGL(mg_resid_dg_tile_kernel<TZ>, gc, dim3(kCgBlock), 0, s, a, ntx, c.state,
                           c.r, z, t, c.part, c.tol2, c.n_running);
    else
        hipLaunchKernelGGL(mg_resid_dg_kernel<TZ>, gc, dim3(256), 0, s, a, c.state, c.r, z, t,
                           c.part, c.tol2, c.n_running);
    // a grid-wide level 0 gets its first smoothing step (into xb) with the restriction
    const bool x_first = vertex_grid_level(p, c, 0);
    hipLaunchKernelGGL(mg_restrict_dg_kernel<TZ>, dim3(blocks_for(L0.nv, 256), p->B), dim3(256),
                       0, s, a, c.state, t, g0, L0.bv, L0.S32, x_first ? L0.xb : nullptr);
    const double *x0 = vcycle(p, c, 0, s);
    // coarse correction and post-smoothing; the preconditioned residual goes to t
    if (tiled)
        hipLaunchKernelGGL(mg_post_dg_tile_kernel<TZ>, dim3(c.nblk, p->B), dim3(kCgBlock), 0, s, a,
                           ntx, c.state, c.r, x0, g0, z, t, c.part, slot_id);
    else
        hipLaunchKernelGGL(mg_post_dg_kernel<TZ>, dim3(c.nblk, p->B), dim3(kCgBlock), 0, s, a,
                           c.state, c.r, x0, g0, z, t, c.part, slot_id);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_mg_precond(const rte_problem *p, const CGSpace &c, int slot_id, hipStream_t s) {
    return c.zf32 ? mg_precond_t<float>(p, c, slot_id, s) : mg_precond_t<double>(p, c, slot_id, s);
}

size_t cg_blocks_per_instance(const rte_problem *p) {
    return (size_t)((p->ncell + kCgBlock - 1) / kCgBlock);
}

hipError_t launch_dsa1d(const rte_problem *p, const double *rho_star, const double *rho_prev,
                        double *delta, const int *kind, int want_kind, double *scratch,
                        hipStream_t s) {
    hipLaunchKernelGGL(dsa1d_kernel, dim3(blocks_for(p->B, 64)), dim3(64), 0, s, p->nx, p->B,
                       p->d_widths, p->sigma_t, p->sigma_s, p->c1, p->c2, p->c3, rho_star,
                       rho_prev, delta, kind, want_kind, scratch);
    return hipGetLastError();
}

hipError_t launch_cg_setup(const rte_problem *p, const CGSpace &c, const double *rho_star,
                           const double *rho_prev, const int *kind, int want_kind,
                           const double *guess, double rtol, hipStream_t s) {
    const MipArgs a = mip_args(p, c);
    hipLaunchKernelGGL(cg_begin_kernel, dim3(1), dim3(64), 0, s, c.n_running, c.tol2,
                       rtol * rtol);
    if (guess)
        hipLaunchKernelGGL(cg_warm_kernel, dim3(c.nblk, p->B), dim3(kCgBlock), 0, s, a, rho_star,
                           rho_prev, kind, want_kind, guess, c.r, c.q, c.part);
    // bj = 1: block-Jacobi preconditioner; bj = 2: first smoothing step of the multigrid one
    const int bj = c.mg.L == 0 ? 1 : 2;
    if (c.zf32)
        hipLaunchKernelGGL(cg_setup_kernel<float>, dim3(c.nblk, p->B), dim3(kCgBlock), 0, s, a,
                           rho_star, rho_prev, kind, want_kind, guess, c.q, c.x, c.r,
                           reinterpret_cast<float *>(c.z), c.part, c.state, c.iters, c.n_running,
                           bj);
    else
        hipLaunchKernelGGL(cg_setup_kernel<double>, dim3(c.nblk, p->B), dim3(kCgBlock), 0, s, a,
                           rho_star, rho_prev, kind, want_kind, guess, c.q, c.x, c.r, c.z, c.part,
                           c.state, c.iters, c.n_running, bj);
    if (bj == 2) {                                        // hierarchy built by launch_dsa_build
        if (c.precond[0]) return hipGraphLaunch(c.precond[0], s);
        return launch_mg_precond(p, c, 0, s);
    }
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const rte_problem *p, const CGSpace &c, int it, double rtol,
                               int maxit, hipStream_t s) {
    const MipArgs a = mip_args(p, c);
    double *p_new = (it & 1) ? c.p1 : c.p0;
    const double *p_old = (it & 1) ? c.p0 : c.p1;
    const double *z = c.mg.L == 0 ? c.z : c.mg.t;    // preconditioned residual
    const int bj = c.mg.L == 0 ? 1 : 2;
    const int ntx = (p->nx + kTile - 1) / kTile, nty = (p->ny + kTile - 1) / kTile;
    const bool tiled = (long long)ntx * nty == c.nblk;
    if (tiled && c.zf32)
        hipLaunchKernelGGL(cg_matvec_tile_kernel<float>, dim3(c.nblk, p->B), dim3(kCgBlock), 0, s,
                           a, ntx, it, rtol * rtol, maxit, reinterpret_cast<const float *>(z),
                           p_old, p_new, c.q, c.part, c.state, c.iters, c.n_running);
    else if (tiled)
        hipLaunchKernelGGL(cg_matvec_tile_kernel<double>, dim3(c.nblk, p->B), dim3(kCgBlock), 0,
                           s, a, ntx, it, rtol * rtol, maxit, z, p_old, p_new, c.q, c.part,
                           c.state, c.iters, c.n_running);
    if (c.zf32) {
        if (!tiled)
            hipLaunchKernelGGL(cg_matvec_kernel<float>, dim3(c.nblk, p->B), dim3(kCgBlock), 0, s,
                               a, it, rtol * rtol, maxit, reinterpret_cast<const float *>(z),
                               p_old, p_new, c.q, c.part, c.state, c.iters, c.n_running);
        hipLaunchKernelGGL(cg_update_kernel<float>, dim3(c.nblk, p->B), dim3(kCgBlock), 0, s, a,
                           it, p_new, c.q, c.x, c.r, reinterpret_cast<float *>(c.z), c.part,
                           c.state, c.iters, bj);
    } else {
        if (!tiled)
            hipLaunchKernelGGL(cg_matvec_kernel<double>, dim3(c.nblk, p->B), dim3(kCgBlock), 0, s,
                               a, it, rtol * rtol, maxit, z, p_old, p_new, c.q, c.part, c.state,
                               c.iters, c.n_running);
        hipLaunchKernelGGL(cg_update_kernel<double>, dim3(c.nblk, p->B), dim3(kCgBlock), 0, s, a,
                           it, p_new, c.q, c.x, c.r, c.z, c.part, c.state, c.iters, bj);
    }
    if (bj == 2) {
        if (c.precond[it & 1]) return hipGraphLaunch(c.precond[it & 1], s);
        return launch_mg_precond(p, c, it & 1, s);
    }
    return hipGetLastError();
}

void mg_precond_release(CGSpace &c) {
    for (int k = 0; k < 2; ++k) {
        if (c.precond[k]) (void)hipGraphExecDestroy(c.precond[k]);
        c.precond[k] = nullptr;
    }
}

void mg_precond_capture(const rte_problem *p, CGSpace &c) {
    mg_precond_release(c);
    if (c.mg.L == 0) return;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return;
    bool ok = true;
    for (int k = 0; k < 2 && ok; ++k) {
        hipGraph_t g = nullptr;
        ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        const hipError_t le = ok ? launch_mg_precond(p, c, k, cs) : hipSuccess;
        const hipError_t ce = ok ? hipStreamEndCapture(cs, &g) : hipErrorUnknown;
        ok = ok && le == hipSuccess && ce == hipSuccess && g;
        if (ok) ok = hipGraphInstantiate(&c.precond[k], g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
    }
    (void)hipStreamDestroy(cs);
    if (!ok) mg_precond_release(c);
    (void)hipGetLastError();
}

hipError_t launch_cg_finish(const rte_problem *p, const CGSpace &c, double *delta, int *iters_out,
                            unsigned long long *total, hipStream_t s) {
    // a CG that iterated in the output itself leaves only the statistics to gather
    const bool copy = c.x != delta;
    dim3 grid(copy ? blocks_for(p->ndof, 256) : 1u, p->B);
    hipLaunchKernelGGL(cg_finish_kernel, grid, dim3(256), 0, s, p->ndof, copy ? c.x : nullptr,
                       delta, c.state,
                       c.iters, iters_out, total, c.fails, p->B);
    return hipGetLastError();
}

}  // namespace rte
