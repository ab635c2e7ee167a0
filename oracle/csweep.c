/*
 * Oracle: plain FP64 transport sweeps (paper Sec. 2.3, eq. (transport_sweep)).
 *
 * Test infrastructure only -- never linked into the product library.
 *
 * For every direction j the block-lower-triangular system (D_j + Sigma_t) f_j = rhs
 * is solved cell by cell in upwind order (row by row, left-to-right for
 * v_x > 0 and right-to-left otherwise; bottom-to-top for v_y > 0).  Each cell
 * solves its small local system by Gaussian elimination with partial
 * pivoting.  The local operators (V: volume + outflow-edge terms, E: inflow
 * coupling to the upwind neighbour, b: unit boundary loads) are computed by
 * the caller from the weak form; this file only runs the loops.
 *
 * rho = sum_j w_j f_j (paper, definition under eq. (dg_matrix_vec)) is
 * accumulated in direction order.
 *
 * Built with -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Solve A x = b (n x n, row-major, copied) by Gaussian elimination with partial pivoting. */
static int gepp(int n, const double *A_in, const double *b_in, double *x)
{
    double A[16], b[4];
    memcpy(A, A_in, sizeof(double) * n * n);
    memcpy(b, b_in, sizeof(double) * n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(A[r * n + k]) > fabs(A[p * n + k])) p = r;
        if (A[p * n + k] == 0.0) return 1;
        if (p != k) {
            for (int c = 0; c < n; ++c) {
                double t = A[k * n + c]; A[k * n + c] = A[p * n + c]; A[p * n + c] = t;
            }
            double t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            double m = A[r * n + k] / A[k * n + k];
            for (int c = k; c < n; ++c) A[r * n + c] -= m * A[k * n + c];
            b[r] -= m * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int c = k + 1; c < n; ++c) s -= A[k * n + c] * x[c];
        x[k] = s / A[k * n + k];
    }
    return 0;
}

/*
 * Slab sweep.
 *   K    [nv][nc][2][2]  local matrices V_jc + (Sigma_t)_c
 *   E    [nv][nc][2][2]  coupling to the upwind neighbour's coefficients
 *   bl   [nv][2]         load of a unit inflow on the inflow boundary cell
 *   src  [nc][2]         isotropic right-hand side (Sigma_s rho + G)_c
 *   q    [nv][nc][2]     optional direction-dependent extra source (NULL = none)
 *   f    [nv][nc][2]     optional angular flux output (NULL = not stored)
 *   rho  [nc][2]         sum_j w_j f_j
 */
int oracle_sweep1d(int nc, int nv, const double *mu, const double *w, const double *K,
                   const double *E, const double *bl, const double *src, const double *q,
                   double g_left, double g_right, double *f, double *rho)
{
    double *cur = (double *)malloc(sizeof(double) * 2 * nc);
    if (!cur) return 2;
    memset(rho, 0, sizeof(double) * 2 * nc);
    for (int j = 0; j < nv; ++j) {
        int fwd = mu[j] > 0.0;
        for (int s = 0; s < nc; ++s) {
            int c = fwd ? s : nc - 1 - s;
            int up = fwd ? c - 1 : c + 1;
            double rhs[2];
            for (int k = 0; k < 2; ++k) {
                rhs[k] = src[2 * c + k];
                if (q) rhs[k] += q[((size_t)j * nc + c) * 2 + k];
            }
            const double *Ej = E + ((size_t)j * nc + c) * 4;
            if (up < 0 || up >= nc) {
                double g = fwd ? g_left : g_right;
                for (int k = 0; k < 2; ++k) rhs[k] += g * bl[2 * j + k];
            } else {
                for (int k = 0; k < 2; ++k)
                    for (int l = 0; l < 2; ++l) rhs[k] -= Ej[2 * k + l] * cur[2 * up + l];
            }
            if (gepp(2, K + ((size_t)j * nc + c) * 4, rhs, cur + 2 * c)) { free(cur); return 3; }
        }
        for (int c = 0; c < nc; ++c)
            for (int k = 0; k < 2; ++k) {
                rho[2 * c + k] += w[j] * cur[2 * c + k];
                if (f) f[((size_t)j * nc + c) * 2 + k] = cur[2 * c + k];
            }
    }
    free(cur);
    return 0;
}

/*
 * 2D sweep on a uniform nx x ny mesh (cell c = jj*nx + ii, local dof k = a + 2b).
 *   V, Ex, Ey [nv][4][4], bx, by [nv][4]   local operators (see oracle/dg.py)
 *   sigma_t [nc], src [nc][4], q [nv][nc][4] optional
 *   g [4]  isotropic inflow on the sides x=0, x=Lx, y=0, y=Ly
 *   f [nv][nc][4] optional, rho [nc][4]
 */
int oracle_sweep2d(int nx, int ny, int nv, const double *vx, const double *vy, const double *w,
                   const double *V, const double *Ex, const double *Ey, const double *bx,
                   const double *by, const double *sigma_t, const double *src, const double *q,
                   const double *g, double *f, double *rho)
{
    size_t ncell = (size_t)nx * ny;
    double *cur = (double *)malloc(sizeof(double) * 4 * ncell);
    if (!cur) return 2;
    memset(rho, 0, sizeof(double) * 4 * ncell);
    for (int j = 0; j < nv; ++j) {
        int px = vx[j] >= 0.0, py = vy[j] >= 0.0;
        const double *Vj = V + (size_t)j * 16, *Exj = Ex + (size_t)j * 16, *Eyj = Ey + (size_t)j * 16;
        for (int sj = 0; sj < ny; ++sj) {
            int jj = py ? sj : ny - 1 - sj;
            int ju = py ? jj - 1 : jj + 1;
            for (int si = 0; si < nx; ++si) {
                int ii = px ? si : nx - 1 - si;
                int iu = px ? ii - 1 : ii + 1;
                size_t c = (size_t)jj * nx + ii;
                double rhs[4], K[16];
                for (int k = 0; k < 4; ++k) {
                    rhs[k] = src[4 * c + k];
                    if (q) rhs[k] += q[((size_t)j * ncell + c) * 4 + k];
                }
                if (iu < 0 || iu >= nx) {
                    double gs = px ? g[0] : g[1];
                    for (int k = 0; k < 4; ++k) rhs[k] += gs * bx[4 * j + k];
                } else {
                    size_t u = (size_t)jj * nx + iu;
                    for (int k = 0; k < 4; ++k)
                        for (int l = 0; l < 4; ++l) rhs[k] -= Exj[4 * k + l] * cur[4 * u + l];
                }
                if (ju < 0 || ju >= ny) {
                    double gs = py ? g[2] : g[3];
                    for (int k = 0; k < 4; ++k) rhs[k] += gs * by[4 * j + k];
                } else {
                    size_t u = (size_t)ju * nx + ii;
                    for (int k = 0; k < 4; ++k)
                        for (int l = 0; l < 4; ++l) rhs[k] -= Eyj[4 * k + l] * cur[4 * u + l];
                }
                for (int k = 0; k < 16; ++k) K[k] = Vj[k];
                for (int k = 0; k < 4; ++k) K[5 * k] += sigma_t[c];
                if (gepp(4, K, rhs, cur + 4 * c)) { free(cur); return 3; }
            }
        }
        for (size_t c = 0; c < ncell; ++c)
            for (int k = 0; k < 4; ++k) {
                rho[4 * c + k] += w[j] * cur[4 * c + k];
                if (f) f[((size_t)j * ncell + c) * 4 + k] = cur[4 * c + k];
            }
    }
    free(cur);
    return 0;
}

/*
 * y_j = D_j x_j for every direction on the uniform 2D mesh (D_j of eq. (dg_matrix_vec):
 * own block V_j plus the coupling to interior upwind neighbours; no boundary load).
 *   x, y [nv][nc][4]
 */
void oracle_apply_D2d(int nx, int ny, int nv, const double *vx, const double *vy,
                      const double *V, const double *Ex, const double *Ey, const double *x,
                      double *y)
{
    size_t ncell = (size_t)nx * ny;
    for (int j = 0; j < nv; ++j) {
        int px = vx[j] >= 0.0, py = vy[j] >= 0.0;
        const double *xj = x + (size_t)j * ncell * 4;
        double *yj = y + (size_t)j * ncell * 4;
        for (int jj = 0; jj < ny; ++jj)
            for (int ii = 0; ii < nx; ++ii) {
                size_t c = (size_t)jj * nx + ii;
                int iu = px ? ii - 1 : ii + 1, ju = py ? jj - 1 : jj + 1;
                for (int k = 0; k < 4; ++k) {
                    double s = 0.0;
                    for (int l = 0; l < 4; ++l) s += V[(size_t)j * 16 + 4 * k + l] * xj[4 * c + l];
                    if (iu >= 0 && iu < nx)
                        for (int l = 0; l < 4; ++l)
                            s += Ex[(size_t)j * 16 + 4 * k + l] * xj[4 * ((size_t)jj * nx + iu) + l];
                    if (ju >= 0 && ju < ny)
                        for (int l = 0; l < 4; ++l)
                            s += Ey[(size_t)j * 16 + 4 * k + l] * xj[4 * ((size_t)ju * nx + ii) + l];
                    yj[4 * c + k] = s;
                }
            }
    }
}

/* y_j = D_j x_j for the slab (V, E as in oracle_sweep1d but V without Sigma_t). */
void oracle_apply_D1d(int nc, int nv, const double *mu, const double *V, const double *E,
                      const double *x, double *y)
{
    for (int j = 0; j < nv; ++j) {
        int fwd = mu[j] > 0.0;
        for (int c = 0; c < nc; ++c) {
            int up = fwd ? c - 1 : c + 1;
            for (int k = 0; k < 2; ++k) {
                double s = 0.0;
                for (int l = 0; l < 2; ++l)
                    s += V[((size_t)j * nc + c) * 4 + 2 * k + l] * x[((size_t)j * nc + c) * 2 + l];
                if (up >= 0 && up < nc)
                    for (int l = 0; l < 2; ++l)
                        s += E[((size_t)j * nc + c) * 4 + 2 * k + l] * x[((size_t)j * nc + up) * 2 + l];
                y[((size_t)j * nc + c) * 2 + k] = s;
            }
        }
    }
}
