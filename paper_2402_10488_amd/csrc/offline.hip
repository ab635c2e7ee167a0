// Offline construction of the correction ROM on the device (Sec. 3.1 POD, Sec. 3.2.1 snapshot
// generation, Sec. 3.1.1 reduced affine operators).
//
//   snapshot columns   delta f = f^mu - f^(mu,l)                         (f_gather_kernel)
//   Gram matrix        G = X^T Y over long columns, optionally restricted to one material class
//                      (v_mfma_f64_16x16x4f64, split over the rows, fixed-order split sum)
//   eigenpairs of G    cyclic Jacobi, one workgroup (the method of snapshots: F = U S V^T with
//                      F^T F = V S^2 V^T, U = F V S^-1)
//   QR route           shifted CholeskyQR3 of F from Gram matrices of F and of two transformed
//                      copies (chol_upper_kernel: R and R^-1 of a small SPD matrix), then a
//                      one-sided Jacobi SVD of the small triangular factor (svd_jacobi_kernel):
//                      singular values far below the largest keep their relative accuracy
//   basis weights      sorted singular values, the rank (fixed or by eq. (pod_truncation)) and
//                      W = V S^-1 of the kept columns (pod_weights_kernel, one workgroup)
//   basis              U = X W for a small W (v_mfma_f64_16x16x4f64)
//   reduced products   W^T G W, reduced inflow loads (small_gemm_kernel)
//   streaming operator y_j = D_j x_j of eq. (dg_matrix_vec) (upwind DG, no boundary load)
//   direction sums     sum_j w_j x_j (density of a basis vector) and sum_j x_j (isotropic
//                      projection), eq. (rho_basis)
#include <cmath>
#include <vector>

#include "rte_internal.h"

namespace rte {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr double kS3 = 1.7320508075688772935;

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// Direction-major, natural-order copy of an angular flux in the sweep's layout (2D:
// [B][n_dir][cell][K] with each direction's cells in band order of its reflected coordinates; 1D:
// [B][cell][n_dir][K]), optionally minus a second one: out[b * stride + (j * ncell + cell) * K + k].
// In 2D a thread owns one stored position, so the reads of a wavefront are contiguous.
template <typename T, typename TO>
__global__ void f_gather_kernel(int dim, int nx, int ny, long long ncell, int K, int n_dir,
                                const double *vxy, const T *fa, const T *fb, TO *out,
                                long long stride) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= (long long)n_dir * ncell) return;
    const long long j = t / ncell, e = t - j * ncell;
    long long cell;
    size_t src;
    if (dim == 2) {
        const int q = (vxy[j] < 0.0 ? 1 : 0) | (vxy[n_dir + j] < 0.0 ? 2 : 0);
        cell = unreflect(nx, ny, band_cell(nx, ny, (int)e), q);
        src = (((size_t)b * n_dir + j) * ncell + e) * K;
    } else {
        cell = e;
        src = (((size_t)b * ncell + e) * n_dir + j) * K;
    }
    TO *o = out + (size_t)b * stride + ((size_t)j * ncell + cell) * K;
    for (int k = 0; k < K; ++k) o[k] = (TO)(fb ? fa[src + k] - fb[src + k] : fa[src + k]);
}

// G_part[split][i][j] = sum over rows in the split of X[i][row] Y[j][row] (row in class cls);
// FP32 inputs are widened to FP64 before the FP64 matrix-core product
template <typename TX, typename TY>
__global__ void __launch_bounds__(64) gram_kernel(const TX *X, int nxc, const TY *Y,
                                                  int nyc, long long len, long long per_split,
                                                  const int *cell_class, int K, long long ncell,
                                                  int cls, double *part) {
    const int lane = threadIdx.x;
    const int split = blockIdx.x, ti = blockIdx.y, tj = blockIdx.z;
    const int n = lane & 15, kq = lane >> 4;
    const int ci = ti * 16 + n, cj = tj * 16 + n;
    const bool li = ci < nxc, lj = cj < nyc;
    const long long k_begin = (long long)split * per_split;
    long long k_end = k_begin + per_split;
    if (k_end > len) k_end = len;
    v4d acc = {0, 0, 0, 0};
    for (long long k0 = k_begin; k0 < k_end; k0 += 16) {
        double av[4], bv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const long long k = k0 + 4 * kq + s;
            bool in = k < k_end;
            if (in && cell_class) in = cell_class[(k / K) % ncell] == cls;
            av[s] = (in && li) ? (double)X[(size_t)ci * len + k] : 0.0;
            bv[s] = (in && lj) ? (double)Y[(size_t)cj * len + k] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gi = ti * 16 + kq + 4 * i, gj = tj * 16 + n;   // D row = q + 4 i (f64)
        if (gi < nxc && gj < nyc) part[((size_t)split * nxc + gi) * nyc + gj] = acc[i];
    }
}

__global__ void sum_splits_kernel(const double *part, int nsplit, long long n, double *out) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(size_t)k * n + t];
    out[t] = s;
}

// Cyclic Jacobi for a symmetric n x n matrix (n <= 256) in global memory, one workgroup.
// Parallel ordering: in every round the n (padded to even) indices are paired by the
// round-robin tournament, the n/2 rotations are independent.  On exit A is diagonal
// (eigenvalues), V holds the eigenvectors as columns.
__global__ void __launch_bounds__(256) jacobi_kernel(double *A, int n, double *V, double *evals,
                                                     int sweeps) {
    __shared__ double cs[128], sn[128];
    __shared__ int pp[128], qq[128];
    __shared__ double off_s[256];
    const int t = threadIdx.x;
    const int m = n + (n & 1);           // padded size (dummy index m-1 when n is odd)
    for (int i = t; i < n * n; i += blockDim.x) V[i] = (i / n == i % n) ? 1.0 : 0.0;
    __syncthreads();
    for (int sw = 0; sw < sweeps; ++sw) {
        // convergence: off-diagonal norm vs diagonal norm
        double o = 0.0, d = 0.0;
        for (int i = t; i < n * n; i += blockDim.x) {
            const double v = A[i];
            if (i / n == i % n) d += v * v; else o += v * v;
        }
        off_s[t] = o;
        __syncthreads();
        if (t == 0) {
            double so = 0.0;
            for (int k = 0; k < (int)blockDim.x; ++k) so += off_s[k];
            off_s[0] = so;
        }
        __syncthreads();
        const double offn = off_s[0];
        __syncthreads();
        off_s[t] = d;
        __syncthreads();
        if (t == 0) {
            double sd = 0.0;
            for (int k = 0; k < (int)blockDim.x; ++k) sd += off_s[k];
            off_s[1] = sd;
        }
        __syncthreads();
        const double dn = off_s[1];
        __syncthreads();
        if (offn <= 1e-30 * dn || offn == 0.0) break;
        for (int round = 0; round < m - 1; ++round) {
            // pairs of the round-robin tournament: fixed element m-1, the others rotate
            if (t < m / 2) {
                int a, b;
                if (t == 0) { a = m - 1; b = round; }
                else {
                    a = (round + t) % (m - 1);
                    b = (round - t + (m - 1)) % (m - 1);
                }
                int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[p * n + q];
                    if (apq != 0.0) {
                        const double app = A[p * n + p], aqq = A[q * n + q];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                pp[t] = p; qq[t] = q < n ? q : p; cs[t] = c; sn[t] = (q < n) ? s : 0.0;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int idx = t; idx < (m / 2) * n; idx += blockDim.x) {
                const int k = idx / n, col = idx % n;
                const int p = pp[k], q = qq[k];
                if (p == q) continue;
                const double c = cs[k], s = sn[k];
                const double ap = A[p * n + col], aq = A[q * n + col];
                A[p * n + col] = c * ap - s * aq;
                A[q * n + col] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int idx = t; idx < (m / 2) * n; idx += blockDim.x) {
                const int k = idx / n, row = idx % n;
                const int p = pp[k], q = qq[k];
                if (p == q) continue;
                const double c = cs[k], s = sn[k];
                const double ap = A[row * n + p], aq = A[row * n + q];
                A[row * n + p] = c * ap - s * aq;
                A[row * n + q] = s * ap + c * aq;
                const double vp = V[row * n + p], vq = V[row * n + q];
                V[row * n + p] = c * vp - s * vq;
                V[row * n + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    for (int i = t; i < n; i += blockDim.x) evals[i] = A[i * n + i];
}

// out[c][row] = sum_col W[col][c] X[col][row]; one wave per (16 rows x 16 outputs) tile.
__global__ void __launch_bounds__(64) combine_kernel(const double *X, int ncol, long long len,
                                                     const double *W, int r, double *out) {
    const int lane = threadIdx.x;
    const int n = lane & 15, kq = lane >> 4;
    const long long m0 = (long long)blockIdx.x * 16;
    const int c0 = blockIdx.y * 16;
    v4d acc = {0, 0, 0, 0};
    const int kpad = (ncol + 3) & ~3;
    for (int k0 = 0; k0 < kpad; k0 += 4) {
        const int kk = k0 + kq;
        const long long row = m0 + n;
        const double a = (kk < ncol && row < len) ? X[(size_t)kk * len + row] : 0.0;
        const double b = (kk < ncol && c0 + n < r) ? W[(size_t)kk * r + c0 + n] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const long long row = m0 + kq + 4 * i;
        const int c = c0 + n;
        if (row < len && c < r) out[(size_t)c * len + row] = acc[i];
    }
}

// y_j = D_j x_j for every vector and direction (upwind DG streaming operator, no boundary load),
// in the reflected coordinates of the direction's quadrant: D = a (A (x) I) + b (I (x) A) minus
// the inflow coupling to the upwind neighbours' outgoing traces.
template <typename TX>
__global__ void apply_streaming_kernel(int nx, int ny, int n_dir, int nvec, const double *vx,
                                       const double *vy, double hx, double hy, const TX *x,
                                       double *y) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long ncell = (long long)nx * ny;
    const long long tot = (long long)nvec * n_dir * ncell;
    if (t >= tot) return;
    const long long cell = t % ncell;
    const long long vj = t / ncell;                  // vector * n_dir + direction
    const int j = (int)(vj % n_dir);
    const int ix = (int)(cell % nx), iy = (int)(cell / nx);
    const double sx = vx[j] < 0 ? -1.0 : 1.0, sy = vy[j] < 0 ? -1.0 : 1.0;
    const double a = fabs(vx[j]) / hx, b = fabs(vy[j]) / hy, c = kS3;
    const TX *xv = x + (size_t)vj * ncell * 4;
    auto load = [&](long long cc, double f[4]) {
        const TX *e = xv + cc * 4;
        f[0] = (double)e[0]; f[1] = sx * (double)e[1]; f[2] = sy * (double)e[2];
        f[3] = sx * sy * (double)e[3];                                          // reflected
    };
    double f[4];
    load(cell, f);
    // a (A (x) I) f + b (I (x) A) f, A = [[1, c], [-c, 3]], dof k = a + 2 b
    double o[4];
    o[0] = a * (f[0] + c * f[1]) + b * (f[0] + c * f[2]);
    o[1] = a * (-c * f[0] + 3.0 * f[1]) + b * (f[1] + c * f[3]);
    o[2] = a * (f[2] + c * f[3]) + b * (-c * f[0] + 3.0 * f[2]);
    o[3] = a * (-c * f[2] + 3.0 * f[3]) + b * (-c * f[1] + 3.0 * f[3]);
    // inflow coupling from the upwind neighbours (interior only)
    const int ux = ix - (int)sx, uy = iy - (int)sy;
    if (ux >= 0 && ux < nx) {
        double g[4];
        load((long long)iy * nx + ux, g);
        const double T0 = g[0] + c * g[1], T1 = g[2] + c * g[3];     // traces at its + face
        o[0] -= a * T0; o[1] += a * c * T0; o[2] -= a * T1; o[3] += a * c * T1;
    }
    if (uy >= 0 && uy < ny) {
        double g[4];
        load((long long)uy * nx + ix, g);
        const double T0 = g[0] + c * g[2], T1 = g[1] + c * g[3];
        o[0] -= b * T0; o[2] += b * c * T0; o[1] -= b * T1; o[3] += b * c * T1;
    }
    double4 r;
    r.x = o[0]; r.y = sx * o[1]; r.z = sy * o[2]; r.w = sx * sy * o[3];
    *reinterpret_cast<double4 *>(y + (size_t)vj * ncell * 4 + cell * 4) = r;
}

template <typename TX>
__global__ void direction_sum_kernel(long long ndof, int n_dir, int nvec, const double *w,
                                     const TX *x, double *out) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (t >= ndof) return;
    const TX *xv = x + (size_t)v * n_dir * ndof + t;
    double s = 0.0;
    for (int j = 0; j < n_dir; ++j) s += (w ? w[j] : 1.0) * (double)xv[(size_t)j * ndof];
    out[(size_t)v * ndof + t] = s;
}

// out[side][v] = sum_j sum_{cells on the side} U[v][j][cell] . load_j: the load of a unit
// isotropic inflow on a side (eq. (dg_matrix_vec)) enters the cells next to it for the
// directions entering there, |v.n| g (h_t / sqrt(hx hy)) L_a(-+1) on the face-normal index a
// (tangential index 0), h_t the face length.  One workgroup per (vector, side), fixed-order sum.
template <typename TU>
__global__ void __launch_bounds__(256) inflow_load_kernel(int nx, int ny, long long ndof, int n_dir,
                                                         const double *vxy, double hx, double hy,
                                                         const TU *U, int nvec, double *out) {
    const int v = blockIdx.x, side = blockIdx.y;
    const bool xs = side < 2;                      // x = 0 / x = Lx faces
    const int nface = xs ? ny : nx;                // cells along the side
    const double scale = xs ? sqrt(hy / hx) : sqrt(hx / hy);
    const double s3 = kS3;
    double acc = 0.0;
    for (long long t = threadIdx.x; t < (long long)n_dir * nface; t += blockDim.x) {
        const int j = (int)(t / nface), m = (int)(t - (long long)j * nface);
        const double vn = xs ? vxy[j] : vxy[n_dir + j];
        const bool enters = (side == 0 || side == 2) ? vn > 0.0 : vn < 0.0;
        if (!enters) continue;
        int cell;
        if (side == 0) cell = m * nx;
        else if (side == 1) cell = m * nx + nx - 1;
        else if (side == 2) cell = m;
        else cell = (ny - 1) * nx + m;
        // trace of the face-normal Legendre index on the face: -sqrt(3) at the low, +sqrt(3) at
        // the high face of the cell (dof 1 for x faces, dof 2 for y faces)
        const double tr = (side == 0 || side == 2) ? -s3 : s3;
        const TU *u = U + ((size_t)v * n_dir + j) * ndof + (size_t)cell * 4;
        acc += fabs(vn) * scale * ((double)u[0] + tr * (double)(xs ? u[1] : u[2]));
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[side * nvec + v] = sh[0];
}

}  // namespace
}  // namespace rte

using namespace rte;

namespace rte {
namespace {

// POD of the method of snapshots (Sec. 3.1): eigenpairs (lambda_i, v_i) of F^T F give the
// singular values sigma = sqrt(lambda) and the basis U = F V Sigma^-1.  One workgroup of up to
// 256 threads: thread i ranks eigenvalue i (descending, ties by index, as a stable sort), the rank
// and its truncation are chosen by thread 0, and thread i writes row i of W = V Sigma^-1 for the
// kept columns (W [ncol][ncol], leading dimension ncol).
__global__ void __launch_bounds__(256) pod_weights_kernel(const double *evals, const double *evecs,
                                                          int ncol, int r_fixed, double eps_pod,
                                                          double *sv, double *W, int *r_out,
                                                          double *eps_out) {
    __shared__ double lam[256];
    __shared__ double svs[256];
    __shared__ int order[256];
    __shared__ int r_sh;
    const int i = threadIdx.x;
    if (i < ncol) lam[i] = evals[i];
    __syncthreads();
    if (i < ncol) {
        int rank = 0;
        for (int j = 0; j < ncol; ++j)
            rank += (lam[j] > lam[i]) || (lam[j] == lam[i] && j < i);
        order[rank] = i;
        svs[rank] = sqrt(lam[i] > 0.0 ? lam[i] : 0.0);
    }
    __syncthreads();
    if (i == 0) {
        double total = 0.0;
        for (int k = 0; k < ncol; ++k) total += svs[k];
        int r = ncol;
        if (r_fixed > 0) {
            r = r_fixed < ncol ? r_fixed : ncol;
        } else {                                  // eq. (pod_truncation): sum ratio >= 1 - eps
            double acc = 0.0;
            for (int k = 0; k < ncol; ++k) {
                acc += svs[k];
                if (acc / total >= 1.0 - eps_pod) { r = k + 1; break; }
            }
        }
        int nz = 0;                               // singular values above rounding of the largest
        for (int k = 0; k < ncol; ++k) nz += svs[k] > svs[0] * 1e-13;
        if (r > nz) r = nz > 0 ? nz : 1;
        double kept = 0.0;
        for (int k = 0; k < r; ++k) kept += svs[k];
        const double drop = total > 0.0 ? 1.0 - kept / total : 0.0;
        *r_out = r;
        *eps_out = drop > 0.0 ? drop : 0.0;
        r_sh = r;
    }
    __syncthreads();
    if (i < ncol) {
        sv[i] = svs[i];
        const int r = r_sh;
        for (int k = 0; k < r; ++k) W[(size_t)i * ncol + k] = evecs[(size_t)i * ncol + order[k]] / svs[k];
    }
}

// Cholesky factor of a small SPD matrix, G + shift I = R^T R (R upper triangular, n <= 256), and
// T = R^-1, one workgroup.  W (n x n scratch) receives G + shift I and is overwritten by the
// right-looking elimination.  With shifted != 0 the shift is 11 (m n + n (n + 1)) u trace(G)
// (u the FP64 unit roundoff): the shift of shifted CholeskyQR, which keeps the factorization of
// the Gram matrix of an m x n matrix defined for condition numbers up to about 1/u.  A pivot that
// is not positive leaves info = its index + 1 (else 0) and stops.  dev (optional) receives
// max |G_ij - delta_ij|, how far the factored columns are from orthonormal.
__global__ void __launch_bounds__(256) chol_upper_kernel(const double *G, int n, int shifted,
                                                         long long m, double *W, double *R,
                                                         double *T, int *info, double *dev) {
    __shared__ double piv;
    __shared__ double tr_part[256], dv_part[256];
    __shared__ int bad;
    const int t = threadIdx.x;
    double tr = 0.0, dv = 0.0;
    for (int i = t; i < n; i += blockDim.x) tr += G[(size_t)i * n + i];
    for (int i = t; i < n * n; i += blockDim.x)
        dv = fmax(dv, fabs(G[i] - (i / n == i % n ? 1.0 : 0.0)));
    tr_part[t] = tr;
    dv_part[t] = dv;
    if (t == 0) bad = 0;
    __syncthreads();
    if (t == 0) {
        double s = 0.0, d = 0.0;
        for (int k = 0; k < (int)blockDim.x; ++k) { s += tr_part[k]; d = fmax(d, dv_part[k]); }
        tr_part[0] = s;
        if (dev) *dev = d;
    }
    __syncthreads();
    const double u = 0.5 * 2.220446049250313e-16;
    const double shift = shifted ? 11.0 * ((double)m * n + (double)n * (n + 1)) * u * tr_part[0] : 0.0;
    for (int i = t; i < n * n; i += blockDim.x) {
        const int r = i / n, c = i % n;
        W[i] = G[i] + (r == c ? shift : 0.0);
        R[i] = 0.0;
        T[i] = 0.0;
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (t == 0) {
            const double d = W[(size_t)j * n + j];
            if (!(d > 0.0)) {
                bad = j + 1;
                piv = 1.0;
            } else {
                piv = sqrt(d);
            }
            R[(size_t)j * n + j] = piv;
        }
        __syncthreads();
        if (bad) break;
        const double rjj = piv;
        for (int i = j + 1 + t; i < n; i += blockDim.x) R[(size_t)j * n + i] = W[(size_t)j * n + i] / rjj;
        __syncthreads();
        // trailing update of the upper triangle: W[i][k] -= R[j][i] R[j][k], j < i <= k
        const int nt = n - j - 1;
        for (int idx = t; idx < nt * nt; idx += blockDim.x) {
            const int i = j + 1 + idx / nt, k = j + 1 + idx % nt;
            if (k >= i) W[(size_t)i * n + k] -= R[(size_t)j * n + i] * R[(size_t)j * n + k];
        }
        __syncthreads();
    }
    if (t == 0) *info = bad;
    if (bad) return;
    // T = R^-1 column by column (back substitution), one thread per column
    for (int c = t; c < n; c += blockDim.x) {
        T[(size_t)c * n + c] = 1.0 / R[(size_t)c * n + c];
        for (int i = c - 1; i >= 0; --i) {
            double acc = 0.0;
            for (int k = i + 1; k <= c; ++k) acc += R[(size_t)i * n + k] * T[(size_t)k * n + c];
            T[(size_t)i * n + c] = -acc / R[(size_t)i * n + i];
        }
    }
}

// One-sided (Hestenes) Jacobi SVD of a small n x n matrix A (n <= 256), one workgroup of four
// waves.  Columns are stored transposed (At[col][row]) so that each column is contiguous; pairs of
// columns are orthogonalized by plane rotations applied from the right, A J and V J, in the
// round-robin order of the tournament (n/2 disjoint pairs per round, one wave per pair, rounds
// separated by barriers), until a sweep applies no rotation (|a_p . a_q| <= 1e-15 |a_p| |a_q| for
// every pair) or after max_sweeps.  Then A V = U S with orthogonal columns: lam[k] = |A v_k|^2 =
// s_k^2 (unsorted), V[i][k] = v_k[i] (right singular vectors as columns) and, if US is given,
// US[i][k] = (A v_k)[i] = s_k u_k[i].  Each s_k comes with a small relative error, also for
// singular values far below the largest.
__global__ void __launch_bounds__(256) svd_jacobi_kernel(const double *A, int n, double *At,
                                                         double *Vt, double *lam, double *V,
                                                         double *US, int max_sweeps,
                                                         int *sweeps_out) {
    __shared__ int rotated;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6, nw = (int)blockDim.x >> 6;
    const int m = n + (n & 1);                  // padded size (dummy column m-1 when n is odd)
    for (int i = t; i < n * n; i += blockDim.x) {
        const int r = i / n, c = i % n;
        At[(size_t)c * n + r] = A[i];
        Vt[i] = (r == c) ? 1.0 : 0.0;
    }
    int sw = 0;
    for (; sw < max_sweeps; ++sw) {
        if (t == 0) rotated = 0;
        __syncthreads();
        for (int round = 0; round < m - 1; ++round) {
            for (int k = wave; k < m / 2; k += nw) {
                int a, b;
                if (k == 0) { a = m - 1; b = round; }
                else {
                    a = (round + k) % (m - 1);
                    b = (round - k + (m - 1)) % (m - 1);
                }
                const int p = a < b ? a : b, q = a < b ? b : a;
                if (q >= n) continue;                    // the dummy column
                double *cp = At + (size_t)p * n, *cq = At + (size_t)q * n;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = lane; i < n; i += 64) {
                    const double x = cp[i], y = cq[i];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                for (int off = 32; off > 0; off >>= 1) {
                    al += __shfl_xor(al, off, 64);
                    be += __shfl_xor(be, off, 64);
                    ga += __shfl_xor(ga, off, 64);
                }
                if (!(fabs(ga) > 1e-15 * sqrt(al * be))) continue;   // wave-uniform
                const double zeta = (be - al) / (2.0 * ga);
                const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
                for (int i = lane; i < n; i += 64) {
                    const double x = cp[i], y = cq[i];
                    cp[i] = c * x - s * y;
                    cq[i] = s * x + c * y;
                }
                double *vp = Vt + (size_t)p * n, *vq = Vt + (size_t)q * n;
                for (int i = lane; i < n; i += 64) {
                    const double x = vp[i], y = vq[i];
                    vp[i] = c * x - s * y;
                    vq[i] = s * x + c * y;
                }
                if (lane == 0) rotated = 1;
            }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }
    for (int k = wave; k < n; k += nw) {
        double s2 = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double x = At[(size_t)k * n + i];
            s2 += x * x;
        }
        for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
        if (lane == 0) lam[k] = s2;
    }
    for (int i = t; i < n * n; i += blockDim.x) {
        const int r = i / n, c = i % n;
        V[i] = Vt[(size_t)c * n + r];
        if (US) US[i] = At[(size_t)c * n + r];
    }
    if (t == 0) *sweeps_out = sw;
}

// C[m][n] = alpha op(A)[m][k] B[k][n] (B null: the k x n identity, so C = alpha op(A)); op(A) = A
// [m][k] or, transposed, A [k][m]; row-major FP64, one thread per entry, for the reduced (r x r,
// ncol x r) products of the offline ROM construction.
__global__ void small_gemm_kernel(int trans_a, int m, int n, int k, double alpha, const double *A,
                                  const double *B, double *C) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)m * n) return;
    const int row = (int)(t / n), col = (int)(t - (long long)row * n);
    double s = 0.0;
    if (B) {
        for (int q = 0; q < k; ++q) {
            const double a = trans_a ? A[(size_t)q * m + row] : A[(size_t)row * k + q];
            s += a * B[(size_t)q * n + col];
        }
    } else {
        s = trans_a ? A[(size_t)col * m + row] : A[(size_t)row * k + col];
    }
    C[t] = alpha * s;
}

}  // namespace
}  // namespace rte

extern "C" {

int rte_pod_snapshots(const rte_problem *p, const double *f_final, const double *f_iter,
                      void *cols, long long stride, rte_precision cols_prec, rte_stream_t stream) {
    if (!p || !f_final || !cols) return RTE_EINVAL;
    if (cols_prec != RTE_FP64 && cols_prec != RTE_MIXED) return RTE_EINVAL;
    const long long len = (long long)p->n_dir * p->ndof;
    if (stride < len) return RTE_EINVAL;
    const dim3 grid(cdiv((long long)p->n_dir * p->ncell, 256), p->B);
    hipStream_t s = (hipStream_t)stream;
    if (cols_prec == RTE_MIXED)
        hipLaunchKernelGGL((f_gather_kernel<double, float>), grid, dim3(256), 0, s, p->dim, p->nx,
                           p->ny, p->ncell, p->K, p->n_dir, p->d_vxy, f_final, f_iter, (float *)cols,
                           stride);
    else
        hipLaunchKernelGGL((f_gather_kernel<double, double>), grid, dim3(256), 0, s, p->dim, p->nx,
                           p->ny, p->ncell, p->K, p->n_dir, p->d_vxy, f_final, f_iter,
                           (double *)cols, stride);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_f_natural(const rte_problem *p, const void *f, void *out, rte_precision prec,
                  rte_stream_t stream) {
    if (!p || !f || !out) return RTE_EINVAL;
    if (prec != RTE_FP64 && prec != RTE_MIXED) return RTE_EINVAL;
    const dim3 grid(cdiv((long long)p->n_dir * p->ncell, 256), p->B);
    const long long stride = (long long)p->n_dir * p->ndof;
    hipStream_t s = (hipStream_t)stream;
    if (prec == RTE_MIXED)
        hipLaunchKernelGGL((f_gather_kernel<float, float>), grid, dim3(256), 0, s, p->dim, p->nx,
                           p->ny, p->ncell, p->K, p->n_dir, p->d_vxy, (const float *)f,
                           (const float *)nullptr, (float *)out, stride);
    else
        hipLaunchKernelGGL((f_gather_kernel<double, double>), grid, dim3(256), 0, s, p->dim, p->nx,
                           p->ny, p->ncell, p->K, p->n_dir, p->d_vxy, (const double *)f,
                           (const double *)nullptr, (double *)out, stride);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_gram(const void *X, rte_precision xprec, int nxc, const void *Y, rte_precision yprec,
             int nyc, long long len, const int *cell_class, int K, long long ncell, int cls,
             double *G, void *ws, size_t ws_bytes, rte_stream_t stream) {
    if (!X || !Y || !G || nxc < 1 || nyc < 1 || len < 1 || !ws) return RTE_EINVAL;
    if ((xprec != RTE_FP64 && xprec != RTE_MIXED) || (yprec != RTE_FP64 && yprec != RTE_MIXED))
        return RTE_EINVAL;
    if (cell_class && (K < 1 || ncell < 1)) return RTE_EINVAL;
    const long long tiles = (long long)cdiv(nxc, 16) * cdiv(nyc, 16);
    long long nsplit = (4096 + tiles - 1) / tiles;
    const long long maxs = (len + 4095) / 4096;
    if (nsplit > maxs) nsplit = maxs;
    if (nsplit < 1) nsplit = 1;
    while ((size_t)nsplit * nxc * nyc * 8 > ws_bytes && nsplit > 1) nsplit /= 2;
    if ((size_t)nsplit * nxc * nyc * 8 > ws_bytes) return RTE_ENOMEM;
    long long per = (len + nsplit - 1) / nsplit;
    per = (per + 15) / 16 * 16;
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid((unsigned)nsplit, cdiv(nxc, 16), cdiv(nyc, 16));
    double *part = (double *)ws;
    const bool xf = xprec == RTE_MIXED, yf = yprec == RTE_MIXED;
    if (xf && yf)
        hipLaunchKernelGGL((gram_kernel<float, float>), grid, dim3(64), 0, s, (const float *)X, nxc,
                           (const float *)Y, nyc, len, per, cell_class, K, ncell, cls, part);
    else if (xf)
        hipLaunchKernelGGL((gram_kernel<float, double>), grid, dim3(64), 0, s, (const float *)X, nxc,
                           (const double *)Y, nyc, len, per, cell_class, K, ncell, cls, part);
    else if (yf)
        hipLaunchKernelGGL((gram_kernel<double, float>), grid, dim3(64), 0, s, (const double *)X,
                           nxc, (const float *)Y, nyc, len, per, cell_class, K, ncell, cls, part);
    else
        hipLaunchKernelGGL((gram_kernel<double, double>), grid, dim3(64), 0, s, (const double *)X,
                           nxc, (const double *)Y, nyc, len, per, cell_class, K, ncell, cls, part);
    const long long n = (long long)nxc * nyc;
    hipLaunchKernelGGL(sum_splits_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, (const double *)ws,
                       (int)nsplit, n, G);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_sym_eig(double *A, int n, double *evals, double *evecs, rte_stream_t stream) {
    if (!A || !evals || !evecs || n < 1 || n > 256) return RTE_EINVAL;
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, A, n, evecs,
                       evals, 30);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_pod_weights(const double *evals, const double *evecs, int ncol, int r, double eps_pod,
                    double *sv, double *W, int *r_out, double *eps_out, rte_stream_t stream) {
    if (!evals || !evecs || !sv || !W || !r_out || !eps_out || ncol < 1 || ncol > 256 || r < 0)
        return RTE_EINVAL;
    if (r == 0 && !(eps_pod >= 0.0 && eps_pod < 1.0)) return RTE_EINVAL;
    hipLaunchKernelGGL(rte::pod_weights_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, evals,
                       evecs, ncol, r, eps_pod, sv, W, r_out, eps_out);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_chol_upper(const double *G, int n, int shifted, long long m, double *work, double *R,
                   double *T, int *info, double *dev, rte_stream_t stream) {
    if (!G || !work || !R || !T || !info || n < 1 || n > 256 || (shifted && m < 1))
        return RTE_EINVAL;
    hipLaunchKernelGGL(rte::chol_upper_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, G, n,
                       shifted, m, work, R, T, info, dev);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_svd_jacobi(const double *A, int n, double *work, double *lam, double *V, double *US,
                   int max_sweeps, int *sweeps_out, rte_stream_t stream) {
    if (!A || !work || !lam || !V || !sweeps_out || n < 1 || n > 256 || max_sweeps < 1)
        return RTE_EINVAL;
    hipLaunchKernelGGL(rte::svd_jacobi_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, A, n,
                       work, work + (size_t)n * n, lam, V, US, max_sweeps, sweeps_out);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_small_gemm(int trans_a, int m, int n, int k, double alpha, const double *A, const double *B,
                   double *C, rte_stream_t stream) {
    if (!A || !C || m < 1 || n < 1 || k < 1 || (trans_a != 0 && trans_a != 1)) return RTE_EINVAL;
    if (!B && k != n) return RTE_EINVAL;
    if ((long long)m * n > (1LL << 26) || (long long)k > (1LL << 20)) return RTE_EUNSUPPORTED;
    hipLaunchKernelGGL(rte::small_gemm_kernel, dim3(cdiv((long long)m * n, 256)), dim3(256), 0,
                       (hipStream_t)stream, trans_a, m, n, k, alpha, A, B, C);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_combine(const double *X, int ncol, long long len, const double *W, int r, double *out,
                rte_stream_t stream) {
    if (!X || !W || !out || ncol < 1 || r < 1 || len < 1) return RTE_EINVAL;
    hipLaunchKernelGGL(combine_kernel, dim3(cdiv(len, 16), cdiv(r, 16)), dim3(64), 0,
                       (hipStream_t)stream, X, ncol, len, W, r, out);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_apply_streaming(const rte_problem *p, const void *x, rte_precision xprec, int nvec,
                        double *y, rte_stream_t stream) {
    if (!p || !x || !y || nvec < 1 || p->dim != 2) return RTE_EINVAL;
    if (xprec != RTE_FP64 && xprec != RTE_MIXED) return RTE_EINVAL;
    const long long tot = (long long)nvec * p->n_dir * p->ncell;
    hipStream_t s = (hipStream_t)stream;
    if (xprec == RTE_MIXED)
        hipLaunchKernelGGL(apply_streaming_kernel<float>, dim3(cdiv(tot, 256)), dim3(256), 0, s,
                           p->nx, p->ny, p->n_dir, nvec, p->d_vxy, p->d_vxy + p->n_dir, p->hx,
                           p->hy, (const float *)x, y);
    else
        hipLaunchKernelGGL(apply_streaming_kernel<double>, dim3(cdiv(tot, 256)), dim3(256), 0, s,
                           p->nx, p->ny, p->n_dir, nvec, p->d_vxy, p->d_vxy + p->n_dir, p->hx,
                           p->hy, (const double *)x, y);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_inflow_loads(const rte_problem *p, const void *U, rte_precision uprec, int nvec,
                     double *out, rte_stream_t stream) {
    if (!p || !U || !out || nvec < 1) return RTE_EINVAL;
    if (uprec != RTE_FP64 && uprec != RTE_MIXED) return RTE_EINVAL;
    if (p->dim != 2) return RTE_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (uprec == RTE_MIXED)
        hipLaunchKernelGGL(inflow_load_kernel<float>, dim3(nvec, 4), dim3(256), 0, s, p->nx, p->ny,
                           p->ndof, p->n_dir, p->d_vxy, p->hx, p->hy, (const float *)U, nvec, out);
    else
        hipLaunchKernelGGL(inflow_load_kernel<double>, dim3(nvec, 4), dim3(256), 0, s, p->nx, p->ny,
                           p->ndof, p->n_dir, p->d_vxy, p->hx, p->hy, (const double *)U, nvec, out);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

int rte_direction_sum(const rte_problem *p, const void *x, rte_precision xprec, int nvec,
                      int weighted, double *out, rte_stream_t stream) {
    if (!p || !x || !out || nvec < 1) return RTE_EINVAL;
    if (xprec != RTE_FP64 && xprec != RTE_MIXED) return RTE_EINVAL;
    const dim3 grid(cdiv(p->ndof, 256), nvec);
    const double *w = weighted ? p->d_w : nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (xprec == RTE_MIXED)
        hipLaunchKernelGGL(direction_sum_kernel<float>, grid, dim3(256), 0, s, p->ndof, p->n_dir,
                           nvec, w, (const float *)x, out);
    else
        hipLaunchKernelGGL(direction_sum_kernel<double>, grid, dim3(256), 0, s, p->ndof, p->n_dir,
                           nvec, w, (const double *)x, out);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EDEVICE;
}

}  // extern "C"
