// DSA-preconditioned restarted GMRES (the paper's Krylov baseline, Sec. 2.4 and its appendix
// algorithm) for every instance of a batch: the left-preconditioned system
//   (I + C Sigma_s)(I - L) rho = (I + C Sigma_s) b_bar
// with L v one transport sweep of the source Sigma_s v (no G, vacuum inflow) and C Sigma_s the
// diffusion correction.  The sweeps and the corrections are the library's kernels; this file holds
// the Krylov bookkeeping, all FP64, one state per instance:
//   - vector updates and fixed-order partial dot products (no float atomics);
//   - Arnoldi orthogonalization by classical Gram-Schmidt with one reorthogonalization (the
//     Krylov basis of modified Gram-Schmidt up to rounding, in four passes over the vectors);
//   - Givens rotations of the Hessenberg column and the residual estimate, one thread per instance.
#include "rte_internal.h"

namespace rte {
namespace {

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }
constexpr int kGmBlock = 256;

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[kGmBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kGmBlock / 64; ++k) s += sh[k];
    __syncthreads();
    return s;
}

// part[b][slot0 + k][blk] = sum over the block's chunk of x_k[b] . w[b], k < nv
__global__ void __launch_bounds__(kGmBlock) gm_dots_kernel(long long n, int nv, const double *X,
                                                           size_t xstride, const double *w,
                                                           const int *flag, double *part,
                                                           int nslot, int slot0, int nblk) {
    const int b = blockIdx.y;
    if (!flag[b]) return;
    const long long chunk = (n + nblk - 1) / nblk;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < n ? lo + chunk : n;
    const double *wb = w + (size_t)b * n;
    for (int k = 0; k < nv; ++k) {
        const double *xb = X + k * xstride + (size_t)b * n;
        double acc = 0.0;
        for (long long t = lo + threadIdx.x; t < hi; t += kGmBlock) acc += xb[t] * wb[t];
        acc = block_sum(acc);
        if (threadIdx.x == 0) part[((size_t)b * nslot + slot0 + k) * nblk + blockIdx.x] = acc;
    }
}

// h[b][slot0 + k] (+)= sum_blk part[b][slot0 + k][blk], fixed order
__global__ void gm_sum_kernel(int B, int nv, const double *part, int nslot, int slot0, int nblk,
                              const int *flag, int accumulate, double *h) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * nv) return;
    const int b = t / nv, k = t - b * nv;
    if (!flag[b]) return;
    const double *p = part + ((size_t)b * nslot + slot0 + k) * nblk;
    double s = 0.0;
    for (int j = 0; j < nblk; ++j) s += p[j];
    double &dst = h[(size_t)b * nslot + slot0 + k];
    dst = accumulate ? dst + s : s;
}

// w[b] += sign * sum_{k < nv} c[b][k] x_k[b]; optionally the partials of |w|^2 into norm slot
__global__ void __launch_bounds__(kGmBlock) gm_axpy_kernel(long long n, int nv, const double *X,
                                                           size_t xstride, const double *c,
                                                           int cstride, double sign, double *w,
                                                           const int *flag, double *part,
                                                           int nslot, int normslot, int nblk) {
    const int b = blockIdx.y;
    if (!flag[b]) return;
    const long long chunk = (n + nblk - 1) / nblk;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < n ? lo + chunk : n;
    double *wb = w + (size_t)b * n;
    const double *cb = c + (size_t)b * cstride;
    double nrm = 0.0;
    for (long long t = lo + threadIdx.x; t < hi; t += kGmBlock) {
        double v = wb[t];
        for (int k = 0; k < nv; ++k) v += sign * cb[k] * X[k * xstride + (size_t)b * n + t];
        wb[t] = v;
        nrm += v * v;
    }
    if (part) {
        nrm = block_sum(nrm);
        if (threadIdx.x == 0) part[((size_t)b * nslot + normslot) * nblk + blockIdx.x] = nrm;
    }
}

// out = a + sa * x + sb * y (per element), for the flagged instances
__global__ void gm_lincomb_kernel(long long n, int B, const double *a, const double *x, double sa,
                                  const double *y, double sb, double *out, const int *flag) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= n || !flag[b]) return;
    const size_t i = (size_t)b * n + t;
    double v = a ? a[i] : 0.0;
    if (x) v += sa * x[i];
    if (y) v += sb * y[i];
    out[i] = v;
}

// out = w / s[b] for the flagged instances (s > 0)
__global__ void gm_scale_kernel(long long n, const double *w, const double *s, int sstride,
                                int sslot, double *out, const int *flag) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= n || !flag[b]) return;
    const double d = s[(size_t)b * sstride + sslot];
    out[(size_t)b * n + t] = d > 0.0 ? w[(size_t)b * n + t] / d : 0.0;
}

// start of a cycle: beta = ||r|| (from the norm slot); converged if beta <= tol ||M^-1 b||
__global__ void gm_cycle_start_kernel(int B, int m, const double *h, int nslot, int normslot,
                                      const double *nb, double tol, int *act, int *cyc, int *kused,
                                      double *g, double *y, int *count) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    if (!act[b]) { cyc[b] = 0; return; }
    const double beta = sqrt(h[(size_t)b * nslot + normslot]);
    double *gb = g + (size_t)b * (m + 1);
    for (int k = 0; k <= m; ++k) gb[k] = 0.0;
    for (int k = 0; k < m; ++k) y[(size_t)b * m + k] = 0.0;
    kused[b] = 0;
    if (!(beta > tol * nb[b])) {          // converged (also when the residual is exactly zero)
        act[b] = 0;
        cyc[b] = 0;
        return;
    }
    gb[0] = beta;
    cyc[b] = 1;
    atomicAdd(count, 1);
}

// Hessenberg column i from the Gram-Schmidt coefficients h[0..i] and the norm, the earlier
// rotations, the new one, and the residual estimate |g[i+1]|
__global__ void gm_givens_kernel(int B, int i, int m, const double *h, int nslot, int normslot,
                                 double *H, double *cs, double *sn, double *g, const double *nb,
                                 double tol, int *cyc, int *kused, int *n_iter, double *est,
                                 double *nrm_out, int *count) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || !cyc[b]) return;
    const double *hb = h + (size_t)b * nslot;
    double *Hb = H + (size_t)b * (m + 1) * m;
    double *cb = cs + (size_t)b * m, *sb = sn + (size_t)b * m, *gb = g + (size_t)b * (m + 1);
    for (int k = 0; k <= i; ++k) Hb[k * m + i] = hb[k];
    Hb[(i + 1) * m + i] = sqrt(hb[normslot]);
    nrm_out[b] = Hb[(i + 1) * m + i];         // the new basis vector is w / |w|
    for (int k = 0; k < i; ++k) {
        const double a0 = Hb[k * m + i], a1 = Hb[(k + 1) * m + i];
        Hb[k * m + i] = cb[k] * a0 + sb[k] * a1;
        Hb[(k + 1) * m + i] = -sb[k] * a0 + cb[k] * a1;
    }
    const double d = hypot(Hb[i * m + i], Hb[(i + 1) * m + i]);
    cb[i] = d > 0.0 ? Hb[i * m + i] / d : 1.0;
    sb[i] = d > 0.0 ? Hb[(i + 1) * m + i] / d : 0.0;
    Hb[i * m + i] = d;
    Hb[(i + 1) * m + i] = 0.0;
    gb[i + 1] = -sb[i] * gb[i];
    gb[i] = cb[i] * gb[i];
    kused[b] = i + 1;
    n_iter[b] += 1;
    est[b] = fabs(gb[i + 1]) / nb[b];
    if (fabs(gb[i + 1]) <= tol * nb[b] || i + 1 == m) cyc[b] = 0;
    else atomicAdd(count, 1);
}

// y = H^-1 g on the cycle's kused steps (upper triangular after the rotations)
__global__ void gm_solve_kernel(int B, int m, const double *H, const double *g, const int *kused,
                                const int *act, double *y) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || !act[b]) return;
    const int k = kused[b];
    const double *Hb = H + (size_t)b * (m + 1) * m;
    const double *gb = g + (size_t)b * (m + 1);
    double *yb = y + (size_t)b * m;
    for (int r = m - 1; r >= 0; --r) {
        if (r >= k) { yb[r] = 0.0; continue; }
        double s = gb[r];
        for (int c = r + 1; c < k; ++c) s -= Hb[r * m + c] * yb[c];
        yb[r] = s / Hb[r * m + r];
    }
}

__global__ void gm_sqrt_kernel(int B, const double *h, int nslot, int slot, const int *flag,
                               double *out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B && flag[b]) out[b] = sqrt(h[(size_t)b * nslot + slot]);
}

__global__ void gm_add_sweep_kernel(int B, const int *flag, int *n_sweep) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B && flag[b]) n_sweep[b] += 1;
}

}  // namespace

int gmres_blocks(const rte_problem *p) {
    long long nb = (p->ndof + 4095) / 4096;
    if (nb < 1) nb = 1;
    if (nb > 128) nb = 128;
    return (int)nb;
}

hipError_t gm_dots(const rte_problem *p, const GmresSpace &g, int nv, const double *X,
                   const double *w, const int *flag, double *dst, int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(gm_dots_kernel, dim3(g.nblk, p->B), dim3(kGmBlock), 0, s, p->ndof, nv, X,
                       (size_t)p->B * p->ndof, w, flag, g.part, g.nslot, 0, g.nblk);
    hipLaunchKernelGGL(gm_sum_kernel, dim3(blocks_for((long long)p->B * nv, 256)), dim3(256), 0, s,
                       p->B, nv, g.part, g.nslot, 0, g.nblk, flag, accumulate, dst);
    return hipGetLastError();
}

hipError_t gm_resum(const rte_problem *p, const GmresSpace &g, int nv, const int *flag,
                    double *dst, int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(gm_sum_kernel, dim3(blocks_for((long long)p->B * nv, 256)), dim3(256), 0, s,
                       p->B, nv, g.part, g.nslot, 0, g.nblk, flag, accumulate, dst);
    return hipGetLastError();
}

hipError_t gm_sqrt_norm(const rte_problem *p, const GmresSpace &g, const int *flag, double *out,
                        hipStream_t s) {
    hipLaunchKernelGGL(gm_sqrt_kernel, dim3(blocks_for(p->B, 256)), dim3(256), 0, s, p->B, g.h,
                       g.nslot, g.normslot, flag, out);
    return hipGetLastError();
}

hipError_t gm_axpy(const rte_problem *p, const GmresSpace &g, int nv, const double *X,
                   const double *c, int cstride, double sign, double *w, const int *flag,
                   bool norm, hipStream_t s) {
    hipLaunchKernelGGL(gm_axpy_kernel, dim3(g.nblk, p->B), dim3(kGmBlock), 0, s, p->ndof, nv, X,
                       (size_t)p->B * p->ndof, c, cstride, sign, w, flag, norm ? g.part : nullptr,
                       g.nslot, g.normslot, g.nblk);
    if (norm)
        hipLaunchKernelGGL(gm_sum_kernel, dim3(blocks_for(p->B, 256)), dim3(256), 0, s, p->B, 1,
                           g.part, g.nslot, g.normslot, g.nblk, flag, 0, g.h);
    return hipGetLastError();
}

hipError_t gm_lincomb(const rte_problem *p, const double *a, const double *x, double sa,
                      const double *y, double sb, double *out, const int *flag, hipStream_t s) {
    hipLaunchKernelGGL(gm_lincomb_kernel, dim3(blocks_for(p->ndof, 256), p->B), dim3(256), 0, s,
                       p->ndof, p->B, a, x, sa, y, sb, out, flag);
    return hipGetLastError();
}

hipError_t gm_norm(const rte_problem *p, const GmresSpace &g, const double *w, const int *flag,
                   hipStream_t s) {
    // |w|^2 into the norm slot: an axpy with no terms
    return gm_axpy(p, g, 0, w, g.h, g.nslot, 0.0, const_cast<double *>(w), flag, true, s);
}

hipError_t gm_scale(const rte_problem *p, const GmresSpace &g, const double *w, const double *sv,
                    int sstride, int sslot, double *out, const int *flag, hipStream_t s) {
    hipLaunchKernelGGL(gm_scale_kernel, dim3(blocks_for(p->ndof, 256), p->B), dim3(256), 0, s,
                       p->ndof, w, sv, sstride, sslot, out, flag);
    return hipGetLastError();
}

hipError_t gm_cycle_start(const rte_problem *p, const GmresSpace &g, double tol, hipStream_t s) {
    hipLaunchKernelGGL(gm_cycle_start_kernel, dim3(blocks_for(p->B, 256)), dim3(256), 0, s, p->B,
                       g.m, g.h, g.nslot, g.normslot, g.nb, tol, g.act, g.cyc, g.kused, g.g, g.y,
                       g.count);
    return hipGetLastError();
}

hipError_t gm_givens(const rte_problem *p, const GmresSpace &g, int i, double tol, hipStream_t s) {
    hipLaunchKernelGGL(gm_givens_kernel, dim3(blocks_for(p->B, 256)), dim3(256), 0, s, p->B, i,
                       g.m, g.h, g.nslot, g.normslot, g.H, g.cs, g.sn, g.g, g.nb, tol, g.cyc,
                       g.kused, g.n_iter, g.est, g.wn, g.count);
    return hipGetLastError();
}

hipError_t gm_solve(const rte_problem *p, const GmresSpace &g, hipStream_t s) {
    hipLaunchKernelGGL(gm_solve_kernel, dim3(blocks_for(p->B, 256)), dim3(256), 0, s, p->B, g.m,
                       g.H, g.g, g.kused, g.act, g.y);
    return hipGetLastError();
}

hipError_t gm_count_sweep(const rte_problem *p, const GmresSpace &g, const int *flag,
                          hipStream_t s) {
    hipLaunchKernelGGL(gm_add_sweep_kernel, dim3(blocks_for(p->B, 256)), dim3(256), 0, s, p->B,
                       flag, g.n_sweep);
    return hipGetLastError();
}

}  // namespace rte
