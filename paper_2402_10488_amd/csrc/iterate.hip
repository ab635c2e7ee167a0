// Alg. 1 (source iteration with synthetic acceleration) and Alg. 2 (ROMSAD switch) bookkeeping
// on the device: the stop test, the per-instance choice of correction, and the density update
// rho^(l) = rho^(l,*) + delta rho^(l) fused with the source prologue of the next sweep.
#include "rte_internal.h"

namespace rte {
namespace {

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// kind codes written per instance after its sweep l (l counts that instance's own sweeps, so
// instances admitted at different times each follow Alg. 1 from their own start):
//   0 no correction (SI), 1 DSA, 2 ROMSA, -1 converged at l, -2 stopped at max_iter
__global__ void decide_kernel(int B, int max_iter, double eps, int relative, int mode,
                              int theta, double eps_romsad, unsigned long long *maxd,
                              unsigned long long *maxr, int *active, int *kind, int *n_sweep,
                              int *status, double *change, int *kinds, int *n_active) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    if (!active[b]) { kind[b] = -3; return; }
    const int l = n_sweep[b] + 1;
    const double md = __longlong_as_double((long long)maxd[b]);
    const double mr = __longlong_as_double((long long)maxr[b]);
    maxd[b] = 0ull;
    maxr[b] = 0ull;
    double e;
    if (relative) e = mr > 0.0 ? md / mr : (md == 0.0 ? 0.0 : INFINITY);
    else e = md;
    if (!(e == e)) e = INFINITY;                     // NaN never passes the test
    change[(size_t)b * max_iter + (l - 1)] = e;
    n_sweep[b] = l;
    int k;
    if (e < eps) { k = -1; status[b] = RTE_OK; }
    else if (l >= max_iter) { k = -2; status[b] = RTE_ENOCONV; }
    else if (mode == RTE_SI) k = 0;
    else if (mode == RTE_SI_DSA) k = 1;
    else k = (l >= 1 && l <= theta && e >= eps_romsad) ? 2 : 1;    // Alg. 2
    kind[b] = k;
    kinds[(size_t)b * max_iter + (l - 1)] = k < 0 ? 0 : k;
    if (k >= 0) atomicAdd(&n_active[0], 1);
    if (k > 0) atomicAdd(&n_active[k], 1);            // [1]: DSA this iteration, [2]: ROMSA
}

template <typename T>
__global__ void update_kernel(int dim, long long ncell, int K, int B, int nx, int ny,
                              const int *kind, int *active, const double *rho_star,
                              const double *delta, double *rho, const double *sigma_t,
                              const double *sigma_s, const double *G, const double *cellw,
                              double ghost, T *src) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * ncell) return;
    const int b = (int)(t / ncell);
    const int k = kind[b];
    if (k == -3) return;                              // finished earlier
    const long long cell = t - (long long)b * ncell;
    if (k < 0) {                                      // converged / stopped: keep rho^(l,*)
        for (int q = 0; q < K; ++q) rho[t * K + q] = rho_star[t * K + q];
        if (cell == 0) active[b] = 0;
        return;
    }
    const double ss = sigma_s[t];
    const double g0 = G[t] * (cellw ? sqrt(cellw[cell]) : ghost);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < K; ++q) {
        double r = rho_star[t * K + q];
        if (k > 0 && delta) r += delta[t * K + q];
        rho[t * K + q] = r;
        v[q] = ss * r + (q == 0 ? g0 : 0.0);
    }
    write_sweep_input<T>(dim, ncell, B, b, nx, ny, cell, v, sigma_t[t], src);
}

// 2D update on 16 x 16 cell tiles (grid: tiles x instances): rho = rho* + delta and the source
// part of the sweep input.  sigma_t in the sweep input does not change between iterations (the
// solve's start writes it), so it is not rewritten.  A tile's cells on one diagonal sit on
// consecutive positions of either diagonal layout, so a workgroup's source stores fill whole
// cache lines.
template <typename T>
__global__ void __launch_bounds__(256) update2d_kernel(long long ncell, int B, int nx, int ny,
                                                       int tiles_x, const int *kind, int *active,
                                                       const double *rho_star, const double *delta,
                                                       double *rho, const double *sigma_s,
                                                       const double *G, double ghost, T *src) {
    const int b = blockIdx.y;
    const int k = kind[b];
    if (k == -3) return;                              // finished earlier
    const int x = (int)(blockIdx.x % tiles_x) * 16 + (int)(threadIdx.x & 15);
    const int y = (int)(blockIdx.x / tiles_x) * 16 + (int)(threadIdx.x >> 4);
    if (x >= nx || y >= ny) return;
    const long long cell = (long long)y * nx + x;
    const long long t = (long long)b * ncell + cell;
    const double4 rs = *reinterpret_cast<const double4 *>(rho_star + t * 4);
    double4 r = rs;
    if (k < 0) {                                      // converged / stopped: keep rho^(l,*)
        *reinterpret_cast<double4 *>(rho + t * 4) = r;
        if (cell == 0) active[b] = 0;
        return;
    }
    if (k > 0 && delta) {
        const double4 dv = *reinterpret_cast<const double4 *>(delta + t * 4);
        r.x += dv.x; r.y += dv.y; r.z += dv.z; r.w += dv.w;
    }
    *reinterpret_cast<double4 *>(rho + t * 4) = r;
    const double ss = sigma_s[t];
    const double g0 = G[t] * ghost;
    Vec4<T> o;
    o.x = (T)(ss * r.x + g0);
    o.y = (T)(ss * r.y + 0.0);
    o.z = (T)(ss * r.z + 0.0);
    o.w = (T)(ss * r.w + 0.0);
    const size_t nb4 = (size_t)B * ncell * 4;
    const size_t pa = (size_t)b * ncell + pos_a(nx, ny, x, y);
    const size_t pb = (size_t)b * ncell + pos_b(nx, ny, x, y);
    *reinterpret_cast<Vec4<T> *>(src + pa * 4) = o;
    *reinterpret_cast<Vec4<T> *>(src + nb4 + pb * 4) = o;
}

// start (run = 1) or idle (run = 0) the instances selected by mask (all when mask is null)
__global__ void init_state_kernel(int B, int max_iter, const int *mask, int run,
                                  unsigned long long *maxd, unsigned long long *maxr, int *active,
                                  int *kind, int *n_sweep, int *status, double *change, int *kinds) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < B && (!mask || mask[t])) {
        maxd[t] = 0ull;
        maxr[t] = 0ull;
        active[t] = run;
        kind[t] = run ? 0 : -3;
        n_sweep[t] = 0;
        status[t] = run ? RTE_ENOCONV : RTE_OK;
    }
    if (t < (long long)B * max_iter && (!mask || mask[t / max_iter])) {
        change[t] = 0.0;
        kinds[t] = 0;
    }
}

__global__ void zero_kernel(double *x, long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = 0.0;
}

__global__ void zero_rows_kernel(double *x, long long n, const int *mask) {
    const int b = blockIdx.y;
    if (mask && !mask[b]) return;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[(size_t)b * n + t] = 0.0;
}

__global__ void zero_u64_kernel(unsigned long long *x, long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = 0ull;
}

__global__ void fill_int_kernel(int *x, long long n, int v) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = v;
}

}  // namespace

hipError_t launch_decide(const rte_problem *p, const IterState &st, int max_iter, double eps,
                         int relative, int mode, int theta, double eps_romsad, hipStream_t s) {
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, st.n_active, 3ll, 0);
    hipLaunchKernelGGL(decide_kernel, dim3(blocks_for(p->B, 256)), dim3(256), 0, s, p->B,
                       max_iter, eps, relative, mode, theta, eps_romsad, st.maxd, st.maxr,
                       st.active, st.kind, st.n_sweep, st.status, st.change, st.kinds,
                       st.n_active);
    return hipGetLastError();
}

hipError_t launch_update(const rte_problem *p, const IterState &st, const double *rho_star,
                         const double *delta, double *rho, void *src, int fp32, hipStream_t s) {
    const long long n = (long long)p->B * p->ncell;
    const double ghost = sqrt(p->hx * p->hy);
    const double *cw = p->dim == 1 ? p->d_widths : nullptr;
    if (p->dim == 2) {
        const int tx = (p->nx + 15) / 16, ty = (p->ny + 15) / 16;
        const dim3 grid((unsigned)(tx * ty), p->B);
        if (fp32)
            hipLaunchKernelGGL(update2d_kernel<float>, grid, dim3(256), 0, s, p->ncell, p->B,
                               p->nx, p->ny, tx, st.kind, st.active, rho_star, delta, rho,
                               p->sigma_s, p->source, ghost, (float *)src);
        else
            hipLaunchKernelGGL(update2d_kernel<double>, grid, dim3(256), 0, s, p->ncell, p->B,
                               p->nx, p->ny, tx, st.kind, st.active, rho_star, delta, rho,
                               p->sigma_s, p->source, ghost, (double *)src);
        return hipGetLastError();
    }
    if (fp32)
        hipLaunchKernelGGL(update_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           p->dim, p->ncell, p->K, p->B, p->nx, p->ny, st.kind, st.active,
                           rho_star, delta, rho, p->sigma_t, p->sigma_s, p->source, cw, ghost,
                           (float *)src);
    else
        hipLaunchKernelGGL(update_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           p->dim, p->ncell, p->K, p->B, p->nx, p->ny, st.kind, st.active,
                           rho_star, delta, rho, p->sigma_t, p->sigma_s, p->source, cw, ghost,
                           (double *)src);
    return hipGetLastError();
}

hipError_t launch_init_state(const rte_problem *p, const IterState &st, int max_iter,
                             const int *mask, int run, hipStream_t s) {
    const long long n = (long long)p->B * max_iter > p->B ? (long long)p->B * max_iter : p->B;
    hipLaunchKernelGGL(init_state_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p->B,
                       max_iter, mask, run, st.maxd, st.maxr, st.active, st.kind, st.n_sweep, st.status,
                       st.change, st.kinds);
    return hipGetLastError();
}

hipError_t launch_zero(double *x, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_zero_rows(double *x, int B, long long n, const int *mask, hipStream_t s) {
    if (n <= 0 || B <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_rows_kernel, dim3(blocks_for(n, 256), B), dim3(256), 0, s, x, n, mask);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *x, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *x, long long n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}

}  // namespace rte
