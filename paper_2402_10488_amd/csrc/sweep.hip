// Transport sweeps, quadrature reduction and the source prologue (gfx950).
//
// 2D sweep (eq. (transport_sweep) with the upwind flux of eq. (upwind)):
//   One wavefront owns one (instance, quadrant, group of DG directions).  Its 64 lanes are 64
//   consecutive mesh rows of a band; lane j processes column i of band k at step
//   t = k*P + i + j, so the lanes form a diagonal wavefront that walks the whole mesh band after
//   band without a pipeline restart.  The y-trace of lane j reaches lane j+1 one step later
//   through a cross-lane shuffle, the last lane of a band hands its traces to lane 0 of the next
//   band through an LDS ring indexed by column, and the x-trace stays in registers.  Each lane
//   solves the DG cell system of DG directions per step and accumulates their contribution to
//   rho in FP64, so one partial density per (instance, quadrant group) leaves the kernel.
//
//   Every quadrant is swept in reflected coordinates (the sweep always runs towards +x, +y):
//   flipping the sign of the odd Legendre modes maps the upwind DG system of any quadrant onto
//   the (+,+) one.  In those coordinates the Q1 cell system with a = |vx|/hx, b = |vy|/hy is
//     K = a (A (x) I) + b (I (x) A) + sigma_t I,   A = [[1, s3], [-s3, 3]]   (s3 = sqrt 3)
//   (A from the volume and outflow-edge terms of eq. (DG) in the orthonormal basis), solved in
//   closed form by block elimination: with X = aA + (b+sigma)I, Y = aA + (3b+sigma)I and
//   A^2 = 4A - 6I, the Schur complement X Y + 3 b^2 I = uA + wI is again a polynomial in A.
#include "rte_internal.h"

namespace rte {
namespace {

constexpr double kS3 = 1.7320508075688772935;

template <typename T>
struct Vec4 { T x, y, z, w; };

struct Sweep2DArgs {
    int nx, ny, B, nbands, P, n_dir, nparts;
    int gq[4];
    int qstart[4];
    long long ncell;
    double ghost;            // sqrt(hx hy): coefficient of a unit constant on phi_0
    int zero_inflow;
    const DirEntry *dirs;
    const double *sigma_t;
    const void *src;
    const double *inflow;
    double *partial;
    void *f_out;
    const int *active;
};

// Q1 cell solve in reflected coordinates; unknown order k = a + 2b: (f00, f10, f01, f11).
template <typename T>
__device__ __forceinline__ void q1_solve(T al, T be, T sig, T r0, T r1, T r2, T r3, T &f0, T &f1,
                                         T &f2, T &f3) {
    const T c = T(kS3);
    const T p = be + sig;
    const T q = T(3) * be + sig;
    const T u = al * (T(4) * al + p + q);
    const T w = p * q + T(3) * be * be - T(6) * al * al;
    const T tm = w + T(2) * u;
    const T detM = tm * tm + T(2) * u * u;          // det(uA + wI) = (w+2u)^2 + 2u^2 > 0
    const T tx = p + T(2) * al;
    const T detX = tx * tx + T(2) * al * al;        // det(X) = (p+2a)^2 + 2a^2 > 0
    const T inv = T(1) / (detM * detX);
    const T iM = detX * inv;
    const T iX = detM * inv;
    const T ca = c * al, cb = c * be, cu = c * u;
    // right-hand side of the Schur system: X R1 + c b R0
    const T g0 = (al + p) * r2 + ca * r3 + cb * r0;
    const T g1 = -ca * r2 + (T(3) * al + p) * r3 + cb * r1;
    f2 = ((T(3) * u + w) * g0 - cu * g1) * iM;
    f3 = (cu * g0 + (u + w) * g1) * iM;
    const T h0 = r0 - cb * f2;
    const T h1 = r1 - cb * f3;
    f0 = ((T(3) * al + p) * h0 - ca * h1) * iX;
    f1 = (ca * h0 + (al + p) * h1) * iX;
}

template <typename T>
__device__ __forceinline__ T shfl_up1(T v) {
    return __shfl_up(v, 1, 64);
}

template <typename T, int DG>
__global__ void __launch_bounds__(256) sweep2d_kernel(Sweep2DArgs a) {
    extern __shared__ unsigned char smem_raw[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const long long item = (long long)blockIdx.x * wpb + wv;
    if (item >= (long long)a.B * a.nparts) return;           // whole wavefront leaves
    const int b = (int)(item / a.nparts);
    const int gpart = (int)(item - (long long)b * a.nparts);
    if (a.active && a.active[b] == 0) return;
    int part = gpart, q = 0;
    while (q < 3 && part >= a.gq[q]) { part -= a.gq[q]; ++q; }
    const int d0 = a.qstart[q] + part * DG;
    const bool rx = (q & 1) != 0, ry = (q & 2) != 0;
    T *ring = reinterpret_cast<T *>(smem_raw) + (size_t)wv * a.nx * DG * 2;

    T al[DG], be[DG];
    double wt[DG];
    int orig[DG];
#pragma unroll
    for (int d = 0; d < DG; ++d) {
        const DirEntry e = a.dirs[d0 + d];
        al[d] = (T)e.alpha;
        be[d] = (T)e.beta;
        wt[d] = e.w;
        orig[d] = e.orig;
    }
    const T gx = a.zero_inflow ? T(0) : (T)(a.inflow[4 * b + (rx ? 1 : 0)] * a.ghost);
    const T gy = a.zero_inflow ? T(0) : (T)(a.inflow[4 * b + (ry ? 3 : 2)] * a.ghost);
    const T sx = rx ? T(-1) : T(1), sy = ry ? T(-1) : T(1);
    const double dsx = rx ? -1.0 : 1.0, dsy = ry ? -1.0 : 1.0;
    const T c = T(kS3);

    const T *src = reinterpret_cast<const T *>(a.src) + (size_t)b * a.ncell * 4;
    const double *sig_t = a.sigma_t + (size_t)b * a.ncell;
    double *part_out = a.partial ? a.partial + ((size_t)b * a.nparts + gpart) * a.ncell * 4 : nullptr;
    T *fout = a.f_out ? reinterpret_cast<T *>(a.f_out) + (size_t)b * a.n_dir * a.ncell * 4 : nullptr;

    T tx0[DG], tx1[DG], ty0[DG], ty1[DG];
#pragma unroll
    for (int d = 0; d < DG; ++d) { tx0[d] = tx1[d] = ty0[d] = ty1[d] = T(0); }

    const long long total = (long long)a.nbands * a.P + 63;
    for (long long t = 0; t < total; ++t) {
        T yi0[DG], yi1[DG];
#pragma unroll
        for (int d = 0; d < DG; ++d) {               // all lanes take part in the shuffle
            yi0[d] = shfl_up1(ty0[d]);
            yi1[d] = shfl_up1(ty1[d]);
        }
        const long long u = t - lane;
        if (u < 0) continue;
        const int k = (int)(u / a.P);
        const int i = (int)(u - (long long)k * a.P);
        const int jr = k * 64 + lane;
        if (k >= a.nbands || i >= a.nx || jr >= a.ny) continue;
        if (lane == 0) {
#pragma unroll
            for (int d = 0; d < DG; ++d) {
                if (k == 0) { yi0[d] = gy; yi1[d] = T(0); }
                else { yi0[d] = ring[(i * DG + d) * 2]; yi1[d] = ring[(i * DG + d) * 2 + 1]; }
            }
        }
        if (i == 0) {
#pragma unroll
            for (int d = 0; d < DG; ++d) { tx0[d] = gx; tx1[d] = T(0); }
        }
        const int ip = rx ? a.nx - 1 - i : i;
        const int jp = ry ? a.ny - 1 - jr : jr;
        const long long cell = (long long)jp * a.nx + ip;
        const Vec4<T> sv = *reinterpret_cast<const Vec4<T> *>(src + cell * 4);
        const T s0 = sv.x, s1 = sx * sv.y, s2 = sy * sv.z, s3 = sx * sy * sv.w;
        const T sig = (T)sig_t[cell];
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
#pragma unroll
        for (int d = 0; d < DG; ++d) {
            const T ca = c * al[d], cb = c * be[d];
            const T r0 = s0 + al[d] * tx0[d] + be[d] * yi0[d];
            const T r1 = s1 - ca * tx0[d] + be[d] * yi1[d];
            const T r2 = s2 + al[d] * tx1[d] - cb * yi0[d];
            const T r3 = s3 - ca * tx1[d] - cb * yi1[d];
            T f0, f1, f2, f3;
            q1_solve<T>(al[d], be[d], sig, r0, r1, r2, r3, f0, f1, f2, f3);
            tx0[d] = f0 + c * f1;
            tx1[d] = f2 + c * f3;
            ty0[d] = f0 + c * f2;
            ty1[d] = f1 + c * f3;
            acc0 += wt[d] * (double)f0;
            acc1 += wt[d] * (double)f1;
            acc2 += wt[d] * (double)f2;
            acc3 += wt[d] * (double)f3;
            if (fout && orig[d] >= 0) {
                Vec4<T> o;
                o.x = f0; o.y = sx * f1; o.z = sy * f2; o.w = sx * sy * f3;
                *reinterpret_cast<Vec4<T> *>(fout + ((size_t)orig[d] * a.ncell + cell) * 4) = o;
            }
        }
        if (lane == 63) {
#pragma unroll
            for (int d = 0; d < DG; ++d) {
                ring[(i * DG + d) * 2] = ty0[d];
                ring[(i * DG + d) * 2 + 1] = ty1[d];
            }
        }
        if (part_out) {
            double *o = part_out + cell * 4;
            o[0] = acc0;
            o[1] = dsx * acc1;
            o[2] = dsy * acc2;
            o[3] = dsx * dsy * acc3;
        }
    }
}

// ------------------------------------------------------------------------------------- 1D
template <typename T>
__global__ void __launch_bounds__(256) sweep1d_kernel(int nc, int n_dir, int B, const double *mu,
                                                      const double *widths, const double *sigma_t,
                                                      const T *src, const double *inflow,
                                                      int zero_inflow, T *f_out,
                                                      const int *active) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * n_dir) return;
    const int b = (int)(t / n_dir), j = (int)(t - (long long)b * n_dir);
    if (active && active[b] == 0) return;
    const double m = mu[j];
    const bool rev = m < 0.0;
    const T am = (T)fabs(m);
    const T c = T(kS3);
    T edge = zero_inflow ? T(0) : (T)inflow[4 * b + (rev ? 1 : 0)];   // physical inflow value
    const T *s = src + (size_t)b * nc * 2;
    T *f = f_out + ((size_t)b * n_dir + j) * nc * 2;
    for (int st = 0; st < nc; ++st) {
        const int cc = rev ? nc - 1 - st : st;
        const T h = (T)widths[cc];
        const T sq = sqrt(h);
        const T aa = am / h;
        const T sig = (T)sigma_t[(size_t)b * nc + cc];
        const T e = am * edge / sq;               // |mu| f_edge phi_0(inflow edge)
        const T r0 = s[2 * cc] + e;
        const T r1 = (rev ? -s[2 * cc + 1] : s[2 * cc + 1]) - c * e;
        const T tt = sig + T(2) * aa;
        const T det = tt * tt + T(2) * aa * aa;
        const T f0 = ((T(3) * aa + sig) * r0 - c * aa * r1) / det;
        const T f1 = (c * aa * r0 + (aa + sig) * r1) / det;
        f[2 * cc] = f0;
        f[2 * cc + 1] = rev ? -f1 : f1;
        edge = (f0 + c * f1) / sq;                 // outflow trace value
    }
}

// ------------------------------------------------------------------ source, reductions
template <typename T>
__global__ void source_kernel(long long ncell, int K, int B, const double *rho,
                              const double *sigma_s, const double *G, const double *cellw,
                              double ghost, T *src, const int *active) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * ncell) return;
    const int b = (int)(t / ncell);
    if (active && active[b] == 0) return;
    const long long cell = t - (long long)b * ncell;
    const double ss = sigma_s[t];
    const double g0 = G[t] * (cellw ? sqrt(cellw[cell]) : ghost);
    for (int k = 0; k < K; ++k) {
        const double v = ss * rho[t * K + k] + (k == 0 ? g0 : 0.0);
        src[t * K + k] = (T)v;
    }
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ void max_update(unsigned long long *dst, double v) {
    // non-negative doubles order like their bit patterns; max is exact, hence deterministic
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0 && v > 0.0) atomicMax(dst, (unsigned long long)__double_as_longlong(v));
}

__global__ void reduce_parts_kernel(long long ndof, int B, int nparts, const double *partial,
                                    double *rho_star, const double *rho_prev,
                                    unsigned long long *maxd, unsigned long long *maxr,
                                    const int *active) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = (int)(blockIdx.y);
    double d = 0.0, m = 0.0;
    const bool live = t < ndof && (!active || active[b] != 0);
    if (live) {
        const double *p = partial + (size_t)b * nparts * ndof + t;
        double s = 0.0;
        for (int k = 0; k < nparts; ++k) s += p[(size_t)k * ndof];
        rho_star[(size_t)b * ndof + t] = s;
        m = fabs(s);
        if (rho_prev) d = fabs(s - rho_prev[(size_t)b * ndof + t]);
    }
    if (maxd) max_update(maxd + b, d);
    if (maxr) max_update(maxr + b, m);
}

template <typename T>
__global__ void scalar_flux_kernel(long long ndof, int B, int n_dir, const double *w, const T *f,
                                   double *rho, const double *rho_prev, unsigned long long *maxd,
                                   unsigned long long *maxr, const int *active) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = (int)(blockIdx.y);
    double d = 0.0, m = 0.0;
    const bool live = t < ndof && (!active || active[b] != 0);
    if (live) {
        const T *fb = f + (size_t)b * n_dir * ndof + t;
        double s = 0.0;
        for (int j = 0; j < n_dir; ++j) s += w[j] * (double)fb[(size_t)j * ndof];
        rho[(size_t)b * ndof + t] = s;
        m = fabs(s);
        if (rho_prev) d = fabs(s - rho_prev[(size_t)b * ndof + t]);
    }
    if (maxd) max_update(maxd + b, d);
    if (maxr) max_update(maxr + b, m);
}

__global__ void check_kernel(long long n, const double *st, const double *ss, const double *g,
                             int *bad) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double a = st[t], s = ss[t], G = g[t];
    const bool ok = isfinite(a) && isfinite(s) && isfinite(G) && s >= 0.0 && a >= s;
    if (!ok) atomicOr(bad, 1);
}

template <typename T, int DG>
hipError_t sweep2d_launch_t(const SweepLaunch &L, hipStream_t s) {
    const rte_problem *p = L.p;
    Sweep2DArgs a;
    a.nx = p->nx;
    a.ny = p->ny;
    a.B = p->B;
    a.nbands = (p->ny + 63) / 64;
    a.P = p->nx > 64 ? p->nx : 64;
    a.n_dir = p->n_dir;
    a.nparts = 0;
    for (int q = 0; q < 4; ++q) {
        a.gq[q] = (p->quad.count[q] + DG - 1) / DG;
        a.qstart[q] = p->quad.start[q];
        a.nparts += a.gq[q];
    }
    a.ncell = p->ncell;
    a.ghost = sqrt(p->hx * p->hy);
    a.zero_inflow = L.zero_inflow;
    a.dirs = p->d_dirs;
    a.sigma_t = p->sigma_t;
    a.src = L.src;
    a.inflow = p->inflow;
    a.partial = L.partial;
    a.f_out = L.f_out;
    a.active = L.active;
    const int wpb = p->tune.wpb;
    const long long items = (long long)a.B * a.nparts;
    const unsigned grid = (unsigned)((items + wpb - 1) / wpb);
    const size_t lds = (size_t)wpb * p->nx * DG * 2 * sizeof(T);
    hipLaunchKernelGGL((sweep2d_kernel<T, DG>), dim3(grid), dim3(64 * wpb), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t sweep2d_dispatch(const SweepLaunch &L, hipStream_t s) {
    switch (L.p->tune.dg) {
        case 1: return sweep2d_launch_t<T, 1>(L, s);
        case 2: return sweep2d_launch_t<T, 2>(L, s);
        case 4: return sweep2d_launch_t<T, 4>(L, s);
        case 8: return sweep2d_launch_t<T, 8>(L, s);
        case 16: return sweep2d_launch_t<T, 16>(L, s);
        default: return hipErrorInvalidValue;
    }
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_sweep2d(const SweepLaunch &a, hipStream_t s) {
    return a.fp32 ? sweep2d_dispatch<float>(a, s) : sweep2d_dispatch<double>(a, s);
}

hipError_t launch_sweep1d(const rte_problem *p, const void *src, void *f_out, const int *active,
                          int zero_inflow, int fp32, hipStream_t s) {
    const long long n = (long long)p->B * p->n_dir;
    if (fp32)
        hipLaunchKernelGGL(sweep1d_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, p->nx,
                           p->n_dir, p->B, p->d_mu, p->d_widths, p->sigma_t,
                           (const float *)src, p->inflow, zero_inflow, (float *)f_out, active);
    else
        hipLaunchKernelGGL(sweep1d_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, p->nx,
                           p->n_dir, p->B, p->d_mu, p->d_widths, p->sigma_t,
                           (const double *)src, p->inflow, zero_inflow, (double *)f_out, active);
    return hipGetLastError();
}

hipError_t launch_source(const rte_problem *p, const double *rho, void *src, const int *active,
                         int fp32, hipStream_t s) {
    const long long n = (long long)p->B * p->ncell;
    const double ghost = sqrt(p->hx * p->hy);
    const double *cw = p->dim == 1 ? p->d_widths : nullptr;
    if (fp32)
        hipLaunchKernelGGL(source_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, p->ncell,
                           p->K, p->B, rho, p->sigma_s, p->source, cw, ghost, (float *)src, active);
    else
        hipLaunchKernelGGL(source_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           p->ncell, p->K, p->B, rho, p->sigma_s, p->source, cw, ghost,
                           (double *)src, active);
    return hipGetLastError();
}

hipError_t launch_reduce_parts(const rte_problem *p, const double *partial, int nparts,
                               double *rho_star, const double *rho_prev, unsigned long long *maxd,
                               unsigned long long *maxr, const int *active, hipStream_t s) {
    dim3 grid(blocks_for(p->ndof, 256), p->B);
    hipLaunchKernelGGL(reduce_parts_kernel, grid, dim3(256), 0, s, p->ndof, p->B, nparts, partial,
                       rho_star, rho_prev, maxd, maxr, active);
    return hipGetLastError();
}

hipError_t launch_scalar_flux(const rte_problem *p, const void *f, double *rho, int fp32,
                              const double *rho_prev, unsigned long long *maxd,
                              unsigned long long *maxr, const int *active, hipStream_t s) {
    dim3 grid(blocks_for(p->ndof, 256), p->B);
    if (fp32)
        hipLaunchKernelGGL(scalar_flux_kernel<float>, grid, dim3(256), 0, s, p->ndof, p->B, p->n_dir,
                           p->d_w, (const float *)f, rho, rho_prev, maxd, maxr, active);
    else
        hipLaunchKernelGGL(scalar_flux_kernel<double>, grid, dim3(256), 0, s, p->ndof, p->B,
                           p->n_dir, p->d_w, (const double *)f, rho, rho_prev, maxd, maxr, active);
    return hipGetLastError();
}

hipError_t launch_check_materials(const rte_problem *p, int *bad, hipStream_t s) {
    const long long n = (long long)p->B * p->ncell;
    hipLaunchKernelGGL(check_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, p->sigma_t,
                       p->sigma_s, p->source, bad);
    return hipGetLastError();
}

}  // namespace rte
