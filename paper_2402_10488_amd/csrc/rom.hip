// ROM-based kinetic correction (ROMSA) on the device, eq. (rom_correction):
//   y_b   = U_iso^T (Sigma_s (rho*_b - rho_b))      tall-skinny product over all ROMSA instances
//   A_b   = A0 + sum_k psi_bk A_k,   A_b dc_b = y_b  (r x r LU with partial pivoting, FP64)
//   drho_b = U_rho dc_b
// The two products run on the matrix cores: v_mfma_f64_16x16x4f64 in FP64 mode and
// v_mfma_f32_16x16x4f32 in mixed mode.  Operand layout (one element per lane for A and B, four
// results per lane; measured on gfx950):
//   A[m][k]: lane m + 16 k;   B[k][n]: lane n + 16 k;
//   D[m][n]: lane n + 16 q, item i with  m = 4 q + i (f32)  or  m = q + 4 i (f64).
// The reduction over the N_DOF dofs is split over workgroups; the split partials are summed in
// a fixed order, so the result does not depend on scheduling.
#include "rte_internal.h"

namespace rte {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kProjChunk = 256;        // dofs per wave-iteration group in the projection

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> struct VecOf;
template <> struct VecOf<double> { typedef v4d type; };
template <> struct VecOf<float> { typedef v4f type; };

// row of D held in item i of a lane in row group q (see the layout above)
template <typename T> __device__ __forceinline__ int drow(int q, int i);
template <> __device__ __forceinline__ int drow<float>(int q, int i) { return 4 * q + i; }
template <> __device__ __forceinline__ int drow<double>(int q, int i) { return q + 4 * i; }

// grid: x = split index, y = instance tile (16 instances); one wave each, holding all RT rank
// tiles of 16 so that every value of rho* and rho is read once.  ypart[b][split][r]
template <typename T, int RT>
__global__ void __launch_bounds__(64) rom_project_kernel(long long ndof, int K, int B, int r,
                                                         int nsplit, long long per_split,
                                                         const T *U_iso, const double *sigma_s,
                                                         const double *rho_star,
                                                         const double *rho_prev, const int *kind,
                                                         int want, double *ypart) {
    typedef typename VecOf<T>::type V;
    const int lane = threadIdx.x;
    const int split = blockIdx.x;
    const int b0 = blockIdx.y * 16;
    const int n = lane & 15;          // instance within tile (B operand column) / rank row of A
    const int kq = lane >> 4;         // 0..3
    const int b = b0 + n;
    const bool live_b = b < B && (!kind || kind[b] == want);
    // only the ROMSA instances' partials are read; a tile without one has nothing to do
    if (__builtin_amdgcn_ballot_w64(live_b) == 0) return;
    V acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = V{0, 0, 0, 0};
    const long long k_begin = (long long)split * per_split;
    long long k_end = k_begin + per_split;
    if (k_end > ndof) k_end = ndof;
    const double *rs = rho_star + (size_t)(live_b ? b : 0) * ndof;
    const double *rp = rho_prev + (size_t)(live_b ? b : 0) * ndof;
    const double *ss = sigma_s + (size_t)(live_b ? b : 0) * (ndof / K);
    // each group of 16 dofs: lane (n, kq) holds dofs k0 + 4 kq + s, s = 0..3, for 4 MFMA steps
    // per rank tile.  A trip loads two groups before their products, so two groups' loads are in
    // flight together.
    auto load_group = [&](long long k0, T (&bv)[4], T (&av)[RT][4]) __attribute__((always_inline)) {
        const long long kb = k0 + 4 * kq;
        if (live_b && kb + 3 < k_end) {
            // 4 consecutive dofs (16-byte aligned pairs: ndof and kb are multiples of 4)
            const double2 s01 = *reinterpret_cast<const double2 *>(rs + kb);
            const double2 s23 = *reinterpret_cast<const double2 *>(rs + kb + 2);
            const double2 p01 = *reinterpret_cast<const double2 *>(rp + kb);
            const double2 p23 = *reinterpret_cast<const double2 *>(rp + kb + 2);
            bv[0] = (T)(ss[kb / K] * (s01.x - p01.x));
            bv[1] = (T)(ss[(kb + 1) / K] * (s01.y - p01.y));
            bv[2] = (T)(ss[(kb + 2) / K] * (s23.x - p23.x));
            bv[3] = (T)(ss[(kb + 3) / K] * (s23.y - p23.y));
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const long long k = kb + s;
                bv[s] = (live_b && k < k_end) ? (T)(ss[k / K] * (rs[k] - rp[k])) : T(0);
            }
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int rr = t * 16 + n;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const long long k = kb + s;
                av[t][s] = (rr < r && k < k_end) ? U_iso[(size_t)k * r + rr] : T(0);
            }
        }
    };
    auto product = [&](const T (&bv)[4], const T (&av)[RT][4]) __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[t] = mfma(av[t][s], bv[s], acc[t]);
    };
    for (long long k0 = k_begin; k0 < k_end; k0 += 32) {
        T bv0[4], av0[RT][4], bv1[4], av1[RT][4];
        load_group(k0, bv0, av0);
        const bool two = k0 + 16 < k_end;
        if (two) load_group(k0 + 16, bv1, av1);
        product(bv0, av0);
        if (two) product(bv1, av1);
    }
    // D[m][n]: m = rank offset within the tile, n = instance offset
    if (!live_b) return;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rk = t * 16 + drow<T>(kq, i);
            if (rk < r) ypart[((size_t)b * nsplit + split) * r + rk] = (double)acc[t][i];
        }
}

// The reduced system of every ROMSA instance, grid (r + ceil(r^2 / 256), B) x 256 threads:
//   blocks i < r:  y[b][i] = sum over the splits of ypart[b][split][i]  (each thread a fixed
//                  stride of splits, then a fixed-order tree in LDS: no dependence on scheduling)
//   later blocks:  A[b] = A0 + sum_k psi[b][k] A_k, one entry per thread
__global__ void __launch_bounds__(256) rom_assemble_kernel(int B, int r, int m, int nsplit,
                                                           const double *ypart, const double *A0,
                                                           const double *Ak, const double *psi,
                                                           const int *kind, int want, double *y,
                                                           double *A) {
    const int b = blockIdx.y;
    if (kind && kind[b] != want) return;
    const int t = threadIdx.x;
    if ((int)blockIdx.x < r) {
        __shared__ double sh[256];
        const int i = blockIdx.x;
        double s = 0.0;
        for (int k = t; k < nsplit; k += 256) s += ypart[((size_t)b * nsplit + k) * r + i];
        sh[t] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (t < h) sh[t] += sh[t + h];
            __syncthreads();
        }
        if (t == 0) y[(size_t)b * r + i] = sh[0];
        return;
    }
    const long long e = (long long)(blockIdx.x - r) * 256 + t;
    if (e >= (long long)r * r) return;
    double a = A0[e];
    for (int k = 0; k < m; ++k) a += psi[(size_t)b * m + k] * Ak[(size_t)k * r * r + e];
    A[(size_t)b * r * r + e] = a;
}

// one wave per instance: LU with partial pivoting of the assembled A; dc = A^{-1} y;
// singular -> status 1 and kind falls back to DSA (want -> 1).
__global__ void __launch_bounds__(64) rom_solve_kernel(int B, int r, const double *yv,
                                                       const double *Av, int *kind, int want,
                                                       int *status, double *dc, int *n_fallback) {
    __shared__ double A[64][65];
    __shared__ double y[64];
    __shared__ int piv_row;
    const int b = blockIdx.x;
    const int i = threadIdx.x;
    if (kind && kind[b] != want) return;
    if (i < r) {
        y[i] = yv[(size_t)b * r + i];
        for (int j = 0; j < r; ++j) A[i][j] = Av[((size_t)b * r + i) * r + j];
    }
    __syncthreads();
    // scale of A for the singularity test
    double amax = 0.0;
    if (i < r)
        for (int j = 0; j < r; ++j) amax = fmax(amax, fabs(A[i][j]));
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    bool singular = false;
    for (int k = 0; k < r; ++k) {
        // pivot: largest |A[i][k]| over i >= k, smallest index on ties
        double v = (i >= k && i < r) ? fabs(A[i][k]) : -1.0;
        int idx = i;
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(v, off, 64);
            const int oi = __shfl_xor(idx, off, 64);
            if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
        }
        if (i == 0) piv_row = idx;
        __syncthreads();
        const int pr = piv_row;
        if (!(v >= 1e-14 * amax) || v == 0.0) singular = true;
        if (pr != k) {
            if (i < r) {
                // swap rows k and pr column-wise: lane i handles column i
                const double t = A[k][i]; A[k][i] = A[pr][i]; A[pr][i] = t;
            }
            if (i == 0) { const double t = y[k]; y[k] = y[pr]; y[pr] = t; }
        }
        __syncthreads();
        if (!singular && i > k && i < r) {
            const double f = A[i][k] / A[k][k];
            A[i][k] = f;
            for (int j = k + 1; j < r; ++j) A[i][j] -= f * A[k][j];
            y[i] -= f * y[k];
        }
        __syncthreads();
    }
    if (singular) {
        if (i == 0) {
            if (status) status[b] = 1;
            if (kind) kind[b] = 1;           // this iteration falls back to DSA
            if (n_fallback) atomicAdd(n_fallback, 1);
        }
        return;
    }
    // back substitution (lane 0, r <= 64)
    if (i == 0) {
        for (int k = r - 1; k >= 0; --k) {
            double s = y[k];
            for (int j = k + 1; j < r; ++j) s -= A[k][j] * y[j];
            y[k] = s / A[k][k];
        }
        if (status) status[b] = 0;
    }
    __syncthreads();
    if (i < r) dc[(size_t)b * r + i] = y[i];
}

// delta[b][k] = sum_r U_rho[k][r] dc[b][r] for ROMSA instances; one wave per (16 dofs x 16
// instances) tile, looping over `tiles` consecutive dof tiles.
template <typename T>
__global__ void __launch_bounds__(64) rom_lift_kernel(long long ndof, int B, int r, int tiles,
                                                      const T *U_rho, const double *dc,
                                                      const int *kind, int want,
                                                      const int *status, double *delta) {
    typedef typename VecOf<T>::type V;
    const int lane = threadIdx.x;
    const int n = lane & 15, kq = lane >> 4;
    const int b0 = blockIdx.y * 16;
    const int b = b0 + n;
    // singular reduced systems (status 1) leave delta untouched
    const bool live_b = b < B && (!kind || kind[b] == want) && status[b] == 0;
    if (__builtin_amdgcn_ballot_w64(live_b) == 0) return;    // no ROMSA instance in the tile
    const int rpad = (r + 3) & ~3;
    // the B operand (this instance's reduced coefficients) is the same for every dof tile
    T bcol[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int kk = 4 * q + kq;
        bcol[q] = (live_b && kk < r) ? (T)dc[(size_t)b * r + kk] : T(0);
    }
    for (int t = 0; t < tiles; ++t) {
        const long long m0 = ((long long)blockIdx.x * tiles + t) * 16;
        if (m0 >= ndof) break;
        V acc = {0, 0, 0, 0};
        const long long mrow = m0 + n;          // A operand row (dof) of this lane
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (4 * q >= rpad) break;
            const int kk = 4 * q + kq;
            const T a = (mrow < ndof && kk < r) ? U_rho[(size_t)mrow * r + kk] : T(0);
            acc = mfma(a, bcol[q], acc);
        }
        if (live_b) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long dof = m0 + drow<T>(kq, i);
                if (dof < ndof) delta[(size_t)b * ndof + dof] = (double)acc[i];
            }
        }
    }
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// Reduced load of the ROM initial guess, split over cells like the projections:
//   ypart[b][split][k] = ghost * sum_{cells of the split} U_iso[cell K][k] G[b][cell]
//                        (+ sum_side g[b][side] b_in[side][k] in split 0),
// the isotropic source load being G sqrt(hx hy) on the cell-mean dof of every direction.
__global__ void __launch_bounds__(64) romig_load_kernel(long long ncell, int K, int r, int nsplit,
                                                        long long per_split, const double *U_iso,
                                                        const double *G, double ghost,
                                                        const double *inflow, const double *b_in,
                                                        double *ypart) {
    const int split = blockIdx.x, b = blockIdx.y, k = threadIdx.x;
    if (k >= r) return;
    const long long c0 = (long long)split * per_split;
    const long long c1 = c0 + per_split < ncell ? c0 + per_split : ncell;
    double s = 0.0;
    for (long long c = c0; c < c1; ++c) s += U_iso[(size_t)(c * K) * r + k] * G[(size_t)b * ncell + c];
    s *= ghost;
    if (split == 0)
        for (int side = 0; side < 4; ++side) s += inflow[4 * b + side] * b_in[side * r + k];
    ypart[((size_t)b * nsplit + split) * r + k] = s;
}

}  // namespace

size_t rom_split(const rte_problem *p, const rte_rom *rom) {
    // splits of 256 dofs (16 groups of 16): with 16-instance tiles a C2-sized batch gives about
    // 16 waves per compute unit.  The count depends on the mesh only, so an instance's reduced
    // load is summed in the same order whatever batch it is in.
    (void)rom;
    const long long n = (p->ndof + 255) / 256;
    return (size_t)(n < 1 ? 1 : n);
}

// reduced system assembly and its LU solve (both correction and initial guess)
void launch_rom_system(const rte_problem *p, const rte_rom *rom, const double *psi,
                       const int *kind, int want_kind, int *status, const RomSpace &w,
                       hipStream_t s) {
    const int r = rom->r;
    const unsigned ablk = cdiv((long long)r * r, 256);
    hipLaunchKernelGGL(rom_assemble_kernel, dim3(r + ablk, p->B), dim3(256), 0, s, p->B, r, rom->m,
                       w.nsplit, w.ypart, rom->d_A0, rom->d_A, psi, kind, want_kind, w.y, w.A);
    hipLaunchKernelGGL(rom_solve_kernel, dim3(p->B), dim3(64), 0, s, p->B, r, w.y, w.A,
                       const_cast<int *>(kind), want_kind, status, w.dc,
                       kind ? w.n_fallback : nullptr);
}

hipError_t launch_rom_initial_guess(const rte_problem *p, const rte_rom *rom, const double *psi,
                                    double *rho, int *status, const RomSpace &w, hipStream_t s) {
    const int r = rom->r;
    const int nsplit = w.nsplit;
    long long per_split = (p->ncell + nsplit - 1) / nsplit;
    hipLaunchKernelGGL(romig_load_kernel, dim3(nsplit, p->B), dim3(64), 0, s, p->ncell, p->K, r,
                       nsplit, per_split, rom->d_U_iso, p->source, sqrt(p->hx * p->hy),
                       p->inflow, rom->d_b_in, w.ypart);
    launch_rom_system(p, rom, psi, nullptr, 0, status, w, s);
    const int tiles = 4;
    dim3 gl(cdiv(p->ndof, 16 * tiles), cdiv(p->B, 16));
    hipLaunchKernelGGL(rom_lift_kernel<double>, gl, dim3(64), 0, s, p->ndof, p->B, r, tiles,
                       rom->d_U_rho, w.dc, (const int *)nullptr, 0, status, rho);
    return hipGetLastError();
}

hipError_t launch_rom_correct(const rte_problem *p, const rte_rom *rom, const double *psi,
                              const double *rho_star, const double *rho_prev, double *delta,
                              int *status, const int *kind, int want_kind, const RomSpace &w,
                              int fp32, hipStream_t s) {
    const int r = rom->r;
    const long long ndof = p->ndof;
    const int nsplit = w.nsplit;
    long long per_split = (ndof + nsplit - 1) / nsplit;
    per_split = (per_split + 15) / 16 * 16;
    dim3 gp(nsplit, cdiv(p->B, 16));
    const int rt = (r + 15) / 16;                      // 1..4 rank tiles (r <= 64)
    if (fp32) {
        auto *k = rt == 1 ? rom_project_kernel<float, 1> : rt == 2 ? rom_project_kernel<float, 2>
                : rt == 3 ? rom_project_kernel<float, 3> : rom_project_kernel<float, 4>;
        hipLaunchKernelGGL(k, gp, dim3(64), 0, s, ndof, p->K, p->B, r, nsplit, per_split,
                           rom->d_U_iso_f, p->sigma_s, rho_star, rho_prev, kind, want_kind, w.ypart);
    } else {
        auto *k = rt == 1 ? rom_project_kernel<double, 1> : rt == 2 ? rom_project_kernel<double, 2>
                : rt == 3 ? rom_project_kernel<double, 3> : rom_project_kernel<double, 4>;
        hipLaunchKernelGGL(k, gp, dim3(64), 0, s, ndof, p->K, p->B, r, nsplit, per_split,
                           rom->d_U_iso, p->sigma_s, rho_star, rho_prev, kind, want_kind, w.ypart);
    }
    // the solve may turn `want` instances into DSA ones (kind is written); the lift then skips them
    launch_rom_system(p, rom, psi, kind, want_kind, status, w, s);
    const int tiles = 4;
    dim3 gl(cdiv(ndof, 16 * tiles), cdiv(p->B, 16));
    if (fp32)
        hipLaunchKernelGGL(rom_lift_kernel<float>, gl, dim3(64), 0, s, ndof, p->B, r, tiles,
                           rom->d_U_rho_f, w.dc, kind, want_kind, status, delta);
    else
        hipLaunchKernelGGL(rom_lift_kernel<double>, gl, dim3(64), 0, s, ndof, p->B, r, tiles,
                           rom->d_U_rho, w.dc, kind, want_kind, status, delta);
    return hipGetLastError();
}

}  // namespace rte
