// Internal declarations of the gfx950 RTE library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "rte.h"

namespace rte {

// Direction entry of the quadrant-sorted direction table used by the 2D sweep.
// alpha = |v_x| / h_x, beta = |v_y| / h_y; w = 0 marks a padding entry.
struct DirEntry {
    double alpha;
    double beta;
    double w;
    int orig;   // index in the caller's direction order, -1 for padding
    int pad;
};

constexpr int kQuadPad = 16;
constexpr int kMaxMat = 16;    // materials (distinct sigma_t) of an instance swept from its table   // each quadrant's block of the sorted table is padded to this multiple

// Per-quadrant layout of the sorted direction table.
struct QuadLayout {
    int start[4];   // first sorted entry of quadrant q (q = (vx<0) | 2 (vy<0))
    int count[4];   // directions in quadrant q
};

struct Tuning {
    int dg;         // directions per lane in the 2D sweep (1, 2, 4, 8, 16)
    int wpb;        // waves per band in a 2D sweep workgroup (direction groups summed in LDS)
    int bands;      // bands of the mesh in flight per 2D sweep workgroup (1: one after another)
};
// LDS a 2D sweep workgroup may use (partial-sum buffers and y-trace rings)
constexpr size_t kSweepLdsBytes = 64 * 1024;

struct Workspace;   // carve-up of the caller's workspace, see rte_api.hip

}  // namespace rte

struct rte_problem {
    int dim, nx, ny, B, n_dir, K;
    long long ncell, ndof;
    double hx, hy, lx, ly;
    std::vector<double> vx, vy, w, widths;
    // angular moments of the direction set
    double cxx, cyy;          // sum w vx^2, sum w vy^2
    double kmin_x, kmin_y;    // sum_{vx>0} w vx, sum_{vy>0} w vy
    double c1, c2, c3;        // 1D: sum_{mu>0} w mu, sum w mu^2, sum_{mu>0} w mu^3
    const double *sigma_t, *sigma_s, *source, *inflow;
    rte::QuadLayout quad;
    rte::Tuning tune;
    int n_sorted;
    rte::DirEntry *d_dirs;    // device [n_sorted]
    double *d_mu;             // 1D: device [n_dir] directions
    double *d_w;              // device [n_dir] weights (caller order)
    double *d_widths;         // 1D: device [nx]
    double *d_vxy;            // 2D: device [2][n_dir] directions in caller order
    int dsa_mg;               // 2D diffusion CG preconditioner: 1 multigrid, 0 block-Jacobi
    int n_cu;                 // compute units of the device the handle was created on
    int lds_per_cu;           // bytes of LDS per compute unit (and per workgroup)
    int nparts() const;       // 2D sweep partial-sum slots per instance for the current tuning
    // the outer iteration of rte_sisa_solve / rte_sisa_iterate captured as a HIP graph for the
    // last (workspace, arguments) it was used with; owned by the handle (rte_api.hip)
    mutable struct rte_iter_graph *iter_graph;
    // the multigrid preconditioner of the 2D diffusion CG captured as HIP graphs for the last
    // workspace carve-up it was used with; owned by the handle (rte_api.hip)
    mutable struct rte_precond_graphs *precond_graphs;
};

namespace rte {
// Diagonal-major cell layouts of the 2D sweep.  A wavefront of the sweep visits, at every step,
// cells of one anti-diagonal x + y = const (quadrants (+,+), (-,-)) or of one diagonal
// x - y = const (quadrants (-,+), (+,-)) in consecutive rows; storing the per-cell sweep inputs
// and outputs diagonal by diagonal, row-ascending, makes those accesses contiguous.
//   layout A: d = x + y,            row range y in [max(0, d-nx+1), min(d, ny-1)]
//   layout B: d = x - y + ny - 1,   row range y in [max(0, ny-1-d), min(ny-1, nx+ny-2-d)]
// cells on the diagonals before diagonal d of an nx x ny grid: diagonal d holds
// min(d + 1, m, nx + ny - 1 - d) cells (m = min(nx, ny), M = max(nx, ny)); the same count for
// anti-diagonals (x + y = d) and diagonals (x - y + ny - 1 = d).  Arithmetic only, so a sweep
// step never waits on a memory load for its position.
// With len(e) = (e + 1) - max(0, e + 1 - m) - max(0, e + 1 - M), the count is
// tri(d) - tri(d - m) - tri(d - M) for tri(x) = x (x + 1) / 2 on x > 0 and 0 otherwise: no branch,
// so the lanes of a sweep step that sit in different parts of the grid do not diverge.
__host__ __device__ __forceinline__ int tri_pos(int x) {
    x = x > 0 ? x : 0;
    return (x * (x + 1)) >> 1;
}
__host__ __device__ __forceinline__ int diag_off(int nx, int ny, int d) {
    const int m = nx < ny ? nx : ny, M = nx < ny ? ny : nx;
    return tri_pos(d) - tri_pos(d - m) - tri_pos(d - M);
}
__host__ __device__ __forceinline__ int pos_a(int nx, int ny, int x, int y) {
    const int d = x + y;
    const int ylo = d - nx + 1 > 0 ? d - nx + 1 : 0;
    return diag_off(nx, ny, d) + y - ylo;
}
__host__ __device__ __forceinline__ int pos_b(int nx, int ny, int x, int y) {
    const int d = x - y + ny - 1;
    const int ylo = ny - 1 - d > 0 ? ny - 1 - d : 0;
    return diag_off(nx, ny, d) + y - ylo;
}
// The (anti)diagonal holding position pos: the largest d with diag_off(d) <= pos (bisection).
__host__ __device__ __forceinline__ int diag_at(int nx, int ny, int pos) {
    int lo = 0, hi = nx + ny - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (diag_off(nx, ny, mid) <= pos) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
// Inverse of pos_a / pos_b: the natural cell index y * nx + x at position pos.
__host__ __device__ __forceinline__ int cell_at(int nx, int ny, int pos, bool layout_a) {
    const int d = diag_at(nx, ny, pos);
    const int k = pos - diag_off(nx, ny, d);
    if (layout_a) {
        const int ylo = d - nx + 1 > 0 ? d - nx + 1 : 0;
        const int y = ylo + k;
        return y * nx + (d - y);
    }
    const int ylo = ny - 1 - d > 0 ? ny - 1 - d : 0;
    const int y = ylo + k;
    return y * nx + (d + y - ny + 1);
}
// Storage order of the 2D angular flux, in a direction's reflected coordinates (x', y') (the
// frame in which its sweep runs +x, +y): the 64-row bands of the sweep one after the other, each
// band (nx x h cells, h = min(64, ny - 64 k)) in its own anti-diagonal order (pos_a of that
// band).  A wavefront of the sweep writes one band diagonal per step, right after the one of its
// previous step, so its writes run through memory sequentially.
__host__ __device__ __forceinline__ int band_pos(int nx, int ny, int x, int y) {
    const int k = y >> 6, r = y & 63;
    const int h = ny - 64 * k < 64 ? ny - 64 * k : 64;
    return 64 * nx * k + pos_a(nx, h, x, r);
}
// Inverse of band_pos: y' * nx + x' of the cell at position pos.
__host__ __device__ __forceinline__ int band_cell(int nx, int ny, int pos) {
    const int k = pos / (64 * nx);
    const int h = ny - 64 * k < 64 ? ny - 64 * k : 64;
    const int c = cell_at(nx, h, pos - 64 * nx * k, true);
    return (64 * k + c / nx) * nx + c % nx;
}
// Natural cell index of the reflected cell index c' = y' * nx + x' of quadrant q.
__host__ __device__ __forceinline__ int unreflect(int nx, int ny, int c, int q) {
    const int yr = c / nx, xr = c - yr * nx;
    const int x = (q & 1) ? nx - 1 - xr : xr, y = (q & 2) ? ny - 1 - yr : yr;
    return y * nx + x;
}

// quadrant q = (vx<0) | 2 (vy<0): q = 0, 3 sweep anti-diagonals (layout A), q = 1, 2 diagonals (B)
__device__ __forceinline__ bool quad_uses_a(int q) { return q == 0 || q == 3; }

template <typename T>
struct Vec4 { T x, y, z, w; };

// Logical block (x, y) of a 2D grid (x: cells or vertices of an instance, y: instance),
// renumbered for the XCDs.  The hardware hands workgroups to the 8 XCDs in turn by linear id
// (x fastest), and each XCD has its own L2.  When the row of blocks is a multiple of 8 long,
// XCD k takes the k-th eighth of every instance's blocks: the neighbouring rows that a block
// gathers are then mostly loaded by blocks of its own XCD, and every XCD still works on every
// instance (instances that stop early leave the load balanced).  Any one-to-one renumbering is
// correct; otherwise the numbering is left as it is.
struct Blk {
    int x, y;
};
__device__ __forceinline__ Blk xcd_block() {
    const unsigned gx = gridDim.x;
    Blk o;
    o.y = (int)blockIdx.y;
    if (gx & 7u) {
        o.x = (int)blockIdx.x;
        return o;
    }
    o.x = (int)((blockIdx.x & 7u) * (gx >> 3) + (blockIdx.x >> 3));
    return o;
}

// sweep input block from rho (2D: both diagonal layouts and sigma_t; 1D: natural order)
template <typename T>
__device__ __forceinline__ void write_sweep_input(int dim, long long ncell, int B, int b, int nx,
                                                  int ny, long long cell, const double v[4], double st,
                                                  T *src) {
    if (dim == 1) {
        T *o = src + ((size_t)b * ncell + cell) * 2;
        o[0] = (T)v[0];
        o[1] = (T)v[1];
        return;
    }
    const int x = (int)(cell % nx), y = (int)(cell / nx);
    const size_t nb4 = (size_t)B * ncell * 4;
    const size_t pa = (size_t)b * ncell + pos_a(nx, ny, x, y);
    const size_t pb = (size_t)b * ncell + pos_b(nx, ny, x, y);
    Vec4<T> o;
    o.x = (T)v[0]; o.y = (T)v[1]; o.z = (T)v[2]; o.w = (T)v[3];
    *reinterpret_cast<Vec4<T> *>(src + pa * 4) = o;
    *reinterpret_cast<Vec4<T> *>(src + nb4 + pb * 4) = o;
    src[2 * nb4 + pa] = (T)st;
    src[2 * nb4 + (size_t)B * ncell + pb] = (T)st;
}

}  // namespace rte

struct rte_rom {
    int r, m;
    long long ndof;
    double eps_pod, eps_train;
    double *d_U_rho;   // device [ndof][r]
    double *d_U_iso;   // device [ndof][r]
    float *d_U_rho_f;  // device [ndof][r] (FP32 copy for the mixed-precision projections)
    float *d_U_iso_f;
    double *d_A0;      // device [r][r]
    double *d_A;       // device [m][r][r]
    double *d_b_in;    // device [4][r] reduced unit-inflow loads (zeros when not given)
    unsigned long long serial;   // distinct for every ROM created in the process
};

// ---------------------------------------------------------------------------------------------
// kernel launchers (defined in the .hip files); all return hipError_t of the launch
// ---------------------------------------------------------------------------------------------
namespace rte {

// 2D sweep input block (one allocation, T = float or double):
//   srcA [B][ncell][4], srcB [B][ncell][4]  sigma_s rho + G sqrt(hx hy) delta_k0 in layouts A, B
//   sigA [B][ncell],    sigB [B][ncell]     sigma_t in layouts A, B (an instance with a
//                                           material table: the cell's material index)
// 1D: src [B][ncell][2] in natural order.
struct SweepLaunch {
    const rte_problem *p;
    const void *src;          // sweep input block (see above)
    double *partial;          // [B][nparts][ndof] or nullptr
    void *f_out;              // [B][ncell][n_dir][K] T or nullptr
    const int *active;        // [B] or nullptr
    int zero_inflow;
    int fp32;
    int bands = 0;            // bands in flight (0: the handle's schedule); results do not depend on it
    // material tables (launch_materials; both null: every instance by the per-cell kernel)
    const int *mat_ok = nullptr;      // [B] 1: swept by the table kernel
    const void *mat_coef = nullptr;   // [B][n_sorted][kMaxMat][8] T
};
hipError_t launch_sweep2d(const SweepLaunch &a, hipStream_t s);
// Per instance (mask[b] != 0, all if null): the distinct sigma_t values (vals [B][kMaxMat]
// ascending, nmat [B]), each cell's index among them (mat [B][ncell]), mat_ok [B] = 1 when there
// are at most kMaxMat and every cell has one, and the cell-solve coefficients of every (sorted
// direction, material) in T (coef [B][n_sorted][kMaxMat][8]); cvals [B][mat_chunks][kMaxMat + 1]
// is scratch.
int mat_chunks(const rte_problem *p);
hipError_t launch_materials(const rte_problem *p, const int *mask, int *mat, int *mat_ok,
                            int *nmat, double *vals, double *cvals, void *coef, int fp32,
                            hipStream_t s);
// LDS bytes a table kernel adds to a sweep workgroup (elem: sizeof T), and whether the table
// kernels fit the device's LDS for every launch of the handle's schedule
size_t sweep_mat_lds_bytes(const rte_problem *p, size_t elem);
bool sweep_mat_fits(const rte_problem *p, size_t elem);
// dynamic LDS limit of every 2D sweep kernel (once per process)
void sweep_lds_limits(int bytes);
// wavefronts per sweep workgroup (direction groups summed in LDS) and partial slots per instance
int sweep_waves(const rte_problem *p);
int sweep_bands(const rte_problem *p);
// bands a 2D sweep launch runs in flight for a request (clamped to the mesh's bands, 1024 threads
// and the LDS budget for partial sums (if any) and rings of elem-byte values); the number a solve
// of precision prec uses
int bands_in_flight(const rte_problem *p, int requested, bool partial, size_t elem);
// LDS bytes of a per-cell sweep workgroup with `bands` in flight
size_t sweep_lds_bytes(const rte_problem *p, int bands, bool partial, size_t elem);
int sweep_bands_used(const rte_problem *p, rte_precision prec);
int sweep_nparts(const rte_problem *p);

// 1D sweep: writes f (always, T) to f_out [B][ncell][n_dir][2]; src as in 2D (K = 2).
hipError_t launch_sweep1d(const rte_problem *p, const void *src, void *f_out, const int *active,
                          int zero_inflow, int fp32, hipStream_t s);

// sweep input block from rho: src = sigma_s rho + G * (cell integral of phi_0), plus sigma_t, or
// for instances with mat_ok[b] != 0 (mat, mat_ok from launch_materials, nullable) the material
// index (with_G false: src = sigma_s rho, the source of L rho)
hipError_t launch_source(const rte_problem *p, const double *rho, void *src, const int *active,
                         int fp32, hipStream_t s, bool with_G = true, const int *mat = nullptr,
                         const int *mat_ok = nullptr);

// rho = sum of nparts partial slots (fixed order); optional change/magnitude maxima per instance
hipError_t launch_reduce_parts(const rte_problem *p, const double *partial, int nparts,
                               double *rho_star, const double *rho_prev, unsigned long long *maxd,
                               unsigned long long *maxr, const int *active, hipStream_t s);

// rho = sum_j w_j f_j over f [B][n_dir][ndof]
hipError_t launch_scalar_flux(const rte_problem *p, const void *f, double *rho, int fp32,
                              const double *rho_prev, unsigned long long *maxd,
                              unsigned long long *maxr, const int *active, hipStream_t s);

hipError_t launch_check_materials(const rte_problem *p, int *bad, hipStream_t s);

// diffusion corrections
// scratch: [B][nx][20] doubles
hipError_t launch_dsa1d(const rte_problem *p, const double *rho_star, const double *rho_prev,
                        double *delta, const int *kind, int want_kind, double *scratch,
                        hipStream_t s);

// vertex-grid hierarchy of the multigrid preconditioner of the 2D diffusion CG
constexpr int kMaxLevels = 12;
struct MGLevel {
    int nvx, nvy;          // vertices per axis
    long long nv;
    double *S;             // [B][kStencilPlanes][nv] Galerkin stencils (built in FP64)
    float *S32;            // the same rounded to FP32, read by the V-cycle of the CG
    double *xa, *xb, *bv, *rv;   // [B][nv]
};
struct MGSpace {
    int L;                 // number of vertex levels (0 = multigrid off: block-Jacobi PCG)
    MGLevel lv[kMaxLevels];
    double *t;             // [B][ndof] DG scratch
    double *e;             // [B][nv0] probe vector
    double *cinv;          // [B][nc][nc] inverse of the coarsest operator (nc = its vertices),
                           // when nc <= kDirectCoarse; null otherwise (damped Jacobi sweeps)
};
// coarsest vertex grids up to this many vertices are solved exactly (dense inverse per instance)
constexpr int kDirectCoarse = 60;     // its inversion holds 2 nc^2 + nc doubles in LDS (< 64 KiB)
// levels for an nx x ny mesh (0 when the mesh is too small for a coarse space)
int mg_levels(int nx, int ny, int *nvx, int *nvy);

// planes per instance of a vertex-grid operator: the 9 stencil entries and omega / diagonal
constexpr int kStencilPlanes = 10;

struct CGSpace {
    MGSpace mg;
    double *cf;                        // [B][5][ncell] per-cell operator data (2D)
    float *binv;                       // [B][10][ncell] inverse diagonal blocks (2D), FP32: the
                                       // smoother's data (the operator stays FP64)
    double *x, *r, *z, *p0, *p1, *q;   // [B][ndof]
    double *part;                      // [B][5][nblk] partial sums
    double *scal;                      // [B][8] per-instance scalars
    int *iters;                        // [B]
    int *state;                        // [B] 0 idle, 1 running, 2 converged, 3 failed
    int *n_running;                    // [2] instances still iterating; instances that failed
                                       // (limit reached or a NaN) in the current call
    int *fails;                        // [1] or null: instances that stopped without converging,
                                       // summed over every call until the caller clears it
    double *tol2;                      // [1] the call's squared relative tolerance
    int nblk;                          // blocks per instance
    int zf32;                          // 1: z and the multigrid residual t held in FP32 (mixed
                                       // precision with the multigrid preconditioner; the
                                       // buffers keep their FP64 size), and the preconditioner
                                       // applies the operator with cf32
    float *cf32;                       // [B][5][ncell] cf rounded to FP32 (zf32 only, else null)
    // the multigrid preconditioner's launches captured as HIP graphs, one per parity slot of
    // its (r, z) partial sums (null: launched one by one); valid for this carve-up only
    hipGraphExec_t precond[2] = {nullptr, nullptr};
};
// CG start for the instances with kind == want_kind (all if kind is null); guess (nullable)
// is the previous correction, used as a search direction for the initial iterate
hipError_t launch_cg_setup(const rte_problem *p, const CGSpace &c, const double *rho_star,
                           const double *rho_prev, const int *kind, int want_kind,
                           const double *guess, double rtol, hipStream_t s);
// per-cell operator data, inverse diagonal blocks and (multigrid) the Galerkin vertex operators
// of the instances with mask[b] == 1 (all if mask is null); once per solve, before any CG call
hipError_t launch_dsa_build(const rte_problem *p, const CGSpace &c, const int *mask,
                            hipStream_t s);
// z = M^-1 r and the partial sums of (r, z) in parity slot `slot`
hipError_t launch_mg_precond(const rte_problem *p, const CGSpace &c, int slot, hipStream_t s);
hipError_t launch_cg_iteration(const rte_problem *p, const CGSpace &c, int it, double rtol,
                               int maxit, hipStream_t s);
// Captures the multigrid preconditioner (after launch_dsa_build) into c.precond; on any failure
// c.precond stays null and the kernels are launched one by one.  mg_precond_release frees them.
void mg_precond_capture(const rte_problem *p, CGSpace &c);
void mg_precond_release(CGSpace &c);
// delta = x for the instances of the call; iters_out[b] (nullable) and *total (nullable, summed)
// receive the iteration counts
hipError_t launch_cg_finish(const rte_problem *p, const CGSpace &c, double *delta, int *iters_out,
                            unsigned long long *total, hipStream_t s);
size_t cg_blocks_per_instance(const rte_problem *p);

// ROM correction
struct RomSpace {
    double *y;        // [B][r] reduced load
    double *A;        // [B][r][r] reduced operator A0 + sum_k psi_k A_k
    double *ypart;    // [B][nsplit][r] split-K partials
    double *dc;       // [B][r]
    int nsplit;
    int *n_fallback;  // [1] or null: incremented for every instance whose reduced system is
                      // singular (sent to DSA for the iteration)
};
hipError_t launch_rom_correct(const rte_problem *p, const rte_rom *rom, const double *psi,
                              const double *rho_star, const double *rho_prev, double *delta,
                              int *status, const int *kind, int want_kind, const RomSpace &w,
                              int fp32, hipStream_t s);
size_t rom_split(const rte_problem *p, const rte_rom *rom);
// ROM initial guess: rho = U^rho c, (A0 + sum psi_k A_k) c = (U^iso)^T q_G + sum g_side b_in[side]
hipError_t launch_rom_initial_guess(const rte_problem *p, const rte_rom *rom, const double *psi,
                                    double *rho, int *status, const RomSpace &w, hipStream_t s);

// DSA-preconditioned restarted GMRES (krylov.hip); per-instance FP64 state
struct GmresSpace {
    int m;                 // restart length
    int nblk;              // reduction blocks per instance
    int nslot, normslot;   // partial / coefficient slots per instance: m + 2, the last for |w|^2
    double *V;             // [m+1][B][ndof] Krylov basis
    double *w, *t, *u, *bbar, *lv;   // [B][ndof]
    double *part;          // [B][nslot][nblk]
    double *h, *h2;        // [B][nslot] Gram-Schmidt coefficients of the two passes
    double *H;             // [B][m+1][m] Hessenberg matrix (rotated)
    double *cs, *sn, *y;   // [B][m]
    double *g;             // [B][m+1] rotated residual vector
    double *nb;            // [B] |M^-1 b_bar|
    double *est;           // [B] estimated relative residual of the last step
    double *wn;            // [B] norm of the newest orthogonalized vector
    int *act;              // [B] 1 while the instance's solve runs
    int *cyc;              // [B] 1 while it extends its Krylov space in the current cycle
    int *kused;            // [B] steps of the current cycle
    int *n_sweep, *n_iter; // [B]
    int *count;            // [1] instances still extending (host reads it)
};
int gmres_blocks(const rte_problem *p);
hipError_t gm_dots(const rte_problem *p, const GmresSpace &g, int nv, const double *X,
                   const double *w, const int *flag, double *dst, int accumulate, hipStream_t s);
hipError_t gm_resum(const rte_problem *p, const GmresSpace &g, int nv, const int *flag,
                    double *dst, int accumulate, hipStream_t s);
hipError_t gm_axpy(const rte_problem *p, const GmresSpace &g, int nv, const double *X,
                   const double *c, int cstride, double sign, double *w, const int *flag,
                   bool norm, hipStream_t s);
hipError_t gm_lincomb(const rte_problem *p, const double *a, const double *x, double sa,
                      const double *y, double sb, double *out, const int *flag, hipStream_t s);
hipError_t gm_norm(const rte_problem *p, const GmresSpace &g, const double *w, const int *flag,
                   hipStream_t s);
hipError_t gm_sqrt_norm(const rte_problem *p, const GmresSpace &g, const int *flag, double *out,
                        hipStream_t s);
hipError_t gm_scale(const rte_problem *p, const GmresSpace &g, const double *w, const double *sv,
                    int sstride, int sslot, double *out, const int *flag, hipStream_t s);
hipError_t gm_cycle_start(const rte_problem *p, const GmresSpace &g, double tol, hipStream_t s);
hipError_t gm_givens(const rte_problem *p, const GmresSpace &g, int i, double tol, hipStream_t s);
hipError_t gm_solve(const rte_problem *p, const GmresSpace &g, hipStream_t s);
hipError_t gm_count_sweep(const rte_problem *p, const GmresSpace &g, const int *flag,
                          hipStream_t s);

// Alg. 1 / Alg. 2 bookkeeping
struct IterState {
    unsigned long long *maxd, *maxr;   // [B]
    int *active;                       // [B] 1 while iterating
    int *kind;                         // [B] correction chosen after the current sweep
    int *n_sweep;                      // [B]
    int *status;                       // [B]
    double *change;                    // [B][max_iter]
    int *kinds;                        // [B][max_iter]
    int *n_active;                     // [3] after a decision: instances still iterating,
                                       // taking DSA, taking ROMSA
};
// stop test and choice of correction after every active instance's latest sweep
hipError_t launch_decide(const rte_problem *p, const IterState &st, int max_iter, double eps,
                         int relative, int mode, int theta, double eps_romsad, hipStream_t s);
// rho = rho* + delta (delta may be null) for instances corrected at iteration l; converged
// instances keep rho* ; then src for the next sweep.
hipError_t launch_update(const rte_problem *p, const IterState &st, const double *rho_star,
                         const double *delta, double *rho, void *src, int fp32, hipStream_t s);
// start (run = 1) or idle (run = 0) the instances with mask[b] != 0 (all if mask is null)
hipError_t launch_init_state(const rte_problem *p, const IterState &st, int max_iter,
                             const int *mask, int run, hipStream_t s);
hipError_t launch_zero(double *x, long long n, hipStream_t s);
// x[b][:] = 0 for the rows with mask[b] != 0 (every row if mask is null), x is [B][n]
hipError_t launch_zero_rows(double *x, int B, long long n, const int *mask, hipStream_t s);
hipError_t launch_fill_int(int *x, long long n, int v, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *x, long long n, hipStream_t s);

}  // namespace rte
