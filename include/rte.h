/*
 * rte.h -- C ABI of the MI355X (gfx950) library for the S_N upwind-DG radiative
 * transfer equation with source iteration and synthetic acceleration.
 *
 * Method: Z. Peng, "Reduced Order Model Enhanced Source Iteration with Synthetic
 * Acceleration for Parametric Radiative Transfer Equation" (arXiv 2402.10488).
 *
 * Problem statement (Sec. 2, eq. (rte), slab form eq. (slab_geometry)):
 *   v . grad f + sigma_t f = sigma_s rho + G,  rho = sum_j w_j f(., v_j),
 *   f = g on the inflow boundary,  sigma_t >= sigma_s >= 0,  sum_j w_j = 1.
 * Discretization (Sec. 2.2): upwind DG with K = 1 (P1 in 1D, Q1 in 2D) in the
 * orthonormal Legendre basis, eq. (dg_matrix_vec).
 *
 * Conventions shared by every entry point
 *  - Data layout (all row-major, C order):
 *      cell index       c = iy * nx + ix            (1D: c = ix)
 *      local dof        k = a + 2 b                 (a: x-degree, b: y-degree); K = 4 in 2D,
 *                                                   K = 2 in 1D (k = a)
 *      rho, delta_rho   [B][N_DOF], N_DOF = nx * ny * K
 *      angular flux f   2D: [B][n_dir][ncell][4] in sweep order: the cells of direction j
 *                       are stored in the order its sweep visits them, so that the sweep
 *                       writes them sequentially.  Reflect to the sweep's frame,
 *                         x' = x (vx_j >= 0) or nx-1-x (vx_j < 0),  y' likewise with vy_j, ny;
 *                       cut y' into bands of 64 rows, k = floor(y'/64), r = y' - 64k, band height
 *                       h = min(64, ny - 64k); within a band order by anti-diagonal d = x' + r,
 *                       then by r.  Cell (x, y) of direction j is stored at position
 *                         64 nx k + T(d) + r - max(0, d - nx + 1),
 *                       where, with m = min(nx, h), M = max(nx, h), T(d) counts the cells of the
 *                       band's anti-diagonals before d:
 *                         T(d) = d(d+1)/2                                     d <= m
 *                              = m(m+1)/2 + (d-m) m                           m < d <= M
 *                              = m(m+1)/2 + (M-m) m + e(m-1) - e(e-1)/2,      e = d - M > 0.
 *                       rte_f_natural converts to [B][n_dir][N_DOF] in natural cell order
 *                       (the paper's f_j is then row j).
 *                       1D: [B][ncell][n_dir][2] (per cell and direction the 2 coefficients).
 *      materials        [B][ny][nx]  cell-constant sigma_t, sigma_s, G
 *      inflow           [B][4]  isotropic g on the sides x=0, x=Lx, y=0, y=Ly (1D: first two)
 *  - Basis: on a cell of size hx x hy, phi_ab = L_a(xi) L_b(eta) / sqrt(hx hy) with
 *    L_0 = 1, L_1 = sqrt(3) t on [-1, 1]; a constant c has coefficients (c sqrt(hx hy), 0, 0, 0).
 *  - Every device pointer is caller-owned device memory (hipMalloc / torch), FP64
 *    unless stated.  Host pointers are read during the call only.
 *  - Hot calls (sweep, scalar flux, corrections, solve) allocate no device memory;
 *    they use the caller's workspace (rte_workspace_size).  Handle creation copies
 *    small tables (directions, cell widths, reduced operators) to the device.
 *  - Calls enqueue on the given stream and return without synchronizing, except
 *    rte_sisa_solve, which polls small device flags and fills host statistics.
 *  - Every function returns an rte_status; no exception crosses the ABI.  Argument
 *    errors are detected on the host before any device work is enqueued.
 *  - Handles are immutable after creation; concurrent calls on different streams
 *    are allowed when their outputs and workspaces are disjoint.
 */
#ifndef RTE_H
#define RTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *rte_stream_t;   /* hipStream_t */

typedef enum {
    RTE_OK = 0,
    RTE_EINVAL = 1,        /* invalid argument (shape, NULL, sigma_t < sigma_s, weights, ...) */
    RTE_ENOCONV = 2,       /* iteration limit reached; rho holds the last rho^(l,*) */
    RTE_ESINGULAR = 3,     /* a reduced ROM system was singular (instance fell back to DSA) */
    RTE_ECG = 4,           /* diffusion CG did not reach its tolerance within its limit */
    RTE_ENOMEM = 5,        /* workspace too small */
    RTE_EDEVICE = 6,       /* a HIP runtime call failed */
    RTE_EUNSUPPORTED = 7   /* valid but unsupported configuration */
} rte_status;

typedef enum {
    RTE_FP64 = 0,          /* every kernel in FP64 */
    RTE_MIXED = 1          /* FP32 sweep and ROM projections; FP64 accumulation of rho, FP64
                              diffusion CG, reduced LU, norms and switch test */
} rte_precision;

typedef enum { RTE_SI = 0, RTE_SI_DSA = 1, RTE_ROMSAD = 2 } rte_mode;

typedef struct rte_problem rte_problem;
typedef struct rte_rom rte_rom;

/* Problem description: mesh, direction set and per-instance materials of a batch of B
 * independent instances that share mesh and directions (Sec. 2.1-2.2). */
typedef struct {
    int dim;                  /* 1 (slab) or 2 (X-Y) */
    int nx, ny;               /* cells per axis; ny = 1 when dim == 1 */
    int batch;                /* B >= 1 */
    int n_dir;                /* N_v >= 1 (1D: >= 1; 2D: any set, no direction with vx = vy = 0) */
    double lx, ly;            /* 2D: domain [0,lx] x [0,ly], uniform mesh */
    const double *widths;     /* 1D: host [nx] cell widths (> 0), may be non-uniform; NULL in 2D */
    const double *dir_x;      /* host [n_dir]: v_x (1D: mu) */
    const double *dir_y;      /* host [n_dir]: v_y; NULL in 1D */
    const double *weight;     /* host [n_dir]: w_j > 0, sum_j w_j = 1 (normalized rule, Sec. 2.1) */
    const double *sigma_t;    /* device [B][ny][nx] */
    const double *sigma_s;    /* device [B][ny][nx], 0 <= sigma_s <= sigma_t */
    const double *source;     /* device [B][ny][nx]  isotropic G */
    const double *inflow;     /* device [B][4]       isotropic inflow g per side */
} rte_problem_desc;

/* Creates a problem handle.  Validates host data; device arrays are checked by
 * rte_problem_check.  The device arrays must stay valid for the handle's lifetime. */
int rte_problem_create(const rte_problem_desc *desc, rte_problem **out);
void rte_problem_destroy(rte_problem *p);

/* rte_problem_create with an explicit 2D sweep schedule (used by the autotuner): dg directions
 * of one quadrant per lane (1, 2, 4, 8; 0 = automatic) and wpb wavefronts per workgroup
 * (1..4; 0 = automatic).  Results do not depend on the schedule beyond FP rounding of the
 * partial-density order. */
int rte_problem_create_tuned(const rte_problem_desc *desc, int dg, int wpb, rte_problem **out);

/* rte_problem_create_tuned with the number of mesh bands (64 rows each) a 2D sweep workgroup
 * keeps in flight: 1 sweeps the bands one after another; b > 1 runs b consecutive bands at once,
 * each 64 pipeline steps behind the one above, which cuts the dependent steps of an instance
 * from about nbands * nx to about nx + 64 nbands (a single large instance, or the last
 * iterations of a batch, run that many times more wavefronts).  The cells, solves and sums are
 * the same, so results are bitwise independent of bands.  0 = automatic: 1 when the batch has
 * at least 4096 wavefronts of work (16 per CU), 2 below that, and 4 below 1024 (where an
 * automatic wpb also drops to 2).  The launch uses fewer when the mesh has fewer bands, or
 * 64 wpb bands threads or the workgroup's LDS (partial sums and y-trace rings, 64 KiB) would not
 * fit.  bands in [0, 16].  rte_problem_create and rte_problem_create_tuned choose bands
 * automatically. */
int rte_problem_create_sched(const rte_problem_desc *desc, int dg, int wpb, int bands,
                             rte_problem **out);

/* Autotuner measurement: times the 2D sweep (source prologue, sweep, partial-density reduction:
 * one iteration's sweep of rte_sisa_solve; with f_out != NULL the angular flux is written too, as
 * rte_sweep does) of the batch described by desc under each candidate schedule (dg[i], wpb[i],
 * bands[i]) of rte_problem_create_sched (bands NULL: 1 band in flight).  ms_out[i] receives the average milliseconds per sweep over `reps`
 * timed sweeps after `warmup` untimed ones (HIP events on the stream), or -1 for a candidate the
 * library does not run as given (unknown values, or one the LDS budget or the mesh would
 * change: for bands, the number a solve in precision prec would run).
 *   rho_in   device [B][N_DOF] density swept;  f_out  device angular flux (layout above) or NULL
 * A setup call, not a hot one: it creates a handle and allocates and frees a workspace per
 * candidate, and synchronizes the stream.  2D only (RTE_EUNSUPPORTED otherwise). */
int rte_tune_sweep(const rte_problem_desc *desc, rte_precision prec, int n_cand, const int *dg,
                   const int *wpb, const int *bands, const double *rho_in, void *f_out,
                   int warmup, int reps, double *ms_out, rte_stream_t stream);

/* Selects the preconditioner of the 2D diffusion CG: on != 0 (default) the two-level
 * multigrid (block-Jacobi smoothing on the DG space, continuous-Q1 vertex-grid coarse space with
 * Galerkin operators, one V-cycle); on == 0 block-Jacobi alone.  Changes the workspace size; call
 * before sizing the workspace and not concurrently with other calls on the handle. */
int rte_problem_dsa_multigrid(rte_problem *p, int on);

/* Reports the schedule in use: directions per lane, wavefronts per workgroup and the number of
 * per-instance partial densities the 2D sweep produces. */
int rte_problem_tuning(const rte_problem *p, int *dg, int *wpb, int *nparts);

/* The bands in flight the handle's 2D sweeps ask for (rte_problem_create_sched). */
int rte_problem_bands(const rte_problem *p, int *bands);

/* Checks sigma_t >= sigma_s >= 0 and finiteness of the device materials; synchronizes the
 * stream.  Returns RTE_EINVAL on violation. */
int rte_problem_check(const rte_problem *p, void *ws, size_t ws_bytes, rte_stream_t stream);

/* Correction reduced-order model (Sec. 3.2, eq. (rom_correction), eq. (rho_basis)).
 *   Online operators of the POD basis delta U (N_v N_DOF x r):
 *     U_rho = sum_j w_j delta U_j,  U_iso = sum_j delta U_j       [N_DOF][r] each
 *     A_r(mu) = A0 + sum_k psi_k(mu) A_k  with m affine terms      A0 [r][r], A [m][r][r]
 *   The parameter vector psi [B][m] is passed to the correction calls. */
typedef struct {
    int r;                    /* rank, 1 <= r <= 64 */
    int m;                    /* number of parameter-dependent affine terms */
    const double *U_rho;      /* host [N_DOF][r] */
    const double *U_iso;      /* host [N_DOF][r] */
    const double *A0;         /* host [r][r] */
    const double *A;          /* host [m][r][r] */
    double eps_pod;           /* truncation tolerance of the basis (eq. (pod_truncation)) */
    double eps_train;         /* SISA tolerance of the training solves */
    const double *b_inflow;   /* host [4][r] or NULL: sum_j U_j^T b_j for a unit isotropic inflow on
                                 each side (x=0, x=Lx, y=0, y=Ly); used by rte_rom_initial_guess
                                 (NULL: no inflow term) */
} rte_rom_desc;

int rte_rom_create(const rte_problem *p, const rte_rom_desc *desc, rte_rom **out);

/* ROM initial guess (ROMIG, Sec. 3.1, eq. (rom_parametric)) from a parametric ROM, i.e. one whose
 * basis U spans converged angular fluxes of training parameters (build it like a correction ROM
 * with a one-iterate window, whose snapshot columns are the solutions themselves).  Per instance:
 *   (A0 + sum_k psi_k A_k) c = U^T b,  U^T b = (U^iso)^T q_G + sum_sides g_side b_inflow[side],
 * q_G the isotropic source load (G sqrt(hx hy) on the cell-mean dof), then rho_out = U^rho c.
 *   rho_out     device [B][N_DOF]; rows of instances whose reduced system is singular are left
 *               unchanged (status_out 1), so callers pass zeros there
 *   status_out  device [B] or NULL; 0 ok, 1 singular
 * 2D only (RTE_EUNSUPPORTED otherwise).  Workspace as for RTE_ROMSAD with this rom. */
int rte_rom_initial_guess(const rte_problem *p, const rte_rom *rom, const double *psi,
                          double *rho_out, int *status_out, void *ws, size_t ws_bytes,
                          rte_stream_t stream);
void rte_rom_destroy(rte_rom *rom);

/* Bytes of device workspace the calls below need for (problem, mode, rom, precision) and an
 * iteration limit max_iter of rte_sisa_solve (the per-iteration history is kept on the device).
 * A workspace sized for (mode, rom, prec, max_iter) serves every call with a mode needing no
 * more (SI < SI_DSA < ROMSAD), the same or no rom, the same precision and max_iter no larger. */
int rte_workspace_size(const rte_problem *p, rte_mode mode, const rte_rom *rom,
                       rte_precision prec, int max_iter, size_t *bytes);

/* One transport sweep, eq. (transport_sweep): for every instance and direction solve
 * (D_j + Sigma_t) f_j = Sigma_s rho_in + G + g_j^(bc) in upwind order.
 *   rho_in        device [B][N_DOF]
 *   f_out         device angular flux in the layout above (2D sweep order, 1D cell-major),
 *                 double (RTE_FP64) or float (RTE_MIXED); may be NULL; 16-byte aligned (32 for
 *                 double).  2D with f_out: fewer than 2^26 cells per instance (RTE_EUNSUPPORTED
 *                 beyond)
 *   rho_star_out  device [B][N_DOF], rho^* = sum_j w_j f_j; may be NULL
 *   zero_inflow   nonzero: use g = 0 (the kinetic correction equation's boundary condition)
 * 2D: an instance whose sigma_t takes at most 16 distinct values is swept from a table of the
 * cell solve's sigma_t-dependent coefficients per (direction, value), formed in FP64 in the
 * workspace at the start of the call (rte_sisa_solve: of the solve; rte_sisa_admit: of the
 * admitted slots); an instance with more values, or a NaN, by the per-cell solve.  Both are
 * the same cell solve; the table form rounds its coefficients once instead of forming them in
 * the sweep's precision at every cell. */
int rte_sweep(const rte_problem *p, const double *rho_in, void *f_out, double *rho_star_out,
              int zero_inflow, rte_precision prec, void *ws, size_t ws_bytes, rte_stream_t stream);

/* rte_sweep without a workspace argument, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The sweep's
 * input block, partial densities and material tables live in a library-owned device array of
 * RTE_NOALLOC_SCRATCH_BYTES per GPU, held from the library's first use on that GPU until the
 * process ends; the call itself allocates and frees nothing.  Arguments, layouts and results are
 * those of rte_sweep (the same kernels run).
 *   Returns RTE_ENOMEM, before any device work, when the problem needs more scratch than
 *   RTE_NOALLOC_SCRATCH_BYTES (the rte_workspace_size of mode RTE_SI, max_iter 1, for prec;
 *   one 128 x 128 instance with 64 directions needs about 11 MB in FP64).
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (different
 * streams, or host threads) race and must be serialized by the caller. */
#define RTE_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int rte_sweep_noalloc(const rte_problem *p, const double *rho_in, void *f_out,
                      double *rho_star_out, int zero_inflow, rte_precision prec,
                      rte_stream_t stream);

/* Quadrature reduction rho = sum_j w_j f_j (definition under eq. (dg_matrix_vec)).
 *   f     device angular flux in the layout above, double or float per prec;
 *   rho_out device [B][N_DOF] */
int rte_scalar_flux(const rte_problem *p, const void *f, double *rho_out, rte_precision prec,
                    rte_stream_t stream);

/* Diffusion synthetic acceleration, eq. (diffusion_correction):
 *   delta rho = C Sigma_s (rho^* - rho_prev).
 * 1D: consistent DSA of Appendix B (eq. (dsa_rho)-(dsa_J)), direct block solve.
 * 2D: symmetric interior-penalty (MIP) diffusion form on the Q1 space, FP64 PCG to
 *     relative residual cg_rtol within cg_maxit iterations (cg_iters_out: device int [B]). */
int rte_dsa_correct(const rte_problem *p, const double *rho_star, const double *rho_prev,
                    double *delta_rho, double cg_rtol, int cg_maxit, int *cg_iters_out,
                    void *ws, size_t ws_bytes, rte_stream_t stream);

/* ROM-based kinetic correction (ROMSA), eq. (rom_correction):
 *   y = U_iso^T Sigma_s (rho^* - rho_prev), A_r(psi_b) dc = y (LU, partial pivoting),
 *   delta rho = U_rho dc.
 *   psi        device [B][m]
 *   status_out device int [B]: 0 ok, 1 singular reduced system (delta_rho left untouched) */
int rte_rom_correct(const rte_problem *p, const rte_rom *rom, const double *psi,
                    const double *rho_star, const double *rho_prev, double *delta_rho,
                    int *status_out, rte_precision prec, void *ws, size_t ws_bytes,
                    rte_stream_t stream);

/* Options of rte_sisa_solve (Alg. 1 and Alg. 2). */
typedef struct {
    double eps;               /* stop when e_l < eps */
    int max_iter;             /* N_iter */
    int relative;             /* 1: e_l = ||rho* - rho||_inf / ||rho*||_inf; 0: absolute (Alg. 1) */
    int theta;                /* ROMSAD: ROMSA allowed for 1 <= l <= theta */
    double eps_romsad;        /* ROMSAD threshold; < 0: eta * max(eps_train, eps_pod), eta = 0.1 */
    double cg_rtol;           /* diffusion CG relative residual tolerance */
    int cg_maxit;             /* diffusion CG iteration limit per correction */
    rte_precision precision;
    int poll_every;           /* host reads the active-instance count every poll_every iterations */
    int graph_cg_iters;       /* 0: every kernel launched from the host, which reads the decision's
                                 counts and the diffusion CG's running count as it goes.  > 0: one
                                 outer iteration (sweep, reduction, stop test and switch, ROMSA and
                                 diffusion correction for the instances that chose them, update) is
                                 one HIP graph launch with no host read inside; the graph holds
                                 min(cg_maxit, graph_cg_iters) CG iterations per correction, so an
                                 instance needing more stops there and counts as a CG failure
                                 (RTE_ECG).  The graph is captured on first use and kept by the
                                 problem handle for the same workspace and arguments; the host
                                 reads the active count every poll_every launches only. */
} rte_solve_opts;

/* Host-visible statistics (arrays supplied by the caller; any may be NULL). */
typedef struct {
    int *n_sweep;             /* [B] sweeps until convergence (including the last) */
    int *status;              /* [B] RTE_OK or RTE_ENOCONV */
    double *change;           /* [B][max_iter] e_l per iteration */
    int *kind;                /* [B][max_iter] correction applied after sweep l: 0 none, 1 DSA, 2 ROMSA */
    long long cg_iterations;  /* out: total CG iterations over all instances */
    int iterations;           /* out: iterations run by the batch (max over instances) */
} rte_solve_stats;

/* Source iteration with synthetic acceleration (Alg. 1) for every instance of the batch.
 *   mode RTE_SI: no correction; RTE_SI_DSA: DSA every iteration; RTE_ROMSAD: Alg. 2 switch.
 *   rho_inout  device [B][N_DOF]: initial guess in, rho^(l,*) of the stopping iteration out
 *   psi        device [B][m] (ROMSAD only)
 *   f_out      device angular flux of the last sweep (layout above), or NULL
 * Returns RTE_ENOCONV if any instance hit max_iter (per-instance status in stats), RTE_ECG
 * (before RTE_ENOCONV) if a diffusion CG stopped at cg_maxit or on a non-finite residual; the
 * statistics are filled in either case. */
int rte_sisa_solve(const rte_problem *p, rte_mode mode, const rte_rom *rom, const double *psi,
                   const rte_solve_opts *opts, double *rho_inout, void *f_out,
                   rte_solve_stats *stats, void *ws, size_t ws_bytes, rte_stream_t stream);

/* Several independent batches solved at once (Alg. 1, as rte_sisa_solve): batch i on its own
 * problem handle, density array rho[i], workspace ws[i] (ws_bytes[i]) and stream streams[i], in
 * its own host thread (batch 0 in the caller's), all with the caller's current device.  While one
 * batch's host waits on a poll or its kernels leave the device idle between launches, another's
 * run, so a batch split into sub-batches finishes sooner than in one piece; every instance's
 * result is the one a solve of its sub-batch alone gives (and, with the same sweep schedule, the
 * one of the whole batch).  roms, psi, f_out, stats and status may be NULL (else arrays of n; a
 * NULL entry of roms, psi or f_out as for rte_sisa_solve).  status[i] receives batch i's return
 * code.  Returns an argument or device error of any batch first, then RTE_ECG, then
 * RTE_ENOCONV, else RTE_OK.  RTE_EINVAL for n outside [1, RTE_MULTI_MAX], a NULL required
 * array or entry, or two batches sharing a handle, a density array or workspace bytes. */
#define RTE_MULTI_MAX 16
int rte_sisa_solve_multi(int n, const rte_problem *const *probs, rte_mode mode,
                         const rte_rom *const *roms, const double *const *psi,
                         const rte_solve_opts *opts, double *const *rho, void *const *f_out,
                         rte_solve_stats *stats, void *const *ws, const size_t *ws_bytes,
                         const rte_stream_t *streams, int *status);

/* ------------------------------------------------------------------------------------------
 * DSA-preconditioned restarted GMRES (the paper's Krylov baseline: Sec. 2.4 and the appendix on
 * restarted GMRES).  For every instance it solves the left-preconditioned system
 *   (I + C Sigma_s)(I - L) rho = (I + C Sigma_s) b_bar
 * with L v the density of one sweep of the source Sigma_s v (no G, vacuum inflow), b_bar the
 * density of one sweep from rho = 0, and C Sigma_s the diffusion correction of rte_dsa_correct.
 * GMRES(restart): Arnoldi (classical Gram-Schmidt with one reorthogonalization), Givens
 * rotations; an instance stops once its estimated preconditioned residual is at most
 * tol * |(I + C Sigma_s) b_bar| and the residual recomputed from the iterate (one sweep) passes
 * too; otherwise it restarts from the iterate.  All FP64.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
    double tol;               /* relative residual of the preconditioned system */
    int restart;              /* Arnoldi steps per cycle, 1..200 */
    int max_cycles;           /* cycles before RTE_ENOCONV */
    double cg_rtol;           /* diffusion CG tolerance (preconditioner) */
    int cg_maxit;
    int precondition;         /* 0: plain GMRES on (I - L) */
} rte_krylov_opts;

typedef struct {
    int *n_sweep;             /* [B] transport sweeps (right-hand side, every (re)start, every step) */
    int *iterations;          /* [B] Arnoldi steps */
    int *status;              /* [B] RTE_OK or RTE_ENOCONV */
    double *residual;         /* [B] estimated relative residual at the last step */
    int cycles;               /* out: cycles run by the batch */
} rte_krylov_stats;

int rte_pgmres_workspace_size(const rte_problem *p, int restart, size_t *bytes);

/* rho: device [B][N_DOF], initial guess in (zeros, or e.g. rte_rom_initial_guess), solution out.
 * stats: host arrays (any may be NULL).  Returns RTE_ENOCONV if an instance did not converge. */
int rte_pgmres_solve(const rte_problem *p, const rte_krylov_opts *opts, double *rho,
                     rte_krylov_stats *stats, void *ws, size_t ws_bytes, rte_stream_t stream);

/* ------------------------------------------------------------------------------------------
 * Resumable solve for serving (continuous batching).  The problem's B instances are slots; the
 * workspace keeps every slot's Alg. 1 state between calls, so requests can be admitted into free
 * slots while others are mid-iteration.  Each slot counts its own sweeps l (stop test, ROMSAD
 * window 1 <= l <= theta and max_iter are per slot), so a request's result does not depend on
 * when it was admitted or on what shares the batch.  mode, rom, opts and the workspace must be
 * the same in every call of one session; sigma_t, sigma_s, source and inflow rows of a slot (the
 * problem's device arrays) and its psi row may be rewritten by the caller while the slot is free.
 * ------------------------------------------------------------------------------------------ */

/* Marks every slot free.  Call once per workspace before the first rte_sisa_admit. */
int rte_sisa_begin(const rte_problem *p, rte_mode mode, const rte_rom *rom,
                   const rte_solve_opts *opts, void *ws, size_t ws_bytes, rte_stream_t stream);

/* Starts Alg. 1 in the listed slots (host array of n_slots distinct indices in [0, B)): resets
 * their state, builds their diffusion operators (DSA modes) and forms their first sweep input
 * from rho (device [B][N_DOF]; the slots' rows are the initial guesses).  Synchronises with the
 * stream before returning.  RTE_EINVAL for an index out of range. */
int rte_sisa_admit(const rte_problem *p, rte_mode mode, const rte_rom *rom,
                   const rte_solve_opts *opts, const int *slots, int n_slots, const double *rho,
                   void *ws, size_t ws_bytes, rte_stream_t stream);

/* Runs up to n_iter outer iterations of every running slot (fewer if all stop), then fills
 * active_out (host [B], nullable: 1 while a slot still iterates) and stats (n_sweep, status,
 * change, kind per slot).  A slot that stopped holds rho^(l,*) in its row of rho.  Slots that
 * are still running are not an error: returns RTE_OK unless a call fails. */
int rte_sisa_iterate(const rte_problem *p, rte_mode mode, const rte_rom *rom, const double *psi,
                     const rte_solve_opts *opts, double *rho, int n_iter, int *active_out,
                     rte_solve_stats *stats, void *ws, size_t ws_bytes, rte_stream_t stream);

/* ------------------------------------------------------------------------------------------
 * Offline construction of the correction ROM (Sec. 3.1 POD, Sec. 3.2.1 snapshots, Sec. 3.1.1
 * reduced affine operators).  Building blocks driven by the Python offline builder.  Results
 * and accumulations are FP64; the long snapshot columns may be stored in FP32 (RTE_MIXED), which
 * halves the memory of bases whose FP64 columns would not fit in HBM.
 * ------------------------------------------------------------------------------------------ */

/* Snapshot columns delta f = f_final - f_iter per instance (Sec. 3.2.1); f_iter == NULL stands
 * for the zero initial state.  f_final, f_iter: device FP64 angular fluxes in the sweep's layout
 * (see the conventions above); the difference is formed in FP64 and written as double
 * (cols_prec RTE_FP64) or rounded to float (RTE_MIXED), direction-major in natural cell order,
 * entry j * N_DOF + dof; column b is written at cols + b * stride elements
 * (stride >= n_dir * N_DOF). */
int rte_pod_snapshots(const rte_problem *p, const double *f_final, const double *f_iter,
                      void *cols, long long stride, rte_precision cols_prec, rte_stream_t stream);

/* The angular flux f (layout of the conventions above, double for RTE_FP64, float for
 * RTE_MIXED) in natural order: out device [B][n_dir][N_DOF], same type, out[b][j] = f_j of
 * instance b (the vector of eq. (dg_matrix_vec)).  out must not overlap f. */
int rte_f_natural(const rte_problem *p, const void *f, void *out, rte_precision prec,
                  rte_stream_t stream);

/* G = X^T Y for column-major X [nx][len], Y [ny][len] (device; double for RTE_FP64, float for
 * RTE_MIXED, widened to double), G [nx][ny] FP64 device, on the FP64 matrix cores.  With
 * cell_class != NULL only rows whose cell ((row / K) mod ncell) has class cls are summed (the
 * material-class restriction of the reduced affine operators).  ws: device scratch for the
 * split partial sums (ENOMEM if too small for one split). */
int rte_gram(const void *X, rte_precision xprec, int nx, const void *Y, rte_precision yprec,
             int ny, long long len, const int *cell_class, int K, long long ncell, int cls,
             double *G, void *ws, size_t ws_bytes, rte_stream_t stream);

/* Eigen-decomposition of a symmetric n x n device matrix A (n <= 256, overwritten) by cyclic
 * Jacobi: evals [n] (unsorted), evecs [n][n] with eigenvectors as columns (method of snapshots,
 * Sec. 3.1: F^T F = V Lambda^2 V^T). */
int rte_sym_eig(double *A, int n, double *evals, double *evecs, rte_stream_t stream);

/* Basis weights of the method of snapshots (Sec. 3.1): from the eigenpairs of F^T F (rte_sym_eig:
 * evals [ncol], evecs [ncol][ncol] with eigenvectors as columns; device FP64, ncol <= 256) the
 * singular values sv = sqrt(max(lambda, 0)) sorted descending (device [ncol]; ties keep index
 * order), the rank -- r if r > 0, else the smallest rank whose share of the sum of singular values
 * reaches 1 - eps_pod (eq. (pod_truncation)), capped at the count of singular values above
 * 1e-13 of the largest -- in r_out (device int [1]), the dropped share 1 - sum_{k<r} sv_k / sum sv
 * in eps_out (device [1]), and W = V Sigma^-1 of the kept columns, W[i][k] = v_i of the k-th
 * largest eigenvalue / sv_k, in W (device [ncol][ncol], leading dimension ncol; columns k >= r
 * are not written).  U = F W is then the POD basis. */
int rte_pod_weights(const double *evals, const double *evecs, int ncol, int r, double eps_pod,
                    double *sv, double *W, int *r_out, double *eps_out, rte_stream_t stream);

/* Upper Cholesky factor of a small SPD matrix and its inverse (the QR route of the POD, Sec. 3.1:
 * CholeskyQR of the snapshot matrix F from Gram matrices): G [n][n] (device FP64, row-major,
 * symmetric), n <= 256; R and T = R^-1 [n][n] upper triangular with G + shift I = R^T R; work
 * [n][n] scratch.  shifted = 0: no shift; else shift = 11 (m n + n (n+1)) u trace(G), u = 2^-53,
 * for the Gram matrix of an m x n matrix (shifted CholeskyQR, m >= 1).  info (device int [1]):
 * 0, or k + 1 if pivot k was not positive (R, T then incomplete).  dev (device [1], or NULL):
 * max |G_ij - delta_ij|, how far the columns whose Gram matrix G is are from orthonormal. */
int rte_chol_upper(const double *G, int n, int shifted, long long m, double *work, double *R,
                   double *T, int *info, double *dev, rte_stream_t stream);

/* One-sided Jacobi SVD of a small matrix A [n][n] (device FP64, row-major, n <= 256): lam [n] the
 * squared singular values (unsorted), V [n][n] the right singular vectors as columns, and US
 * [n][n] (or NULL) = A V, whose column k is s_k u_k; work: 2 n^2 doubles of scratch.  Rounds of
 * the round-robin ordering until a sweep applies no rotation or max_sweeps; sweeps_out (device
 * int [1]) the sweeps run (max_sweeps: not converged).  (lam, V) or (lam, US) plug into
 * rte_pod_weights in place of the Gram eigenpairs: with US it returns the kept left singular
 * vectors u_k = US[:, k] / s_k. */
int rte_svd_jacobi(const double *A, int n, double *work, double *lam, double *V, double *US,
                   int max_sweeps, int *sweeps_out, rte_stream_t stream);

/* C = alpha op(A) B for small dense FP64 matrices (device, row-major): op(A) = A [m][k]
 * (trans_a = 0) or the transpose of A [k][m] (trans_a = 1); B [k][n], or NULL for the identity
 * (then k == n and C = alpha op(A)); C [m][n].  The reduced products of the offline construction
 * (W^T G W, the reduced inflow loads, signs).  RTE_EUNSUPPORTED beyond 2^26 entries of C. */
int rte_small_gemm(int trans_a, int m, int n, int k, double alpha, const double *A, const double *B,
                   double *C, rte_stream_t stream);

/* out[c] = sum_col W[col][c] X[col] for X [ncol][len], W [ncol][r], out [r][len] (device FP64),
 * on the matrix cores (the basis U = F V Lambda^-1 of the method of snapshots). */
int rte_combine(const double *X, int ncol, long long len, const double *W, int r, double *out,
                rte_stream_t stream);

/* y_j = D_j x_j of eq. (dg_matrix_vec) (streaming + upwind flux, no boundary load) for nvec
 * vectors x [nvec][n_dir][N_DOF] (double or float per xprec), y FP64 of the same shape (2D). */
int rte_apply_streaming(const rte_problem *p, const void *x, rte_precision xprec, int nvec,
                        double *y, rte_stream_t stream);

/* out[side][k] = sum_j U_k,j^T b_side,j: projections of the load of a unit isotropic inflow on each
 * side (x=0, x=Lx, y=0, y=Ly; eq. (dg_matrix_vec)) on the vectors U [nvec][n_dir][N_DOF]
 * (device, direction-major, double or float per uprec).  out: device FP64 [4][nvec].  2D only. */
int rte_inflow_loads(const rte_problem *p, const void *U, rte_precision uprec, int nvec,
                     double *out, rte_stream_t stream);

/* out[v] = sum_j w_j x[v][j] (weighted != 0) or sum_j x[v][j] (weighted == 0) for
 * x [nvec][n_dir][N_DOF] (double or float per xprec), out FP64 [nvec][N_DOF]: U^rho and U^iso of
 * eq. (rho_basis). */
int rte_direction_sum(const rte_problem *p, const void *x, rte_precision xprec, int nvec,
                      int weighted, double *out, rte_stream_t stream);

/* Kernel timing with HIP events recorded on the launch stream around every launch of the
 * named kernel group (process-wide; not for concurrent use from several threads).
 * rte_profile_enable(1) clears and starts recording, (0) stops; rte_profile_read returns the
 * summed event time in milliseconds and the number of timed launches since the last enable. */
enum {
    RTE_PROF_SWEEP2D = 0,     /* 2D transport sweep kernel */
    RTE_PROF_REDUCE = 1,      /* partial-density reduction + change maxima */
    RTE_PROF_DSA = 2,         /* one diffusion correction (all its CG kernels and polls) */
    RTE_PROF_ROM = 3,         /* one ROM correction (projection, reduced solve, lift) */
    RTE_PROF_SWEEP1D = 4,     /* 1D transport sweep kernel */
    RTE_PROF_NKERNELS = 5
};
int rte_profile_enable(int on);
int rte_profile_read(int kernel, double *total_ms, long long *count);

const char *rte_strerror(int status);
/* The HIP runtime's description of the last HIP error for which a call made on this thread
 * returned RTE_EDEVICE ("" if none).  The string is static; the library owns it. */
const char *rte_last_device_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RTE_H */
