"""ctypes binding of librte.so (argument marshalling only).

Every numerical step runs in the library's gfx950 kernels; PyTorch provides device memory and
the stream.  Importing this module on a machine without the built library raises at once.
Names follow the C ABI in include/rte.h.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librte.so")

RTE_OK, RTE_EINVAL, RTE_ENOCONV, RTE_ESINGULAR, RTE_ECG, RTE_ENOMEM, RTE_EDEVICE, RTE_EUNSUPPORTED = range(8)
FP64, MIXED = 0, 1
SI, SI_DSA, ROMSAD = 0, 1, 2
MODES = {"si": SI, "si_dsa": SI_DSA, "romsad": ROMSAD}
PRECISIONS = {"fp64": FP64, "mixed": MIXED}


class RteError(RuntimeError):
    def __init__(self, status, what):
        detail = ""
        if status == RTE_EDEVICE:
            detail = lib.rte_last_device_error().decode()
        super().__init__(f"{what}: {strerror(status)} ({status})" + (f": {detail}" if detail else ""))
        self.status = status


_D = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class ProblemDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("batch", ctypes.c_int), ("n_dir", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("widths", _D), ("dir_x", _D), ("dir_y", _D), ("weight", _D),
                ("sigma_t", _vp), ("sigma_s", _vp), ("source", _vp), ("inflow", _vp)]


class RomDesc(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int), ("m", ctypes.c_int), ("U_rho", _D), ("U_iso", _D),
                ("A0", _D), ("A", _D), ("eps_pod", ctypes.c_double),
                ("eps_train", ctypes.c_double), ("b_inflow", _D)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("max_iter", ctypes.c_int), ("relative", ctypes.c_int),
                ("theta", ctypes.c_int), ("eps_romsad", ctypes.c_double),
                ("cg_rtol", ctypes.c_double), ("cg_maxit", ctypes.c_int),
                ("precision", ctypes.c_int), ("poll_every", ctypes.c_int),
                ("graph_cg_iters", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("n_sweep", ctypes.POINTER(ctypes.c_int)), ("status", ctypes.POINTER(ctypes.c_int)),
                ("change", _D), ("kind", ctypes.POINTER(ctypes.c_int)),
                ("cg_iterations", ctypes.c_longlong), ("iterations", ctypes.c_int)]


class KrylovOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("cg_rtol", ctypes.c_double), ("cg_maxit", ctypes.c_int),
                ("precondition", ctypes.c_int)]


class KrylovStats(ctypes.Structure):
    _fields_ = [("n_sweep", ctypes.POINTER(ctypes.c_int)),
                ("iterations", ctypes.POINTER(ctypes.c_int)),
                ("status", ctypes.POINTER(ctypes.c_int)), ("residual", _D),
                ("cycles", ctypes.c_int)]


EXPORTED = ["rte_problem_create", "rte_problem_create_tuned", "rte_problem_destroy",
            "rte_problem_tuning", "rte_problem_check", "rte_rom_create", "rte_rom_destroy",
            "rte_workspace_size", "rte_sweep", "rte_scalar_flux", "rte_dsa_correct",
            "rte_rom_correct", "rte_sisa_solve", "rte_strerror", "rte_profile_enable",
            "rte_profile_read", "rte_problem_dsa_multigrid", "rte_pod_snapshots", "rte_gram",
            "rte_sym_eig", "rte_combine", "rte_apply_streaming", "rte_direction_sum",
            "rte_sisa_begin", "rte_sisa_admit", "rte_sisa_iterate", "rte_rom_initial_guess",
            "rte_inflow_loads", "rte_pgmres_workspace_size", "rte_pgmres_solve", "rte_f_natural",
            "rte_last_device_error", "rte_sweep_noalloc", "rte_tune_sweep",
            "rte_pod_weights", "rte_small_gemm", "rte_chol_upper", "rte_svd_jacobi",
            "rte_sisa_solve_multi", "rte_problem_create_sched", "rte_problem_bands"]


def _load():
    # The library takes torch's device pointers and streams, so it must bind to the HIP runtime
    # torch carries.  torch's copy of libamdhip64 has the same soname as the system one the
    # library was linked against: loading torch first makes the library's dependency resolve to
    # torch's copy.  Loaded the other way round, the process would hold two HIP runtimes.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2402_10488_amd/build.py "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    missing = [n for n in EXPORTED if not hasattr(L, n)]
    if missing:
        raise ImportError(f"{LIB_PATH} lacks {missing}: it was built from older sources, rebuild it")
    P = ctypes.c_void_p
    L.rte_strerror.restype = ctypes.c_char_p
    L.rte_strerror.argtypes = [ctypes.c_int]
    L.rte_last_device_error.restype = ctypes.c_char_p
    L.rte_last_device_error.argtypes = []
    L.rte_problem_create_tuned.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(P)]
    L.rte_problem_create_sched.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.POINTER(P)]
    L.rte_problem_bands.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
    L.rte_problem_destroy.argtypes = [P]
    L.rte_problem_destroy.restype = None
    L.rte_problem_tuning.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int)]
    L.rte_problem_check.argtypes = [P, _vp, ctypes.c_size_t, _vp]
    L.rte_rom_create.argtypes = [P, ctypes.POINTER(RomDesc), ctypes.POINTER(P)]
    L.rte_rom_destroy.argtypes = [P]
    L.rte_rom_destroy.restype = None
    L.rte_workspace_size.argtypes = [P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_size_t)]
    L.rte_sweep.argtypes = [P, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t, _vp]
    L.rte_sweep_noalloc.argtypes = [P, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
    _ip = ctypes.POINTER(ctypes.c_int)
    L.rte_tune_sweep.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.c_int, ctypes.c_int, _ip, _ip,
                                 _ip, _vp, _vp, ctypes.c_int, ctypes.c_int, _D, _vp]
    L.rte_scalar_flux.argtypes = [P, _vp, _vp, ctypes.c_int, _vp]
    L.rte_f_natural.argtypes = [P, _vp, _vp, ctypes.c_int, _vp]
    L.rte_dsa_correct.argtypes = [P, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _vp, _vp,
                                  ctypes.c_size_t, _vp]
    L.rte_rom_correct.argtypes = [P, P, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_size_t,
                                  _vp]
    L.rte_sisa_solve.argtypes = [P, ctypes.c_int, P, _vp, ctypes.POINTER(SolveOpts), _vp, _vp,
                                 ctypes.POINTER(SolveStats), _vp, ctypes.c_size_t, _vp]
    L.rte_sisa_begin.argtypes = [P, ctypes.c_int, P, ctypes.POINTER(SolveOpts), _vp, ctypes.c_size_t,
                                 _vp]
    L.rte_sisa_solve_multi.argtypes = [ctypes.c_int, ctypes.POINTER(P), ctypes.c_int,
                                       ctypes.POINTER(P), ctypes.POINTER(_vp),
                                       ctypes.POINTER(SolveOpts), ctypes.POINTER(_vp),
                                       ctypes.POINTER(_vp), ctypes.POINTER(SolveStats),
                                       ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_int)]
    L.rte_sisa_admit.argtypes = [P, ctypes.c_int, P, ctypes.POINTER(SolveOpts),
                                 ctypes.POINTER(ctypes.c_int), ctypes.c_int, _vp, _vp,
                                 ctypes.c_size_t, _vp]
    L.rte_sisa_iterate.argtypes = [P, ctypes.c_int, P, _vp, ctypes.POINTER(SolveOpts), _vp,
                                   ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(SolveStats), _vp, ctypes.c_size_t, _vp]
    L.rte_rom_initial_guess.argtypes = [P, P, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.rte_pgmres_workspace_size.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.rte_pgmres_solve.argtypes = [P, ctypes.POINTER(KrylovOpts), _vp, ctypes.POINTER(KrylovStats),
                                   _vp, ctypes.c_size_t, _vp]
    L.rte_problem_dsa_multigrid.argtypes = [P, ctypes.c_int]
    L.rte_profile_enable.argtypes = [ctypes.c_int]
    L.rte_profile_read.argtypes = [ctypes.c_int, _D, ctypes.POINTER(ctypes.c_longlong)]
    return L


lib = _load()


PROF = {"sweep2d": 0, "reduce": 1, "dsa": 2, "rom": 3, "sweep1d": 4}


def profile_enable(on=True):
    """Start (clear) or stop per-kernel HIP-event timing inside the library."""
    _check(lib.rte_profile_enable(int(bool(on))), "rte_profile_enable")


def profile_read(kernel):
    """(total milliseconds, number of timed launches) of a kernel group since profile_enable."""
    ms, n = ctypes.c_double(), ctypes.c_longlong()
    _check(lib.rte_profile_read(PROF[kernel], ctypes.byref(ms), ctypes.byref(n)), "rte_profile_read")
    return ms.value, n.value


def strerror(status: int) -> str:
    return lib.rte_strerror(int(status)).decode()


def _check(status, what):
    if status != RTE_OK:
        raise RteError(status, what)


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _host(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


class Problem:
    """A batch of B instances sharing mesh and directions; materials live on the device.

    sigma_t, sigma_s, G: float64 CUDA tensors [B, ny, nx]; inflow [B, 4].
    Directions and weights are host arrays (normalized weights).
    """

    def __init__(self, dim, nx, ny, dirs_x, weights, sigma_t, sigma_s, G, inflow, dirs_y=None,
                 lx=1.0, ly=1.0, widths=None, dg=0, wpb=0, bands=0):
        import torch
        for t in (sigma_t, sigma_s, G, inflow):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        self.dim, self.nx, self.ny = dim, nx, ny
        self.B = int(sigma_t.shape[0])
        self.K = 4 if dim == 2 else 2
        self.ncell = nx * ny
        self.ndof = self.ncell * self.K
        self.n_dir = len(dirs_x)
        self._keep = [sigma_t, sigma_s, G, inflow]
        self.sigma_t, self.sigma_s, self.G, self.inflow = sigma_t, sigma_s, G, inflow
        self._dx, pdx = _host(dirs_x)
        self._w, pw = _host(weights)
        pdy, pwd = None, None
        if dirs_y is not None:
            self._dy, pdy = _host(dirs_y)
        if widths is not None:
            self._wd, pwd = _host(widths)
        d = ProblemDesc(dim, nx, ny, self.B, self.n_dir, float(lx), float(ly), pwd, pdx, pdy, pw,
                        _ptr(sigma_t), _ptr(sigma_s), _ptr(G), _ptr(inflow))
        h = ctypes.c_void_p()
        _check(lib.rte_problem_create_sched(ctypes.byref(d), int(dg), int(wpb), int(bands),
                                            ctypes.byref(h)), "rte_problem_create")
        self.handle = h
        self._desc = d            # host arrays it points to are kept above
        self.weights = np.asarray(weights, dtype=np.float64)

    def tuning(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.rte_problem_tuning(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "rte_problem_tuning")
        nb = ctypes.c_int()
        _check(lib.rte_problem_bands(self.handle, ctypes.byref(nb)), "rte_problem_bands")
        return {"dg": a.value, "wpb": b.value, "nparts": c.value, "bands": nb.value}

    def dsa_multigrid(self, on=True):
        """Multigrid (default) or block-Jacobi preconditioning of the 2D diffusion CG."""
        _check(lib.rte_problem_dsa_multigrid(self.handle, int(bool(on))), "rte_problem_dsa_multigrid")

    def workspace_bytes(self, mode="si", rom=None, precision="fp64", max_iter=1):
        n = ctypes.c_size_t()
        _check(lib.rte_workspace_size(self.handle, MODES[mode], rom.handle if rom else None,
                                      PRECISIONS[precision], int(max_iter), ctypes.byref(n)),
               "rte_workspace_size")
        return n.value

    def workspace(self, mode="si", rom=None, precision="fp64", max_iter=1):
        import torch
        nb = self.workspace_bytes(mode, rom, precision, max_iter)
        return torch.empty(max(nb, 256), dtype=torch.uint8, device=self.sigma_t.device)

    def pgmres_workspace(self, restart=25):
        import torch
        n = ctypes.c_size_t()
        _check(lib.rte_pgmres_workspace_size(self.handle, int(restart), ctypes.byref(n)),
               "rte_pgmres_workspace_size")
        return torch.empty(max(n.value, 256), dtype=torch.uint8, device=self.sigma_t.device)

    def check(self, ws=None):
        ws = ws if ws is not None else self.workspace()
        _check(lib.rte_problem_check(self.handle, _ptr(ws), ws.numel(), _stream()), "rte_problem_check")

    def close(self):
        if getattr(self, "handle", None):
            lib.rte_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Rom:
    """ROM operators (host arrays, copied to the device at creation): a correction ROM for ROMSA,
    or a parametric one (with b_inflow [4][r]) for the ROM initial guess."""

    def __init__(self, problem: Problem, U_rho, U_iso, A0, A, eps_pod, eps_train, b_inflow=None):
        self._u_rho, pur = _host(U_rho)
        self._u_iso, pui = _host(U_iso)
        self._a0, pa0 = _host(A0)
        A = np.asarray(A, dtype=np.float64).reshape(-1, self._a0.shape[0], self._a0.shape[0])
        self._a, pa = _host(A)
        self.r = int(self._a0.shape[0])
        self.m = int(A.shape[0])
        assert self._u_rho.shape == (problem.ndof, self.r)
        pb = None
        if b_inflow is not None:
            self._b_in, pb = _host(np.asarray(b_inflow).reshape(4, self.r))
        d = RomDesc(self.r, self.m, pur, pui, pa0, pa, float(eps_pod), float(eps_train), pb)
        h = ctypes.c_void_p()
        _check(lib.rte_rom_create(problem.handle, ctypes.byref(d), ctypes.byref(h)), "rte_rom_create")
        self.handle = h
        self.eps_pod, self.eps_train = float(eps_pod), float(eps_train)

    def close(self):
        if getattr(self, "handle", None):
            lib.rte_rom_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sweep(p: Problem, rho_in, f_out=None, rho_star_out=None, zero_inflow=False, precision="fp64",
          ws=None):
    ws = ws if ws is not None else p.workspace("si", None, precision)
    _check(lib.rte_sweep(p.handle, _ptr(rho_in), _ptr(f_out), _ptr(rho_star_out), int(zero_inflow),
                         PRECISIONS[precision], _ptr(ws), ws.numel(), _stream()), "rte_sweep")


def sweep_noalloc(p: Problem, rho_in, f_out=None, rho_star_out=None, zero_inflow=False,
                  precision="fp64"):
    """rte_sweep on the library's own per-device scratch array: no workspace, no allocation.
    Calls on one GPU share that array and must not overlap."""
    _check(lib.rte_sweep_noalloc(p.handle, _ptr(rho_in), _ptr(f_out), _ptr(rho_star_out),
                                 int(zero_inflow), PRECISIONS[precision], _stream()),
           "rte_sweep_noalloc")


NOALLOC_SCRATCH_BYTES = 32 << 20      # RTE_NOALLOC_SCRATCH_BYTES of include/rte.h


def tune_sweep(p: Problem, candidates, rho_in, precision="mixed", f_out=None, warmup=1, reps=3):
    """Milliseconds per 2D sweep of p's batch under each (dg, wpb) or (dg, wpb, bands) candidate
    (rte_tune_sweep); -1 marks a candidate the library does not run as given."""
    rows = [tuple(c_) + (1,) * (3 - len(c_)) for c_ in candidates]
    c = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1, 3)
    dg = np.ascontiguousarray(c[:, 0])
    wpb = np.ascontiguousarray(c[:, 1])
    bands = np.ascontiguousarray(c[:, 2])
    ms = np.zeros(len(c))
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    _check(lib.rte_tune_sweep(ctypes.byref(p._desc), PRECISIONS[precision], len(c), ip(dg), ip(wpb),
                              ip(bands), _ptr(rho_in), _ptr(f_out), int(warmup), int(reps),
                              ms.ctypes.data_as(_D), _stream()), "rte_tune_sweep")
    return ms


def f_shape(p: Problem):
    """Shape of the angular flux the library writes and reads: 2D (B, n_dir, ncell, 4), each
    direction's cells in its quadrant's diagonal order; 1D (B, ncell, n_dir, 2)."""
    return (p.B, p.n_dir, p.ncell, p.K) if p.dim == 2 else (p.B, p.ncell, p.n_dir, p.K)


def f_natural(p: Problem, f, precision="fp64"):
    """The angular flux as (B, n_dir, N_DOF) in natural cell order (row j is f_j)."""
    import torch
    dt = torch.float64 if precision == "fp64" else torch.float32
    out = torch.empty((p.B, p.n_dir, p.ndof), dtype=dt, device=f.device)
    _check(lib.rte_f_natural(p.handle, _ptr(f), _ptr(out), PRECISIONS[precision], _stream()),
           "rte_f_natural")
    return out


def scalar_flux(p: Problem, f, rho_out, precision="fp64"):
    _check(lib.rte_scalar_flux(p.handle, _ptr(f), _ptr(rho_out), PRECISIONS[precision], _stream()),
           "rte_scalar_flux")


def dsa_correct(p: Problem, rho_star, rho_prev, delta_out, cg_rtol=1e-10, cg_maxit=5000,
                iters_out=None, ws=None):
    ws = ws if ws is not None else p.workspace("si_dsa")
    _check(lib.rte_dsa_correct(p.handle, _ptr(rho_star), _ptr(rho_prev), _ptr(delta_out),
                               float(cg_rtol), int(cg_maxit), _ptr(iters_out), _ptr(ws), ws.numel(),
                               _stream()), "rte_dsa_correct")


def rom_initial_guess(p: Problem, rom: Rom, psi, rho_out, status_out=None, ws=None):
    """ROMIG: rho_out = U^rho c with the reduced parametric system of every instance."""
    ws = ws if ws is not None else p.workspace("romsad", rom, "fp64")
    _check(lib.rte_rom_initial_guess(p.handle, rom.handle, _ptr(psi), _ptr(rho_out),
                                     _ptr(status_out), _ptr(ws), ws.numel(), _stream()),
           "rte_rom_initial_guess")


def rom_correct(p: Problem, rom: Rom, psi, rho_star, rho_prev, delta_out, status_out=None,
                precision="fp64", ws=None):
    ws = ws if ws is not None else p.workspace("romsad", rom, precision)
    _check(lib.rte_rom_correct(p.handle, rom.handle, _ptr(psi), _ptr(rho_star), _ptr(rho_prev),
                               _ptr(delta_out), _ptr(status_out), PRECISIONS[precision], _ptr(ws),
                               ws.numel(), _stream()), "rte_rom_correct")


@dataclass
class SolveResult:
    status: int
    n_sweep: np.ndarray
    inst_status: np.ndarray
    change: np.ndarray
    kind: np.ndarray
    iterations: int
    cg_iterations: int = 0      # diffusion CG iterations summed over instances and corrections


def sisa_solve(p: Problem, rho_inout, mode="si_dsa", rom: Optional[Rom] = None, psi=None,
               eps=1e-8, max_iter=500, relative=True, theta=5, eps_romsad=-1.0, cg_rtol=1e-10,
               cg_maxit=5000, precision="fp64", poll_every=4, f_out=None, ws=None,
               raise_on_error=True, graph_cg_iters=0):
    """Alg. 1 (Alg. 2 for ROMSAD) on every instance.  graph_cg_iters > 0 runs each outer
    iteration as one HIP graph launch holding that many diffusion CG iterations per correction
    (rte_solve_opts.graph_cg_iters); 0 launches kernel by kernel."""
    ws = ws if ws is not None else p.workspace(mode, rom, precision, max_iter)
    B = p.B
    n_sweep = np.zeros(B, np.int32)
    st = np.zeros(B, np.int32)
    change = np.zeros((B, max_iter))
    kind = np.zeros((B, max_iter), np.int32)
    stats = SolveStats(n_sweep.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                       st.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), change.ctypes.data_as(_D),
                       kind.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), 0, 0)
    o = SolveOpts(float(eps), int(max_iter), int(relative), int(theta), float(eps_romsad),
                  float(cg_rtol), int(cg_maxit), PRECISIONS[precision], int(poll_every),
                  int(graph_cg_iters))
    rc = lib.rte_sisa_solve(p.handle, MODES[mode], rom.handle if rom else None, _ptr(psi),
                            ctypes.byref(o), _ptr(rho_inout), _ptr(f_out), ctypes.byref(stats),
                            _ptr(ws), ws.numel(), _stream())
    if raise_on_error and rc not in (RTE_OK, RTE_ENOCONV):
        raise RteError(rc, "rte_sisa_solve")
    return SolveResult(rc, n_sweep, st, change, kind, stats.iterations, stats.cg_iterations)


def sisa_solve_multi(problems, rhos, streams, mode="si_dsa", roms=None, psis=None, eps=1e-8,
                     max_iter=500, relative=True, theta=5, eps_romsad=-1.0, cg_rtol=1e-10,
                     cg_maxit=5000, precision="fp64", poll_every=4, wss=None,
                     raise_on_error=True):
    """Independent batches solved together (rte_sisa_solve_multi): batch i on problems[i] with
    densities rhos[i] and workspace wss[i] on the torch stream streams[i].  Returns one
    SolveResult per batch."""
    n = len(problems)
    roms = roms if roms is not None else [None] * n
    psis = psis if psis is not None else [None] * n
    wss = wss if wss is not None else [p.workspace(mode, r, precision, max_iter)
                                       for p, r in zip(problems, roms)]
    arrays, stats = [], (SolveStats * n)()
    for i, p in enumerate(problems):
        B = p.B
        a = (np.zeros(B, np.int32), np.zeros(B, np.int32), np.zeros((B, max_iter)),
             np.zeros((B, max_iter), np.int32))
        arrays.append(a)
        stats[i] = SolveStats(a[0].ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                              a[1].ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                              a[2].ctypes.data_as(_D),
                              a[3].ctypes.data_as(ctypes.POINTER(ctypes.c_int)), 0, 0)
    o = SolveOpts(float(eps), int(max_iter), int(relative), int(theta), float(eps_romsad),
                  float(cg_rtol), int(cg_maxit), PRECISIONS[precision], int(poll_every), 0)
    Parr = ctypes.c_void_p * n
    status = (ctypes.c_int * n)()
    rc = lib.rte_sisa_solve_multi(
        n, Parr(*[p.handle for p in problems]), MODES[mode],
        Parr(*[r.handle if r is not None else None for r in roms]),
        Parr(*[_ptr(x) for x in psis]), ctypes.byref(o), Parr(*[_ptr(x) for x in rhos]),
        None, stats, Parr(*[_ptr(w) for w in wss]),
        (ctypes.c_size_t * n)(*[w.numel() for w in wss]),
        Parr(*[ctypes.c_void_p(s.cuda_stream) for s in streams]), status)
    if raise_on_error and rc not in (RTE_OK, RTE_ENOCONV):
        raise RteError(rc, "rte_sisa_solve_multi")
    return [SolveResult(status[i], a[0], a[1], a[2], a[3], stats[i].iterations,
                        stats[i].cg_iterations) for i, a in enumerate(arrays)]


class Session:
    """Resumable slot-based solve on one problem (rte_sisa_begin / _admit / _iterate).

    The problem's B instances are slots.  Between iterate() calls the caller may rewrite the
    material rows (problem.sigma_t, sigma_s, G, g) and psi row of a free slot and admit it.
    ``stream`` (a torch.cuda.Stream or None for the current stream) carries every call.
    """

    def __init__(self, p: Problem, mode="romsad", rom: Optional[Rom] = None, psi=None, eps=1e-6,
                 max_iter=500, relative=True, theta=5, eps_romsad=-1.0, cg_rtol=1e-10,
                 cg_maxit=5000, precision="mixed", poll_every=1, stream=None, graph_cg_iters=0):
        import torch
        self.p, self.mode, self.rom, self.psi = p, mode, rom, psi
        self.max_iter = int(max_iter)
        self.stream = stream
        self.opts = SolveOpts(float(eps), int(max_iter), int(relative), int(theta),
                              float(eps_romsad), float(cg_rtol), int(cg_maxit),
                              PRECISIONS[precision], int(poll_every), int(graph_cg_iters))
        with self._on_stream():
            self.ws = p.workspace(mode, rom, precision, max_iter)
            self.rho = torch.zeros((p.B, p.ndof), dtype=torch.float64, device="cuda")
            _check(lib.rte_sisa_begin(p.handle, MODES[mode], self._rom(), ctypes.byref(self.opts),
                                      _ptr(self.ws), self.ws.numel(), _stream()), "rte_sisa_begin")
        self.n_sweep = np.zeros(p.B, np.int32)
        self.status = np.zeros(p.B, np.int32)
        self.active = np.zeros(p.B, np.int32)

    def _rom(self):
        return self.rom.handle if self.rom else None

    def _on_stream(self):
        import contextlib
        import torch
        return torch.cuda.stream(self.stream) if self.stream is not None else contextlib.nullcontext()

    def admit(self, slots):
        """Start Alg. 1 in ``slots`` from the initial guesses in their rows of self.rho."""
        slots = np.ascontiguousarray(slots, dtype=np.int32)
        with self._on_stream():
            _check(lib.rte_sisa_admit(self.p.handle, MODES[self.mode], self._rom(),
                                      ctypes.byref(self.opts),
                                      slots.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                      len(slots), _ptr(self.rho), _ptr(self.ws), self.ws.numel(),
                                      _stream()), "rte_sisa_admit")
        self.active[slots] = 1

    def iterate(self, n_iter=1):
        """Up to n_iter outer iterations of the running slots; returns the active flags."""
        stats = SolveStats(self.n_sweep.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           self.status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), None, None,
                           0, 0)
        with self._on_stream():
            _check(lib.rte_sisa_iterate(self.p.handle, MODES[self.mode], self._rom(),
                                        _ptr(self.psi), ctypes.byref(self.opts), _ptr(self.rho),
                                        int(n_iter),
                                        self.active.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                        ctypes.byref(stats), _ptr(self.ws), self.ws.numel(),
                                        _stream()), "rte_sisa_iterate")
        return self.active


@dataclass
class PgmresResult:
    status: int
    n_sweep: np.ndarray
    iterations: np.ndarray
    inst_status: np.ndarray
    residual: np.ndarray
    cycles: int


def pgmres_solve(p: Problem, rho_inout, tol=1e-10, restart=25, max_cycles=40, cg_rtol=1e-10,
                 cg_maxit=5000, precondition=True, ws=None, raise_on_error=True):
    """DSA-preconditioned restarted GMRES for every instance; rho_inout: initial guess / result."""
    ws = ws if ws is not None else p.pgmres_workspace(restart)
    B = p.B
    n_sweep, iters, st = (np.zeros(B, np.int32) for _ in range(3))
    res = np.zeros(B)
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    stats = KrylovStats(ip(n_sweep), ip(iters), ip(st), res.ctypes.data_as(_D), 0)
    o = KrylovOpts(float(tol), int(restart), int(max_cycles), float(cg_rtol), int(cg_maxit),
                   int(bool(precondition)))
    rc = lib.rte_pgmres_solve(p.handle, ctypes.byref(o), _ptr(rho_inout), ctypes.byref(stats),
                              _ptr(ws), ws.numel(), _stream())
    if raise_on_error and rc not in (RTE_OK, RTE_ENOCONV):
        raise RteError(rc, "rte_pgmres_solve")
    return PgmresResult(rc, n_sweep, iters, st, res, stats.cycles)
