"""Offline construction of the correction ROM on the GPU (Sec. 3.1, 3.2.1, 3.1.1).

Orchestrates library entry points (argument marshalling only):
  1. FP64 f-form SI-DSA training solves (Alg. 1) that keep f^(1), f^(2), ... and the converged f;
  2. snapshot columns delta f = f - f^(l) for the window of iterates that starts at the zero
     initial state (so f itself is the first column), Sec. 3.2.1;
  3. method of snapshots: G = dF^T dF on the matrix cores, Jacobi eigenpairs, basis
     dU = dF V_r Lambda_r^{-1/2} (the r largest singular values);
  4. dU^rho = sum_j w_j dU_j, dU^iso = sum_j dU_j (eq. (rho_basis)) and the reduced affine
     operators A0 = sum_j dU_j^T D_j dU_j, A_t,k = sum_j dU_j^T M_k dU_j,
     A_s,k = -(dU^iso)^T M_k dU^rho for the material classes k (Sec. 3.1.1).
"""
import ctypes
from dataclasses import dataclass

import numpy as np

from . import problems
from .rte import _check, _ptr, _stream, lib

_vp = ctypes.c_void_p
lib.rte_pod_snapshots.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_longlong, _vp]
lib.rte_gram.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_longlong, _vp, ctypes.c_int,
                         ctypes.c_longlong, ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp]
lib.rte_sym_eig.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
lib.rte_combine.argtypes = [_vp, ctypes.c_int, ctypes.c_longlong, _vp, ctypes.c_int, _vp, _vp]
lib.rte_apply_streaming.argtypes = [_vp, _vp, ctypes.c_int, _vp, _vp]
lib.rte_direction_sum.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp]
lib.rte_inflow_loads.argtypes = [_vp, _vp, ctypes.c_int, _vp, _vp]


@dataclass
class RomArrays:
    U_rho: np.ndarray      # [N_DOF, r]
    U_iso: np.ndarray      # [N_DOF, r]
    A0: np.ndarray         # [r, r]
    A: np.ndarray          # [2 * n_class, r, r]: sigma_t classes then sigma_s classes
    sv: np.ndarray         # singular values of the snapshot matrix (descending)
    eps_pod: float
    eps_train: float
    n_sweep_train: np.ndarray
    b_inflow: np.ndarray = None   # [4, r] reduced loads of unit side inflows (initial guess)


def gram(X, Y, cell_class=None, K=4, ncell=1, cls=0, scratch=None):
    """G = X^T Y for column-major X [nx, len], Y [ny, len] (CUDA float64)."""
    import torch
    nx, L = X.shape
    ny = Y.shape[0]
    G = torch.empty((nx, ny), dtype=torch.float64, device=X.device)
    if scratch is None:
        scratch = torch.empty(4096 * nx * ny + 256, dtype=torch.float64, device=X.device)
    _check(lib.rte_gram(_ptr(X), nx, _ptr(Y), ny, L, _ptr(cell_class), K, ncell, cls, _ptr(G),
                        _ptr(scratch), scratch.numel() * 8, _stream()), "rte_gram")
    return G


def sym_eig(G):
    import torch
    n = G.shape[0]
    A = G.clone()
    ev = torch.empty(n, dtype=torch.float64, device=G.device)
    V = torch.empty((n, n), dtype=torch.float64, device=G.device)
    _check(lib.rte_sym_eig(_ptr(A), n, _ptr(ev), _ptr(V), _stream()), "rte_sym_eig")
    return ev, V


def combine(X, W):
    import torch
    ncol, L = X.shape
    r = W.shape[1]
    out = torch.empty((r, L), dtype=torch.float64, device=X.device)
    _check(lib.rte_combine(_ptr(X), ncol, L, _ptr(W.contiguous()), r, _ptr(out), _stream()), "rte_combine")
    return out


def apply_streaming(P, x):
    import torch
    y = torch.empty_like(x)
    _check(lib.rte_apply_streaming(P.handle, _ptr(x), x.shape[0], _ptr(y), _stream()),
           "rte_apply_streaming")
    return y


def inflow_loads(P, U3):
    """[4, nvec] projections of unit side-inflow loads on U3 [nvec][n_dir][N_DOF]."""
    import torch
    out = torch.empty((4, U3.shape[0]), dtype=torch.float64, device=U3.device)
    _check(lib.rte_inflow_loads(P.handle, _ptr(U3.contiguous()), U3.shape[0], _ptr(out), _stream()),
           "rte_inflow_loads")
    return out


def direction_sum(P, x, weighted):
    import torch
    out = torch.empty((x.shape[0], P.ndof), dtype=torch.float64, device=x.device)
    _check(lib.rte_direction_sum(P.handle, _ptr(x), x.shape[0], int(bool(weighted)), _ptr(out),
                                 _stream()), "rte_direction_sum")
    return out


def snapshot_columns(P, f_final, f_iters, window):
    """[B * window, n_dir * N_DOF] columns f_b - f_b^(l), l = 0..window-1 (f^(0) = 0)."""
    import torch
    L = P.n_dir * P.ndof
    cols = torch.empty((P.B, window, L), dtype=torch.float64, device=f_final.device)
    for l in range(window):
        src = None if l == 0 else f_iters[l - 1]
        _check(lib.rte_pod_snapshots(P.handle, _ptr(f_final), _ptr(src), _ptr(cols[:, l]),
                                     window * L, _stream()), "rte_pod_snapshots")
    return cols.view(P.B * window, L)


def training_solves(P, window, eps_train, cg_rtol=1e-12, max_iter=500):
    """Converged f and the iterates f^(1..window-1) of FP64 SI-DSA from zero."""
    import torch
    from . import rte
    ws = P.workspace("si_dsa", None, "fp64", max_iter)
    shape = rte.f_shape(P)                   # the sweep's layout
    f_final = torch.empty(shape, dtype=torch.float64, device="cuda")
    rho = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.sisa_solve(P, rho, mode="si_dsa", eps=eps_train, max_iter=max_iter, cg_rtol=cg_rtol,
                         precision="fp64", f_out=f_final, ws=ws)
    if res.status != rte.RTE_OK:
        raise RuntimeError(f"training solves did not converge: {res.inst_status}")
    iters = []
    for l in range(1, window):
        fl = torch.empty(shape, dtype=torch.float64, device="cuda")
        rho.zero_()
        rte.sisa_solve(P, rho, mode="si_dsa", eps=eps_train, max_iter=l, cg_rtol=cg_rtol,
                       precision="fp64", f_out=fl, ws=ws, raise_on_error=False)
        iters.append(fl)
    return f_final, iters, res.n_sweep


def build_correction_rom(train_plane, r=20, window=3, eps_train=1e-10, eps_pod=None,
                         cg_rtol=1e-12, classes=None) -> RomArrays:
    """Correction ROM of rank r (or by eps_pod) from the training instances of ``train_plane``.

    ``classes``: material class of every cell (default: the block map of the lattice); the
    affine parameters are then (sigma_t per class, sigma_s per class).
    """
    import torch
    P = problems.plane_problem(train_plane)
    f_final, f_iters, n_sweep = training_solves(P, window, eps_train, cg_rtol)
    cols = snapshot_columns(P, f_final, f_iters, window)
    del f_iters
    G = gram(cols, cols)
    ev, V = sym_eig(G)
    ev_h = ev.cpu().numpy()
    order = np.argsort(-ev_h, kind="stable")
    sv = np.sqrt(np.clip(ev_h[order], 0.0, None))
    if r is None:
        ratio = np.cumsum(sv) / np.sum(sv)
        r = int(np.argmax(ratio >= 1.0 - eps_pod) + 1)
    r = min(r, int(np.sum(sv > sv[0] * 1e-13)))
    eps_eff = float(max(0.0, 1.0 - np.sum(sv[:r]) / np.sum(sv)))
    Vh = V.cpu().numpy()[:, order[:r]] / sv[:r]
    W = torch.as_tensor(np.ascontiguousarray(Vh), device="cuda")
    dU = combine(cols, W)                         # [r, n_dir * N_DOF]
    del cols
    dU3 = dU.view(r, P.n_dir, P.ndof)
    U_rho = direction_sum(P, dU3, True)           # [r, N_DOF]
    U_iso = direction_sum(P, dU3, False)
    DdU = apply_streaming(P, dU3)
    A0 = gram(dU, DdU.view(r, -1))
    if classes is None:
        classes = train_plane.block.reshape(-1)
    classes = np.asarray(classes, dtype=np.int32).reshape(-1)
    ncls = int(classes.max()) + 1
    cls_d = torch.as_tensor(classes, device="cuda")
    scratch = torch.empty(4096 * r * r + 256, dtype=torch.float64, device="cuda")
    At = [gram(dU, dU, cls_d, 4, P.ncell, k, scratch) for k in range(ncls)]
    As = [-gram(U_iso, U_rho, cls_d, 4, P.ncell, k, scratch) for k in range(ncls)]
    A = torch.stack(At + As).cpu().numpy()
    b_in = inflow_loads(P, dU3).cpu().numpy()
    torch.cuda.synchronize()
    return RomArrays(U_rho.T.contiguous().cpu().numpy(), U_iso.T.contiguous().cpu().numpy(),
                     A0.cpu().numpy(), A, sv, eps_eff, eps_train, np.asarray(n_sweep), b_in)


def build_parametric_rom(train_plane, r=20, eps_train=1e-10, eps_pod=None, cg_rtol=1e-12,
                         classes=None) -> RomArrays:
    """Parametric ROM of Sec. 3.1 for the ROM initial guess (eq. (rom_parametric)): POD of the
    converged angular fluxes of the training parameters.  Those are the snapshot columns of the
    correction ROM with a one-iterate window (f - f^(0) = f), so the same construction applies;
    the reduced unit-inflow loads come with it."""
    return build_correction_rom(train_plane, r=r, window=1, eps_train=eps_train, eps_pod=eps_pod,
                                cg_rtol=cg_rtol, classes=classes)
