"""Offline construction of the correction ROM on the GPU (Sec. 3.1, 3.2.1, 3.1.1).

Orchestrates library entry points (argument marshalling only):
  1. FP64 f-form SI-DSA training solves (Alg. 1) that keep f^(1), f^(2), ... and the converged f,
     a chunk of training instances at a time;
  2. snapshot columns delta f = f - f^(l) for the window of iterates that starts at the zero
     initial state (so f itself is the first column), Sec. 3.2.1, stored in FP64 or FP32;
  3. the POD, dU = dF W with W = V_r S_r^-1 (the r largest singular values), by one of two routes:
     - QR (FP64 columns, the default for them): shifted CholeskyQR3 of dF from Gram matrices on
       the matrix cores and a one-sided Jacobi SVD of the small triangular factor, which keeps
       singular values far below the largest accurate; the basis dU is then formed, and
       dU^rho, dU^iso (eq. (rho_basis)), A0 = sum_j dU_j^T D_j dU_j, A_t,k = sum_j dU_j^T M_k dU_j,
       A_s,k = -(dU^iso)^T M_k dU^rho (Sec. 3.1.1) and the reduced unit-inflow loads come from it;
     - method of snapshots (FP32 columns): G = dF^T dF, Jacobi eigenpairs, and everything the
       reduced model needs formed from the columns and W without the basis itself:
       dU^rho = (sum_j w_j dF_j) W, A0 = W^T (dF^T D dF) W, A_t,k = W^T (dF^T M_k dF) W, ...  The
       Gram matrix squares the conditioning, so singular values below about 1e-8 of the largest
       lose accuracy; FP32 storage limits the columns to about 6e-8 of it anyway.
FP32 columns halve the memory of the snapshot matrix (all products accumulate in FP64), which
lets the 512^2 x 256-direction training set (192 columns of 2.7e8 values) fit on one device.
"""
import ctypes
from dataclasses import dataclass

import numpy as np

from . import problems
from .rte import PRECISIONS, _check, _ptr, _stream, lib

_vp = ctypes.c_void_p
_i, _ll = ctypes.c_int, ctypes.c_longlong
lib.rte_pod_snapshots.argtypes = [_vp, _vp, _vp, _vp, _ll, _i, _vp]
lib.rte_gram.argtypes = [_vp, _i, _i, _vp, _i, _i, _ll, _vp, _i, _ll, _i, _vp, _vp, ctypes.c_size_t,
                         _vp]
lib.rte_sym_eig.argtypes = [_vp, _i, _vp, _vp, _vp]
lib.rte_combine.argtypes = [_vp, _i, _ll, _vp, _i, _vp, _vp]
lib.rte_apply_streaming.argtypes = [_vp, _vp, _i, _i, _vp, _vp]
lib.rte_direction_sum.argtypes = [_vp, _vp, _i, _i, _i, _vp, _vp]
lib.rte_inflow_loads.argtypes = [_vp, _vp, _i, _i, _vp, _vp]
lib.rte_pod_weights.argtypes = [_vp, _vp, _i, _i, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]
lib.rte_small_gemm.argtypes = [_i, _i, _i, _i, ctypes.c_double, _vp, _vp, _vp, _vp]
lib.rte_chol_upper.argtypes = [_vp, _i, _i, _ll, _vp, _vp, _vp, _vp, _vp, _vp]
lib.rte_svd_jacobi.argtypes = [_vp, _i, _vp, _vp, _vp, _vp, _i, _vp, _vp]


def _prec(t):
    """Library precision code of a tensor's element type (float64 or float32)."""
    import torch
    if t.dtype == torch.float64:
        return PRECISIONS["fp64"]
    if t.dtype == torch.float32:
        return PRECISIONS["mixed"]
    raise TypeError(f"unsupported element type {t.dtype}")


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
    """G = X^T Y (FP64) for column-major X [nx, len], Y [ny, len] (CUDA float64 or float32)."""
    import torch
    nx, L = X.shape
    ny = Y.shape[0]
    G = torch.empty((nx, ny), dtype=torch.float64, device=X.device)
    if scratch is None:
        scratch = torch.empty(4096 * nx * ny + 256, dtype=torch.float64, device=X.device)
    _check(lib.rte_gram(_ptr(X), _prec(X), nx, _ptr(Y), _prec(Y), ny, L, _ptr(cell_class), K, ncell,
                        cls, _ptr(G), _ptr(scratch), scratch.numel() * 8, _stream()), "rte_gram")
    return G


def sym_eig(G):
    import torch
    n = G.shape[0]
    A = G.clone()
    ev = torch.empty(n, dtype=torch.float64, device=G.device)
    V = torch.empty((n, n), dtype=torch.float64, device=G.device)
    _check(lib.rte_sym_eig(_ptr(A), n, _ptr(ev), _ptr(V), _stream()), "rte_sym_eig")
    return ev, V


def pod_weights(ev, V, r=0, eps_pod=0.0):
    """(sv descending [ncol], W [ncol, r] = V Sigma^-1 of the kept columns, r, dropped share) from
    the eigenpairs of F^T F (rte_pod_weights); r = 0 truncates by eq. (pod_truncation)."""
    import torch
    n = ev.shape[0]
    sv = torch.empty(n, dtype=torch.float64, device=ev.device)
    W = torch.zeros((n, n), dtype=torch.float64, device=ev.device)
    r_out = torch.zeros(1, dtype=torch.int32, device=ev.device)
    e_out = torch.zeros(1, dtype=torch.float64, device=ev.device)
    _check(lib.rte_pod_weights(_ptr(ev.contiguous()), _ptr(V.contiguous()), n, int(r),
                               float(eps_pod), _ptr(sv), _ptr(W), _ptr(r_out), _ptr(e_out),
                               _stream()), "rte_pod_weights")
    rk = int(r_out.item())
    return sv.cpu().numpy(), W[:, :rk].contiguous(), rk, float(e_out.item())


def chol_upper(G, shift_rows=0):
    """(R, R^-1, info, dev) with G + shift I = R^T R (rte_chol_upper); shift_rows > 0: the shift of
    shifted CholeskyQR for the Gram matrix of a shift_rows x n matrix.  info: 0, or 1 + the
    index of a pivot that was not positive; dev = max |G - I|."""
    import torch
    n = G.shape[0]
    work = torch.empty((n, n), dtype=torch.float64, device=G.device)
    R = torch.empty_like(work)
    T = torch.empty_like(work)
    info = torch.zeros(1, dtype=torch.int32, device=G.device)
    dev = torch.zeros(1, dtype=torch.float64, device=G.device)
    _check(lib.rte_chol_upper(_ptr(G.contiguous()), n, int(shift_rows > 0), int(shift_rows),
                              _ptr(work), _ptr(R), _ptr(T), _ptr(info), _ptr(dev), _stream()),
           "rte_chol_upper")
    return R, T, int(info.item()), float(dev.item())


def svd_jacobi(A, max_sweeps=60):
    """(squared singular values [n] unsorted, right singular vectors V [n, n] as columns, A V) of a
    small square matrix by one-sided Jacobi (rte_svd_jacobi)."""
    import torch
    n = A.shape[0]
    work = torch.empty(2 * n * n, dtype=torch.float64, device=A.device)
    lam = torch.empty(n, dtype=torch.float64, device=A.device)
    V = torch.empty((n, n), dtype=torch.float64, device=A.device)
    US = torch.empty((n, n), dtype=torch.float64, device=A.device)
    sweeps = torch.zeros(1, dtype=torch.int32, device=A.device)
    _check(lib.rte_svd_jacobi(_ptr(A.contiguous()), n, _ptr(work), _ptr(lam), _ptr(V), _ptr(US),
                              int(max_sweeps), _ptr(sweeps), _stream()), "rte_svd_jacobi")
    if int(sweeps.item()) >= max_sweeps:
        raise RuntimeError(f"rte_svd_jacobi: not converged in {max_sweeps} sweeps")
    return lam, V, US


def small_gemm(A, B=None, trans_a=False, alpha=1.0):
    """alpha op(A) B on the device (rte_small_gemm); B None is the identity."""
    import torch
    A = A.contiguous()
    m, k = (A.shape[1], A.shape[0]) if trans_a else A.shape
    n = B.shape[1] if B is not None else k
    if B is not None:
        B = B.contiguous()
        assert B.shape[0] == k
    C = torch.empty((m, n), dtype=torch.float64, device=A.device)
    _check(lib.rte_small_gemm(int(trans_a), m, n, k, float(alpha), _ptr(A), _ptr(B), _ptr(C),
                              _stream()), "rte_small_gemm")
    return C


def combine(X, W):
    import torch
    ncol, L = X.shape
    r = W.shape[1]
    out = torch.empty((r, L), dtype=torch.float64, device=X.device)
    _check(lib.rte_combine(_ptr(X), ncol, L, _ptr(W.contiguous()), r, _ptr(out), _stream()), "rte_combine")
    return out


def apply_streaming(P, x):
    """D_j x_j (FP64) for x [nvec, n_dir, N_DOF] (float64 or float32)."""
    import torch
    y = torch.empty(x.shape, dtype=torch.float64, device=x.device)
    _check(lib.rte_apply_streaming(P.handle, _ptr(x), _prec(x), x.shape[0], _ptr(y), _stream()),
           "rte_apply_streaming")
    return y


def inflow_loads(P, U3):
    """[4, nvec] projections of unit side-inflow loads on U3 [nvec][n_dir][N_DOF]."""
    import torch
    U3 = U3.contiguous()
    out = torch.empty((4, U3.shape[0]), dtype=torch.float64, device=U3.device)
    _check(lib.rte_inflow_loads(P.handle, _ptr(U3), _prec(U3), U3.shape[0], _ptr(out), _stream()),
           "rte_inflow_loads")
    return out


def direction_sum(P, x, weighted):
    import torch
    out = torch.empty((x.shape[0], P.ndof), dtype=torch.float64, device=x.device)
    _check(lib.rte_direction_sum(P.handle, _ptr(x), _prec(x), x.shape[0], int(bool(weighted)),
                                 _ptr(out), _stream()), "rte_direction_sum")
    return out


def snapshot_columns(P, f_final, f_iters, window, out=None, dtype=None):
    """[B * window, n_dir * N_DOF] columns f_b - f_b^(l), l = 0..window-1 (f^(0) = 0), written
    into ``out`` (rows b * window + l) or a new FP64 array."""
    import torch
    L = P.n_dir * P.ndof
    if out is None:
        out = torch.empty((P.B * window, L), dtype=dtype or torch.float64, device=f_final.device)
    assert out.shape == (P.B * window, L) and out.is_contiguous()
    for l in range(window):
        src = None if l == 0 else f_iters[l - 1]
        _check(lib.rte_pod_snapshots(P.handle, _ptr(f_final), _ptr(src), _ptr(out[l]), window * L,
                                     _prec(out), _stream()), "rte_pod_snapshots")
    return out


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


def pod_qr(holder, r=None, eps_pod=None, scratch=None, max_passes=8, orth_tol=1e-12):
    """POD of FP64 snapshot columns by CholeskyQR and a one-sided Jacobi SVD of the triangular
    factor.  ``holder`` is a one-element list with X [ncol, len] (rows = the columns of F); it is
    emptied so that X can be freed after the first pass.

    F = X^T = Q R: each pass factors the Gram matrix of the current Q (the first Q is F) by
    Cholesky, G = R_k^T R_k, shifted as in shifted CholeskyQR when the plain factorization breaks
    down, and replaces Q by Q R_k^-1 (so R = ... R_2 R_1), until the Gram matrix of Q is the
    identity to orth_tol.  Then R = U S V^T (Jacobi) and the POD basis is Q U_r.  Returns
    (sv, Wq, r, dropped share, Q) with Q [ncol, len] and Wq [ncol, r] = U_r, so that the basis is
    combine(Q, Wq).  Unlike the eigenpairs of X X^T, singular values far below the largest keep
    their relative accuracy, and the basis is orthonormal to working precision."""
    Q = holder.pop()
    ncol, L = Q.shape
    R = None
    for it in range(max_passes):
        G = gram(Q, Q, scratch=scratch)
        Rk, Tk, info, dev = chol_upper(G)
        if it > 0 and dev <= orth_tol:
            break
        if info:
            Rk, Tk, info, _ = chol_upper(G, shift_rows=L)
            if info:
                raise RuntimeError(f"CholeskyQR: shifted factorization failed at pivot {info - 1}")
        Q = combine(Q, Tk)
        R = Rk if R is None else small_gemm(Rk, R)
    else:
        raise RuntimeError(f"CholeskyQR: columns not orthonormal after {max_passes} passes")
    lam, _, US = svd_jacobi(R)
    sv, Wq, rk, eps_eff = pod_weights(lam, US, 0 if r is None else r, eps_pod or 0.0)
    return sv, Wq, rk, eps_eff, Q


def build_correction_rom(train_plane, r=20, window=3, eps_train=1e-10, eps_pod=None,
                         cg_rtol=1e-12, classes=None, snapshot_dtype="fp64", chunk=None,
                         slice_cols=8, train_max_iter=500, pod="auto", log=None) -> RomArrays:
    """Correction ROM of rank r (or by eps_pod) from the training instances of ``train_plane``.

    ``classes``: material class of every cell (default: the material map of the description);
    the affine parameters are then (sigma_t per class, sigma_s per class).
    ``snapshot_dtype``: "fp64" or "fp32" storage of the snapshot columns.  ``chunk``: training
    instances solved together (default: all).  ``slice_cols``: columns per D dF slice.
    ``train_max_iter``: iteration limit of each training solve.
    ``pod``: "qr" (pod_qr, then every reduced quantity from the explicit orthonormal basis; FP64
    columns only, about three times the snapshot memory at its peak), "gram" (eigenpairs of the
    Gram matrix, every reduced quantity in snapshot space, no basis-sized memory), or "auto": "qr"
    for FP64 columns, "gram" for FP32 ones.
    """
    import torch
    say = log or (lambda *a: None)
    n_inst = train_plane.B
    chunk = chunk or n_inst
    L = None
    X = None
    n_sweep = []
    for c0 in range(0, n_inst, chunk):
        sub = train_plane.subset(range(c0, min(n_inst, c0 + chunk)))
        P = problems.plane_problem(sub)
        if X is None:
            L = P.n_dir * P.ndof
            dt = torch.float32 if snapshot_dtype == "fp32" else torch.float64
            X = torch.empty((n_inst * window, L), dtype=dt, device="cuda")
        f_final, f_iters, ns = training_solves(P, window, eps_train, cg_rtol, train_max_iter)
        snapshot_columns(P, f_final, f_iters, window, out=X[c0 * window:(c0 + sub.B) * window])
        n_sweep.extend(int(v) for v in ns)
        del f_final, f_iters, P
        say(f"training instances {c0}..{c0 + sub.B - 1}: sweeps {[int(v) for v in ns]}")
    torch.cuda.empty_cache()
    ncol = X.shape[0]
    Pm = problems.plane_problem(train_plane.instance(0))      # mesh and directions
    scratch = torch.empty(4096 * ncol * ncol + 256, dtype=torch.float64, device="cuda")
    if pod == "auto":
        pod = "qr" if X.dtype == torch.float64 else "gram"
    if pod not in ("qr", "gram"):
        raise ValueError(f"pod: 'qr', 'gram' or 'auto', not {pod!r}")
    if classes is None:
        if getattr(train_plane, "block_fields", None) is not None:
            raise ValueError("the offline builder forms class-restricted operators; a medium "
                             "given by cell fields needs its ROM built elsewhere")
        classes = train_plane.block.reshape(-1)
    classes = np.asarray(classes, dtype=np.int32).reshape(-1)
    ncls = int(classes.max()) + 1
    cls_d = torch.as_tensor(classes, device="cuda")
    if pod == "qr":
        if X.dtype != torch.float64:
            raise ValueError("the QR route of the POD needs FP64 snapshot columns")
        holder = [X]
        del X                                    # pod_qr frees the columns after its first pass
        sv, Wq, r, eps_eff, Q = pod_qr(holder, r, eps_pod, scratch)
        say(f"POD of {ncol} columns (CholeskyQR + Jacobi SVD): rank {r}, dropped energy "
            f"{eps_eff:.3e}")
        dU = combine(Q, Wq)                                      # [r, L], orthonormal
        del Q, scratch
        torch.cuda.empty_cache()
        dU3 = dU.view(r, Pm.n_dir, Pm.ndof)
        U_rho = direction_sum(Pm, dU3, True)                     # [r, N_DOF]
        U_iso = direction_sum(Pm, dU3, False)
        sc_r = torch.empty(4096 * r * r + 256, dtype=torch.float64, device="cuda")
        A0 = torch.empty((r, r), dtype=torch.float64, device="cuda")
        for s0 in range(0, r, slice_cols):
            s1 = min(r, s0 + slice_cols)
            DU = apply_streaming(Pm, dU3[s0:s1])
            A0[:, s0:s1] = gram(dU, DU.view(s1 - s0, L), scratch=sc_r)
            del DU
        say("streaming operator projected")
        At = [gram(dU, dU, cls_d, 4, Pm.ncell, k, sc_r) for k in range(ncls)]
        As = [small_gemm(gram(U_iso, U_rho, cls_d, 4, Pm.ncell, k, sc_r), alpha=-1.0)
              for k in range(ncls)]
        A = torch.stack(At + As).cpu().numpy()
        b_in = inflow_loads(Pm, dU3).cpu().numpy()
        torch.cuda.synchronize()
        return RomArrays(U_rho.T.contiguous().cpu().numpy(), U_iso.T.contiguous().cpu().numpy(),
                         A0.cpu().numpy(), A, sv, eps_eff, eps_train, np.asarray(n_sweep), b_in)
    G = gram(X, X, scratch=scratch)
    ev, V = sym_eig(G)
    sv, W, r, eps_eff = pod_weights(ev, V, 0 if r is None else r, eps_pod or 0.0)
    say(f"POD of {ncol} columns: rank {r}, dropped energy {eps_eff:.3e}")
    X3 = X.view(ncol, Pm.n_dir, Pm.ndof)
    U_rho = combine(direction_sum(Pm, X3, True), W)               # [r, N_DOF]
    U_iso = combine(direction_sum(Pm, X3, False), W)
    # dF^T D dF, a slice of columns of D dF at a time
    GD = torch.empty((ncol, ncol), dtype=torch.float64, device="cuda")
    for s0 in range(0, ncol, slice_cols):
        s1 = min(ncol, s0 + slice_cols)
        DX = apply_streaming(Pm, X3[s0:s1])
        GD[:, s0:s1] = gram(X, DX.view(s1 - s0, L), scratch=scratch)
        del DX
    A0 = small_gemm(W, small_gemm(GD, W), trans_a=True)
    say("streaming operator projected")
    At = [small_gemm(W, small_gemm(gram(X, X, cls_d, 4, Pm.ncell, k, scratch), W), trans_a=True)
          for k in range(ncls)]
    sc_r = torch.empty(4096 * r * r + 256, dtype=torch.float64, device="cuda")
    As = [small_gemm(gram(U_iso, U_rho, cls_d, 4, Pm.ncell, k, sc_r), alpha=-1.0)
          for k in range(ncls)]
    A = torch.stack(At + As).cpu().numpy()
    b_in = small_gemm(inflow_loads(Pm, X3), W).cpu().numpy()
    torch.cuda.synchronize()
    return RomArrays(U_rho.T.contiguous().cpu().numpy(), U_iso.T.contiguous().cpu().numpy(),
                     A0.cpu().numpy(), A, sv, eps_eff, eps_train, np.asarray(n_sweep), b_in)


def build_parametric_rom(train_plane, r=20, eps_train=1e-10, eps_pod=None, cg_rtol=1e-12,
                         classes=None, **kw) -> RomArrays:
    """Parametric ROM of Sec. 3.1 for the ROM initial guess (eq. (rom_parametric)): POD of the
    converged angular fluxes of the training parameters.  Those are the snapshot columns of the
    correction ROM with a one-iterate window (f - f^(0) = f), so the same construction applies;
    the reduced unit-inflow loads come with it."""
    return build_correction_rom(train_plane, r=r, window=1, eps_train=eps_train, eps_pod=eps_pod,
                                cg_rtol=cg_rtol, classes=classes, **kw)
