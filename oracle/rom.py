"""Oracle: POD reduced-order models (paper Sec. 3).

Test infrastructure only -- never imported by the product path.

* Correction ROM (Sec. 3.2.1): snapshots delta f^(mu,l) = f^mu - f^(mu,l),
  over a window of min(n_conv, window) iterates, from ordinary SI-DSA runs; SVD; truncation by
  eq. (pod_truncation) (ratio of partial sums of singular values) or a fixed
  rank; delta U^rho = sum_j w_j delta U_j and delta U^iso = sum_j delta U_j
  (eq. (rho_basis)); reduced affine operators (Sec. 3.1.1 "Offline
  precomputations").
* ROMSA (Sec. 3.2.2, eq. (rom_correction)): y = (delta U^iso)^T Sigma_s
  (rho^* - rho), A_r(mu) = sum_k psi_k(mu) A_k,r, delta c = A_r^{-1} y by LU
  with partial pivoting, delta rho = delta U^rho delta c.
* Parametric ROM and ROMIG (Sec. 3.1, eq. (rom_parametric)).

Affine split used for the reduced operators (eq. (one_equation)):
  A_mu = blockdiag_j(D_j) + I_{N_v} (x) Sigma_t(mu) - (1 w^T) (x) Sigma_s(mu),
  Sigma_t(mu) = sum_k psi^t_k(mu) T_k,  Sigma_s(mu) = sum_k psi^s_k(mu) S_k,
so that delta U^T A_mu delta U = sum_j dU_j^T D_j dU_j
  + sum_k psi^t_k sum_j dU_j^T T_k dU_j - sum_k psi^s_k (dU^iso)^T S_k dU^rho.
"""
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .sisa import sisa

ETA = 0.1   # Sec. 4: eta = 0.1 in eq. (romsad_parameters)


@dataclass
class Affine:
    """Sigma_t(mu) = sum psi_t[k] T[k], Sigma_s(mu) = sum psi_s[k] S[k] (sparse N_DOF x N_DOF)."""
    T: List[sp.spmatrix]
    S: List[sp.spmatrix]


def plane_affine(disc) -> Affine:
    """Block lattices: T_b = S_b = indicator of the dofs of material block b.  A medium given by
    cell fields (sigma = sum_k coefficient_k field_k): T_k = S_k = the field on the diagonal."""
    fields = getattr(disc, "block_fields", None)
    if fields is not None:
        diag = [sp.diags(np.repeat(np.asarray(f, np.float64).reshape(-1), 4)).tocsr() for f in fields]
        return Affine(diag, diag)
    nb = int(disc.block.max()) + 1
    masks = [sp.diags(np.repeat((disc.block == b).astype(np.float64), 4)).tocsr() for b in range(nb)]
    return Affine(masks, masks)


def plane_psi(disc):
    return np.asarray(disc.block_sigma_t, dtype=np.float64), np.asarray(disc.block_sigma_s, dtype=np.float64)


def pod_rank(sv, eps_pod):
    """Smallest l with sum_{k<=l} lambda_k / sum_k lambda_k >= 1 - eps_POD (eq. (pod_truncation))."""
    sv = np.asarray(sv, dtype=np.float64)
    ratio = np.cumsum(sv) / np.sum(sv)
    return int(np.argmax(ratio >= 1.0 - eps_pod) + 1)


def pod_dropped(sv, r):
    """Energy ratio dropped by keeping r singular values: 1 - sum_{k<=r} lambda_k / sum lambda_k."""
    sv = np.asarray(sv, dtype=np.float64)
    return float(max(0.0, 1.0 - np.sum(sv[:r]) / np.sum(sv)))


def reduced_operators(disc, U, affine: Affine, log=None):
    """(A0, At[k], As[k]) for a basis U [N_v N_DOF, r] (Sec. 3.1.1).  log (optional) is called
    with a line after every affine term."""
    nv, n = disc.nv, disc.ndof
    r = U.shape[1]
    Uj = U.reshape(nv, n, r)
    U_rho = np.einsum("j,jnr->nr", disc.w, Uj)
    U_iso = Uj.sum(axis=0)
    A0 = np.zeros((r, r))
    for c in range(r):
        DU = disc.apply_D(Uj[:, :, c])                 # [nv, n]
        A0[:, c] = np.einsum("jnr,jn->r", Uj, DU)
    At = []
    for k, T in enumerate(affine.T):
        At.append(sum(Uj[j].T @ (T @ Uj[j]) for j in range(nv)))
        if log:
            log(f"reduced operator: sigma_t term {k + 1} of {len(affine.T)}")
    As = [-(U_iso.T @ (S @ U_rho)) for S in affine.S]
    return A0, At, As, U_rho, U_iso


@dataclass
class CorrectionROM:
    dU_rho: np.ndarray          # [N_DOF, r]
    dU_iso: np.ndarray          # [N_DOF, r]
    A0: np.ndarray              # [r, r]
    At: List[np.ndarray]        # per T_k
    As: List[np.ndarray]        # per S_k
    sv: np.ndarray              # singular values of delta F
    eps_pod: float
    eps_train: float
    psi_fn: object = None       # disc -> (psi_t, psi_s)
    dU: Optional[np.ndarray] = None
    n_singular: int = 0

    @property
    def r(self):
        return self.dU_rho.shape[1]

    def eps_romsad(self, eta=ETA):
        return eta * max(self.eps_train, self.eps_pod)

    def reduced_matrix(self, disc):
        pt, ps = self.psi_fn(disc)
        A = self.A0.copy()
        for k, p in enumerate(pt):
            A += p * self.At[k]
        for k, p in enumerate(ps):
            A += p * self.As[k]
        return A

    def correct(self, disc, resid_src):
        """ROMSA correction; returns None if the reduced system is (numerically) singular."""
        y = self.dU_iso.T @ np.asarray(resid_src).reshape(-1)
        A = self.reduced_matrix(disc)
        lu, piv = sla.lu_factor(A, check_finite=True)
        if np.min(np.abs(np.diag(lu))) < 1e-14 * np.max(np.abs(A)):
            self.n_singular += 1
            return None
        dc = sla.lu_solve((lu, piv), y)
        return self.dU_rho @ dc


def correction_snapshots(discs, window, eps_train, relative=True, dsa_factory=None, first=0):
    """delta F columns f^mu - f^(mu,l) from SI-DSA runs with zero initial guess (Sec. 3.2.1).

    The window holds min(n_conv, window) consecutive iterates starting at l = ``first``.
    ``first = 0`` counts the zero initial state f^(0) = 0 as the first iterate (so the
    converged f^mu itself is a column); this is the reading under which the ranks
    printed in Table 2 are reproduced exactly.  ``first = 1`` starts at the first
    sweep, as the prose of Sec. 3.2.1 reads literally.
    """
    cols = []
    for d in discs:
        dsa = dsa_factory(d) if dsa_factory else None
        res = sisa(d, "si_dsa", eps=eps_train, relative=relative, dsa=dsa, want_f=True,
                   window=window)
        assert res.converged, "training solve did not converge"
        hist = [np.zeros_like(res.f)] + res.window          # hist[l] = f^(l)
        for l in range(first, first + min(res.n_sweep, window)):
            cols.append((res.f - hist[l]).reshape(-1))
    return np.stack(cols, axis=1)


def build_correction_rom(discs, affine, psi_fn, window=3, r=None, eps_pod=None,
                         eps_train=1e-10, relative=True, keep_full=False, dsa_factory=None,
                         first=0):
    dF = correction_snapshots(discs, window, eps_train, relative, dsa_factory, first)
    return correction_rom_from_snapshots(dF, discs[0], affine, psi_fn, r, eps_pod, eps_train,
                                         keep_full)


def correction_rom_from_snapshots(dF, disc, affine, psi_fn, r=None, eps_pod=None,
                                  eps_train=1e-10, keep_full=False, log=None):
    """POD of given snapshot columns dF [N_v N_DOF, n_col] (thin SVD, Sec. 3.1), truncation at
    rank r or by eq. (pod_truncation), and the reduced operators on the discretization ``disc``
    (any instance: only its mesh and directions enter)."""
    U, sv, _ = np.linalg.svd(dF, full_matrices=False)
    if r is None:
        r = pod_rank(sv, eps_pod)
        eps_eff = float(eps_pod)
    else:
        r = min(r, U.shape[1])
        eps_eff = pod_dropped(sv, r)
    dU = np.ascontiguousarray(U[:, :r])
    A0, At, As, U_rho, U_iso = reduced_operators(disc, dU, affine, log)
    return CorrectionROM(U_rho, U_iso, A0, At, As, sv, eps_eff, eps_train, psi_fn,
                         dU if keep_full else None)


# ---------------------------------------------------------------------------
# Parametric ROM + ROM-based initial guess (Sec. 3.1)
# ---------------------------------------------------------------------------
@dataclass
class ParametricROM:
    U: np.ndarray               # [N_v N_DOF, r_p]
    U_rho: np.ndarray
    A0: np.ndarray
    At: List[np.ndarray]
    As: List[np.ndarray]
    sv: np.ndarray
    psi_fn: object

    def initial_guess(self, disc):
        """rho^(0) = U^rho c_mu with U_r^T A_mu U_r c_mu = U_r^T b_mu (eq. (rom_parametric))."""
        pt, ps = self.psi_fn(disc)
        A = self.A0 + sum(p * M for p, M in zip(pt, self.At)) + sum(p * M for p, M in zip(ps, self.As))
        b = (disc.Gvec()[None, :] + disc.bc_load()).reshape(-1)
        c = np.linalg.solve(A, self.U.T @ b)
        return self.U_rho @ c


def build_parametric_rom(discs, affine, psi_fn, r=None, eps_pod=None, eps_train=1e-10,
                         relative=True):
    cols = []
    for d in discs:
        res = sisa(d, "si_dsa", eps=eps_train, relative=relative, want_f=True)
        assert res.converged
        cols.append(res.f.reshape(-1))
    F = np.stack(cols, axis=1)
    U, sv, _ = np.linalg.svd(F, full_matrices=False)
    r = pod_rank(sv, eps_pod) if r is None else min(r, U.shape[1])
    Ur = np.ascontiguousarray(U[:, :r])
    A0, At, As, U_rho, _ = reduced_operators(discs[0], Ur, affine)
    return ParametricROM(Ur, U_rho, A0, At, As, sv, psi_fn)
