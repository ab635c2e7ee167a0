"""Oracle: DSA-preconditioned restarted GMRES (the paper's Krylov baseline, Sec. 2.4 and the
appendix on restarted GMRES).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

SI solves rho = L rho + b_bar (eq. (rho_matrix_vec)), i.e. (I - L) rho = b_bar, with
  L v    the density of one transport sweep of the source Sigma_s v (no G, vacuum inflow);
  b_bar  the density of one sweep from rho = 0 (G and the inflow).
Viewing SI-DSA as a fixed-point iteration gives the left-preconditioned system
  (I + C Sigma_s)(I - L) rho = (I + C Sigma_s) b_bar,
C Sigma_s u being the DSA correction for the residual u (eq. (diffusion_correction) with
rho^* - rho = u).  GMRES(m) on it:
  - Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg matrix;
  - stop when the estimated preconditioned residual falls to tol * ||M^-1 b_bar||, then form the
    iterate, recompute the true preconditioned residual (one sweep) and stop if it also passes,
    otherwise restart from the iterate; a restart after m steps does the same.
Sweeps are counted as the method performs them: one for b_bar, one for every (re)start residual
(including the final check), one per Arnoldi step.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from .dsa import make_dsa


@dataclass
class PgmresResult:
    rho: np.ndarray
    n_sweep: int
    iterations: int             # Arnoldi steps over all cycles
    converged: bool
    residuals: List[float] = field(default_factory=list)   # estimated relative residual per step


def pgmres(disc, tol=1e-10, m=25, max_cycles=40, rho0=None, dsa=None, precondition=True):
    n = disc.ndof
    if precondition and dsa is None:
        dsa = make_dsa(disc)
    count = [0]

    def sweep_L(v):                      # L v: no source G, vacuum inflow
        count[0] += 1
        return disc.sweep(v, src=disc.apply_Ss(v), zero_bc=True)[0]

    def minv(u):                         # (I + C Sigma_s) u
        if not precondition:
            return u
        return u + dsa.correct(disc.apply_Ss(u).reshape(-1))

    count[0] += 1
    b_bar = disc.sweep(np.zeros(n))[0]
    nb = float(np.linalg.norm(minv(b_bar)))
    x = np.zeros(n) if rho0 is None else np.asarray(rho0, dtype=np.float64).copy()
    res = PgmresResult(x, 0, 0, False)
    for _ in range(max_cycles):
        r = minv(b_bar - x + sweep_L(x))     # M^-1 (b - A x), A = I - L
        beta = float(np.linalg.norm(r))
        if beta <= tol * nb:
            res.converged = True
            break
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k_used = 0
        for i in range(m):
            w = minv(V[i] - sweep_L(V[i]))
            res.iterations += 1
            for k in range(i + 1):               # modified Gram-Schmidt
                H[k, i] = float(np.dot(w, V[k]))
                w = w - H[k, i] * V[k]
            H[i + 1, i] = float(np.linalg.norm(w))
            V.append(w / H[i + 1, i] if H[i + 1, i] > 0 else w)
            for k in range(i):                   # earlier rotations on the new column
                t = cs[k] * H[k, i] + sn[k] * H[k + 1, i]
                H[k + 1, i] = -sn[k] * H[k, i] + cs[k] * H[k + 1, i]
                H[k, i] = t
            d = float(np.hypot(H[i, i], H[i + 1, i]))
            cs[i], sn[i] = H[i, i] / d, H[i + 1, i] / d
            H[i, i], H[i + 1, i] = d, 0.0
            g[i + 1] = -sn[i] * g[i]
            g[i] = cs[i] * g[i]
            k_used = i + 1
            res.residuals.append(abs(g[i + 1]) / nb)
            if abs(g[i + 1]) <= tol * nb:
                break
        y = sla.solve_triangular(H[:k_used, :k_used], g[:k_used])
        x = x + sum(y[k] * V[k] for k in range(k_used))
    res.rho = x
    res.n_sweep = count[0]
    return res
