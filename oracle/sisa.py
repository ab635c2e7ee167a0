"""Oracle: Source Iteration with Synthetic Acceleration (paper Alg. 1) and the
ROMSAD switch (paper Alg. 2, eq. (romsad_parameters)).

Test infrastructure only -- never imported by the product path.

Readings of the paper used here (each is a documented choice):
  * the change e_l = ||rho^(l,*) - rho^(l-1)||_inf is taken over the DG
    coefficient vector; with ``relative=True`` (default) it is divided by
    ||rho^(l,*)||_inf, with ``relative=False`` it is the absolute change of
    Alg. 1;
  * the same e_l is compared with eps_ROMSAD in Alg. 2;
  * the sweep uses the source Sigma_s rho + G (+ inflow), i.e.
    rho^(l,*) = L rho^(l-1) + bbar (eq. (rho_matrix_vec_def));
  * Alg. 1 returns the uncorrected rho^(l,*) and f^(l); n_sweep counts every
    sweep including the last one.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

KIND_NONE, KIND_DSA, KIND_ROMSA, KIND_EXACT = 0, 1, 2, 3


@dataclass
class SisaResult:
    rho: np.ndarray
    f: Optional[np.ndarray]
    n_sweep: int
    converged: bool
    changes: List[float] = field(default_factory=list)
    kinds: List[int] = field(default_factory=list)
    window: List[np.ndarray] = field(default_factory=list)   # f^(l), l = 1..window


def change_norm(rho_star, rho_prev, relative=True):
    d = float(np.max(np.abs(rho_star - rho_prev)))
    if relative:
        m = float(np.max(np.abs(rho_star)))
        return d / m if m > 0 else (0.0 if d == 0 else np.inf)
    return d


def sisa(disc, mode="si_dsa", eps=1e-8, max_iter=None, relative=True, rho0=None, dsa=None,
         rom=None, theta=5, eps_romsad=None, want_f=False, window=0, exact=None):
    """Alg. 1 on one discretized instance.

    mode: "si" (no correction), "si_dsa", "romsad" (Alg. 2), "romsa" (ROMSA in every
    iteration), "exact" (ideal kinetic correction, eq. (one_equation_correction), needs
    ``exact`` = brute-force solver).
    """
    if max_iter is None:
        max_iter = 10000 if mode == "si" else 500
    if mode in ("si_dsa", "romsad") and dsa is None:
        from .dsa import make_dsa
        dsa = make_dsa(disc)
    if mode in ("romsad", "romsa"):
        assert rom is not None
        if eps_romsad is None:
            eps_romsad = rom.eps_romsad()
    rho = np.zeros(disc.ndof) if rho0 is None else np.asarray(rho0, dtype=np.float64).copy()
    res = SisaResult(rho, None, 0, False)
    need_f = want_f or window > 0
    for l in range(1, max_iter + 1):
        rho_star, f = disc.sweep(rho, want_f=need_f)
        res.n_sweep = l
        if l <= window:
            res.window.append(f.copy())
        e = change_norm(rho_star, rho, relative)
        res.changes.append(e)
        if e < eps:
            res.rho, res.f, res.converged = rho_star, f, True
            return res
        resid_src = disc.apply_Ss(rho_star - rho).reshape(-1)
        if mode == "si":
            kind, delta = KIND_NONE, 0.0
        elif mode == "si_dsa":
            kind, delta = KIND_DSA, dsa.correct(resid_src)
        elif mode == "romsa":
            kind, delta = KIND_ROMSA, rom.correct(disc, resid_src)
        elif mode == "romsad":
            if 1 <= l <= theta and e >= eps_romsad:
                kind, delta = KIND_ROMSA, rom.correct(disc, resid_src)
                if delta is None:            # singular reduced system: DSA this iteration
                    kind, delta = KIND_DSA, dsa.correct(resid_src)
            else:
                kind, delta = KIND_DSA, dsa.correct(resid_src)
        elif mode == "exact":
            kind, delta = KIND_EXACT, exact.correction(rho_star, rho)
        else:
            raise ValueError(mode)
        res.kinds.append(kind)
        rho = rho_star + delta
    res.rho, res.f = rho_star, f
    return res


def residual(disc, rho):
    """R^rho_inf = ||(I - L) rho - bbar||_inf = ||rho - (L rho + bbar)||_inf (one extra sweep)."""
    r, _ = disc.sweep(rho)
    return float(np.max(np.abs(rho - r)))
