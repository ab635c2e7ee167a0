"""Pins of two oracle parts that the other CPU tests leave open (no GPU):

* ROMIG (Sec. 3.1, eq. (rom_parametric)): the parametric ROM's Galerkin initial guess.
* The boundary-face terms of the MIP diffusion form used as the 2D DSA operator (the reading of
  eq. (diffusion_correction) in two dimensions).
"""
import numpy as np

import rte_workloads as W
from oracle import dsa as D, rom as R
from oracle.brute import BruteForce
from oracle.problem import discretize
from oracle.sisa import sisa


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


# ---------------------------------------------------------------------------- ROMIG
def test_romig_reproduces_training_solutions_exactly():
    """Sec. 3.1: the parametric basis spans the training solutions f^mu.  Untruncated (r equal to
    the number of training solves), the trial space of eq. (rom_parametric) at a training mu
    contains the exact solution of eq. (one_equation), so the Galerkin system U^T A_mu U c =
    U^T b_mu returns it: the guess U^rho c equals the training density (here checked against the
    dense global solve) and SI-DSA started from it stops after its first sweep.  The instances
    carry both a source G and a nonzero inflow on every side, so a load vector missing either
    part, a wrong reduced operator term or the wrong density map (U^iso instead of U^rho) fails."""
    train = W.random_plane(11, nx=6, ny=5, n_phi=8, B=4, inflow=True)
    discs = [discretize(train, b) for b in range(train.B)]
    assert np.all(train.g > 0.0) and np.all(train.G.sum(axis=(1, 2)) > 0.0)
    rom = R.build_parametric_rom(discs, R.plane_affine(discs[0]), R.plane_psi, r=train.B,
                                 eps_train=1e-14)
    assert rom.U.shape[1] == train.B
    for d in discs:
        _, rho_exact = BruteForce(d).solve()
        guess = rom.initial_guess(d)
        assert _rel(guess, rho_exact) < 1e-10, _rel(guess, rho_exact)
        assert sisa(d, "si_dsa", eps=1e-9, rho0=guess).n_sweep == 1


def test_romig_guess_improves_a_new_parameter():
    """Outside the training set the guess is an approximation (Sec. 3.1): started from it,
    SI-DSA needs fewer sweeps than from zero (the paper's Tables 3-11 show the same)."""
    train = W.c2_lattice([30000 + i for i in range(6)], n=8, n_phi=8, left_inflow=True)
    discs = [discretize(train, b) for b in range(train.B)]
    rom = R.build_parametric_rom(discs, R.plane_affine(discs[0]), R.plane_psi, r=6,
                                 eps_train=1e-12)
    test = W.c2_lattice([20000, 20001], n=8, n_phi=8, left_inflow=True)
    for b in range(test.B):
        d = discretize(test, b)
        cold = sisa(d, "si_dsa", eps=1e-10)
        warm = sisa(d, "si_dsa", eps=1e-10, rho0=rom.initial_guess(d))
        assert warm.converged and warm.n_sweep < cold.n_sweep, (warm.n_sweep, cold.n_sweep)
        assert _rel(warm.rho, cold.rho) < 1e-8


# ------------------------------------------------------------ MIP boundary terms
def _leg(t):
    """Orthonormal-on-[-1,1]-up-to-scale Legendre pair L0 = 1, L1 = sqrt(3) t and derivatives."""
    t = np.asarray(t, dtype=np.float64)
    return (np.ones_like(t), np.sqrt(3.0) * t), (np.zeros_like(t), np.full_like(t, np.sqrt(3.0)))


def _basis(x0, y0, hx, hy, x, y):
    """phi_ab = L_a(xi) L_b(eta) / sqrt(hx hy) on one cell, k = a + 2 b: values and gradient."""
    (lx, dlx), (ly, dly) = _leg(2 * (x - x0) / hx - 1), _leg(2 * (y - y0) / hy - 1)
    s = 1.0 / np.sqrt(hx * hy)
    val = np.stack([lx[a] * ly[b] * s for b in range(2) for a in range(2)])
    gx = np.stack([dlx[a] * (2 / hx) * ly[b] * s for b in range(2) for a in range(2)])
    gy = np.stack([lx[a] * dly[b] * (2 / hy) * s for b in range(2) for a in range(2)])
    return val, gx, gy


def test_mip_boundary_terms_manufactured_with_nonzero_trace():
    """The MIP boundary form  int_e kappa_b u w - 1/2 D d_n u w - 1/2 u D d_n w  is consistent with
    the boundary data functional  l(w) = int_e (1/2 D d_n u + kappa_b u) w - 1/2 u D d_n w  of the
    exact solution (integrating the volume term by parts leaves + int_e D d_n u w on every boundary
    edge; the form then differs from it by exactly l).  So for u = exp(0.7 x - 0.4 y) (1 + x y),
    whose trace and normal derivative vanish nowhere on the boundary, the discrete solution of
    A U = (S, w) + l(w) with S = -D lap u + sigma_a u converges at O(h^2) in L2.  A wrong factor
    on kappa_b, on either 1/2 D d_n term, a wrong normal sign or a missing boundary edge breaks
    the consistency and the rate."""
    sa = 0.7
    L = 1.0
    errs = []
    for n in (8, 16, 32):
        d = discretize(W.plane_uniform(n, 1.0 + sa, 1.0, 0.0, n_phi=8, L=L))
        m = D.MIPDSA2D(d)
        Dc = float(m.Dx[0])
        assert np.allclose(m.Dx, Dc) and np.allclose(m.Dy, Dc)
        h = d.hx
        u = lambda x, y: np.exp(0.7 * x - 0.4 * y) * (1 + x * y)
        ux = lambda x, y: np.exp(0.7 * x - 0.4 * y) * (0.7 * (1 + x * y) + y)
        uy = lambda x, y: np.exp(0.7 * x - 0.4 * y) * (-0.4 * (1 + x * y) + x)
        lap = lambda x, y: np.exp(0.7 * x - 0.4 * y) * ((0.49 + 0.16) * (1 + x * y) + 1.4 * y - 0.8 * x)
        S = lambda x, y: -Dc * lap(x, y) + sa * u(x, y)
        # volume load (S, phi_k): 4-point Gauss per axis is exact enough for O(h^2) here
        gx_, gw_ = np.polynomial.legendre.leggauss(4)
        rhs = np.zeros((n * n, 4))
        X, Y = np.meshgrid(0.5 * h * (1 + gx_), 0.5 * h * (1 + gx_), indexing="ij")
        Wq = np.outer(gw_, gw_).ravel() * 0.25 * h * h
        for j in range(n):
            for i in range(n):
                px, py = i * h + X.ravel(), j * h + Y.ravel()
                val, _, _ = _basis(i * h, j * h, h, h, px, py)
                rhs[j * n + i] += val @ (S(px, py) * Wq)
        # boundary functional on the four sides (outward normal n), kappa_b as the form's reading
        kmin_x = float(np.sum(d.w[d.vx > 0] * d.vx[d.vx > 0]))
        kmin_y = float(np.sum(d.w[d.vy > 0] * d.vy[d.vy > 0]))
        t = 0.5 * h * (1 + gx_)
        we = 0.5 * h * gw_
        for k in range(n):
            for side in range(4):
                if side < 2:     # x = 0 (n = -x) or x = L (n = +x), cell row k
                    i, nx_, ny_ = (0, -1.0, 0.0) if side == 0 else (n - 1, 1.0, 0.0)
                    c = k * n + i
                    px = np.full_like(t, 0.0 if side == 0 else L)
                    py = k * h + t
                    kap = max(kmin_x, 4.0 * Dc / h)
                else:            # y = 0 (n = -y) or y = L (n = +y), cell column k
                    j, nx_, ny_ = (0, 0.0, -1.0) if side == 2 else (n - 1, 0.0, 1.0)
                    c = j * n + k
                    px = k * h + t
                    py = np.full_like(t, 0.0 if side == 2 else L)
                    kap = max(kmin_y, 4.0 * Dc / h)
                ci, cj = c % n, c // n
                val, gx, gy = _basis(ci * h, cj * h, h, h, px, py)
                dnw = nx_ * gx + ny_ * gy
                dnu = nx_ * ux(px, py) + ny_ * uy(px, py)
                uu = u(px, py)
                rhs[c] += val @ ((0.5 * Dc * dnu + kap * uu) * we) - 0.5 * Dc * (dnw @ (uu * we))
        U = m.correct(rhs.reshape(-1)).reshape(n * n, 4)
        # L2 error against the exact u by 4-point Gauss per cell
        e2 = 0.0
        for j in range(n):
            for i in range(n):
                px, py = i * h + X.ravel(), j * h + Y.ravel()
                val, _, _ = _basis(i * h, j * h, h, h, px, py)
                e2 += np.sum((U[j * n + i] @ val - u(px, py)) ** 2 * Wq)
        errs.append(np.sqrt(e2))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)
