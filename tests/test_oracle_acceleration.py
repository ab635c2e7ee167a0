"""Pins of the oracle's synthetic-acceleration and ROM machinery (no GPU)."""
import json
import os

import numpy as np
import pytest

import rte_workloads as W
from oracle import dg, dsa as D, rom as R
from oracle.problem import discretize
from oracle.sisa import sisa

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ slab DSA (App. B)
def test_appendix_b_operators_reproduce_sweep_operator():
    """D_j = v_j (D_C - sign(v_j)/2 D_J) (Appendix B) must equal the D_j the sweep
    assembles from eq. (DG) -- two independent constructions."""
    d = discretize(W.random_slab(7, nc=9, n_dir=6))
    Dp, Dm = D.slab_Dpm(d.edges)
    DC, DJ = 0.5 * (Dp + Dm), Dp - Dm
    for j, Dj in enumerate(d.global_D()):
        M = d.mu[j] * (DC - np.sign(d.mu[j]) / 2 * DJ)
        assert abs(M - Dj).max() < 1e-12 * abs(Dj).max()


def test_consistent_dsa_is_exact_for_two_directions():
    """With S2 the P1 ansatz spans every angular flux, so the moment system of
    Appendix B is equivalent to the kinetic correction equation: SI-DSA converges
    in exactly two sweeps."""
    for seed in range(3):
        d = discretize(W.random_slab(seed, nc=11, n_dir=2))
        r = sisa(d, "si_dsa", eps=1e-12)
        assert r.n_sweep == 2, r.changes


def test_consistent_dsa_spectral_radius_slab():
    """Thick homogeneous slab, c = 0.999: SI contracts at ~c, consistent DSA far below."""
    d = discretize(W.slab_uniform(200, 200.0, 1.0, 0.999, 1.0, n_dir=16))
    rs = sisa(d, "si", eps=0.0, max_iter=60)
    rd = sisa(d, "si_dsa", eps=0.0, max_iter=12)
    cs, cd = np.array(rs.changes), np.array(rd.changes)
    assert cs[-1] / cs[-2] > 0.95
    assert np.max(cd[4:] / cd[3:-1]) < 0.3


def test_c0_slab_si_dsa():
    d = discretize(W.c0_slab())
    r = sisa(d, "si_dsa", eps=1e-10)
    s = sisa(d, "si", eps=1e-10)
    assert r.converged and s.converged and r.n_sweep < s.n_sweep
    assert np.abs(r.rho - s.rho).max() < 1e-9 * np.abs(r.rho).max()


# --------------------------------------------------------------- MIP diffusion
@pytest.mark.parametrize("L", [0.01, 1.0, 100.0])
def test_mip_symmetric_positive_definite(L):
    d = discretize(W.random_plane(3, nx=6, ny=5, n_phi=8, Lx=L, Ly=L))
    A = D.MIPDSA2D(d).A.toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


def test_mip_manufactured_order():
    """u = sin^2(pi x) sin^2(pi y) (u = d_n u = 0 on the boundary, so the MIP form is
    consistent): L2 error of the diffusion solve is O(h^2)."""
    errs = []
    for n in (8, 16, 32):
        d = discretize(W.plane_uniform(n, 2.0, 1.0, 0.0, n_phi=8))
        m = D.MIPDSA2D(d)
        Dc, sa = m.Dx[0], 1.0
        pi = np.pi
        u = lambda x, y: np.sin(pi * x) ** 2 * np.sin(pi * y) ** 2
        S = lambda x, y: (-Dc * 2 * pi ** 2 * (np.cos(2 * pi * x) * np.sin(pi * y) ** 2
                                              + np.sin(pi * x) ** 2 * np.cos(2 * pi * y)) + sa * u(x, y))
        U = m.correct(dg.plane_project(n, n, d.hx, d.hy, S).reshape(-1))
        errs.append(np.linalg.norm(U - dg.plane_project(n, n, d.hx, d.hy, u).reshape(-1)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), errs


def test_mip_dsa_accelerates():
    """Homogeneous medium, c = 0.99, 10 mean free paths: the SI contraction is ~0.92,
    the MIP-DSA contraction stays below 0.55 (documented effectiveness of the reading)."""
    d = discretize(W.plane_uniform(32, 1.0, 0.99, 1.0, n_phi=16, L=10.0))
    s = np.array(sisa(d, "si", eps=0.0, max_iter=30).changes)
    a = np.array(sisa(d, "si_dsa", eps=0.0, max_iter=15).changes)
    assert s[-1] / s[-2] > 0.9
    assert np.max(a[3:] / a[2:-1]) < 0.55


# ------------------------------------------------------------------------- ROM
@pytest.fixture(scope="module")
def small_rom():
    train = W.c2_lattice([30000 + i for i in range(4)], n=8, n_phi=8)
    discs = [discretize(train, b) for b in range(train.B)]
    rom = R.build_correction_rom(discs, R.plane_affine(discs[0]), R.plane_psi, window=3,
                                 r=1000, eps_train=1e-12, keep_full=True)
    return rom, discs


def test_rom_identities(small_rom):
    rom, discs = small_rom
    dU, d = rom.dU, discs[0]
    assert np.abs(dU.T @ dU - np.eye(rom.r)).max() < 1e-13
    Uj = dU.reshape(d.nv, d.ndof, rom.r)
    assert np.abs(rom.dU_rho - np.einsum("j,jnr->nr", d.w, Uj)).max() < 1e-15
    # projection of an isotropic right-hand side (paper: (dU^iso)^T Sigma_s (rho^* - rho))
    src = np.random.default_rng(0).normal(size=d.ndof)
    assert np.abs(dU.T @ np.tile(src, d.nv) - rom.dU_iso.T @ src).max() < 1e-12
    # density of a reduced solution
    c = np.random.default_rng(1).normal(size=rom.r)
    assert np.abs(d.w @ (dU @ c).reshape(d.nv, -1) - rom.dU_rho @ c).max() < 1e-13


def test_rom_affine_assembly_equals_direct_projection(small_rom):
    from oracle.brute import BruteForce
    rom, _ = small_rom
    test = W.c2_lattice([20001], n=8, n_phi=8)
    d = discretize(test, 0)
    direct = rom.dU.T @ (BruteForce(d).A @ rom.dU)
    assert np.abs(direct - rom.reduced_matrix(d)).max() < 1e-12 * np.abs(direct).max()


def test_romsa_exact_on_training_parameters(small_rom):
    """For mu in the training set with an untruncated basis, the first kinetic
    correction lies in span(delta U); the Galerkin projection reproduces it and
    SI-ROMSA converges in two sweeps."""
    rom, discs = small_rom
    for d in discs:
        r = sisa(d, "romsa", eps=1e-9, rom=rom)
        assert r.n_sweep == 2, r.changes


def test_romsad_mode_wiring(small_rom):
    """theta = 0 is SI-DSA; theta = inf with eps_ROMSAD = 0 is ROMSA (bitwise)."""
    rom, _ = small_rom
    d = discretize(W.c2_lattice([20002], n=8, n_phi=8), 0)
    a = sisa(d, "romsad", eps=1e-8, rom=rom, theta=0)
    b = sisa(d, "si_dsa", eps=1e-8)
    assert a.n_sweep == b.n_sweep and np.array_equal(a.rho, b.rho)
    c = sisa(d, "romsad", eps=1e-8, rom=rom, theta=10 ** 9, eps_romsad=0.0, max_iter=40)
    e = sisa(d, "romsa", eps=1e-8, rom=rom, max_iter=40)
    assert c.n_sweep == e.n_sweep and np.array_equal(c.rho, e.rho)
    # Alg. 2: ROMSA only while l <= theta and the change is >= eps_ROMSAD
    f = sisa(d, "romsad", eps=1e-8, rom=rom, theta=3)
    assert f.kinds[:3] == [2, 2, 2] and set(f.kinds[3:]) <= {1}


def test_pod_truncation_rule():
    sv = np.array([4.0, 2.0, 1.0, 0.5, 0.5])
    # cumulative ratios 0.5, 0.75, 0.875, 0.9375, 1
    assert R.pod_rank(sv, 0.25) == 2 and R.pod_rank(sv, 0.2) == 3 and R.pod_rank(sv, 0.0) == 5
    assert abs(R.pod_dropped(sv, 3) - 0.125) < 1e-15


@pytest.mark.slow
def test_table2_cross_regime_ranks():
    """Paper Table 2: r_p and r_c for the cross-regime training set.  Reproduced with
    the consistent DSA of Appendix B, the absolute stop test of Alg. 1, the
    sum-of-singular-values truncation of eq. (pod_truncation) and a correction
    window that starts at the zero initial state."""
    gold = json.load(open(os.path.join(GOLDEN, "table2_cross_regime_ranks.json")))
    discs = [discretize(W.cross_regime(m)) for m in W.cross_regime_training()]
    F, d1, d3 = [], [], []
    for d in discs:
        r = sisa(d, "si_dsa", eps=1e-11, relative=False, want_f=True, window=3)
        assert r.converged
        hist = [np.zeros_like(r.f)] + r.window
        F.append(r.f.reshape(-1))
        d1.append((r.f - hist[0]).reshape(-1))
        d3 += [(r.f - hist[l]).reshape(-1) for l in range(3)]
    for key, M in (("r_p", F), ("r_c_window1", d1), ("r_c_window3", d3)):
        sv = np.linalg.svd(np.stack(M, 1), compute_uv=False)
        got = [R.pod_rank(sv, e) for e in gold["eps_pod"]]
        assert got == gold[key], (key, got)
