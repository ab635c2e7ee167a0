"""The paper's pin-cell (Sec. 4.3.3) and variable-scattering (Sec. 4.3.4) families: the generated
media against their definitions, and the oracle's reduced operators for a medium affine in cell
fields (not piecewise constant) against direct Galerkin projection (CPU)."""
import numpy as np

import rte_workloads as W
from oracle import rom as R
from oracle.brute import BruteForce
from oracle.problem import discretize
from oracle.sisa import sisa


def test_pin_cell_medium_follows_its_definition():
    n = 16
    p = W.pin_cell([(0.2, 0.35)], n=n, quad=("cl", (4, 2)))
    h = 2.0 / n
    for iy in range(n):
        for ix in range(n):
            x, y = -1.0 + (ix + 0.5) * h, -1.0 + (iy + 0.5) * h
            pin = abs(x) <= 0.5 and abs(y) <= 0.5
            sa, ss = (0.2, 0.35) if pin else (0.0, 100.0)
            assert np.isclose(p.sigma_s[0, iy, ix], ss) and np.isclose(p.sigma_t[0, iy, ix], sa + ss)
            assert np.isclose(p.G[0, iy, ix], np.exp(-100.0 * (x * x + y * y)))
    assert np.all(p.g == 0.0)
    assert len(W.pin_cell_training()) == 25
    assert all(0.05 <= a <= 0.5 and 0.05 <= s <= 0.5 for a, s in W.pin_cell_test())


def test_variable_scattering_medium_follows_its_definition():
    n = 14
    mu = 77.4356
    p = W.variable_scattering([mu], n=n, quad=("cl", (4, 2)))
    h = 2.0 / n
    for iy in range(n):
        for ix in range(n):
            x, y = -1.0 + (ix + 0.5) * h, -1.0 + (iy + 0.5) * h
            r = np.hypot(x, y)
            ss = mu * r ** 4 * (2.0 - r * r) ** 2 + 0.1 if r <= 1.0 else mu + 0.1
            assert np.isclose(p.sigma_s[0, iy, ix], ss, rtol=1e-14)
            assert p.sigma_t[0, iy, ix] == p.sigma_s[0, iy, ix]          # no absorption
            assert np.isclose(p.G[0, iy, ix], 10.0 / np.pi * np.exp(-100.0 * r * r))
    tr = W.variable_scattering_training()
    assert len(tr) == 50 and tr[0] == 49.9 and np.isclose(tr[-1], 99.9)


def _fields_rom(n=6):
    train = W.variable_scattering([55.0, 70.0, 90.0], n=n, quad=("cl", (4, 2)))
    discs = [discretize(train, b) for b in range(train.B)]
    rom = R.build_correction_rom(discs, R.plane_affine(discs[0]), R.plane_psi, window=3, r=1000,
                                 eps_train=1e-12, keep_full=True)
    return rom, discs


def test_field_affine_assembly_equals_direct_projection():
    """sigma_t = sigma_s = mu_s s(x) + 0.1: the reduced operator assembled from the two field
    terms equals dU^T A_mu dU of the assembled global operator at a parameter outside the
    training set."""
    rom, _ = _fields_rom()
    d = discretize(W.variable_scattering([63.3], n=6, quad=("cl", (4, 2))), 0)
    direct = rom.dU.T @ (BruteForce(d).A @ rom.dU)
    assert np.abs(direct - rom.reduced_matrix(d)).max() < 1e-12 * np.abs(direct).max()


def test_field_romsa_exact_on_training_parameters():
    """With the untruncated basis, ROMSA's first correction is exact on a training parameter and
    source iteration stops after two sweeps (as for the block lattices)."""
    rom, discs = _fields_rom()
    for d in discs:
        assert sisa(d, "romsa", eps=1e-9, rom=rom).n_sweep == 2


def test_field_romig_reproduces_training_solutions():
    train = W.variable_scattering([55.0, 80.0], n=6, quad=("cl", (4, 2)))
    discs = [discretize(train, b) for b in range(train.B)]
    prom = R.build_parametric_rom(discs, R.plane_affine(discs[0]), R.plane_psi, r=1000,
                                  eps_train=1e-13)
    for d in discs:
        ref = sisa(d, "si_dsa", eps=1e-13)
        g = prom.initial_guess(d)
        assert np.abs(g - ref.rho).max() < 1e-9 * np.abs(ref.rho).max()
