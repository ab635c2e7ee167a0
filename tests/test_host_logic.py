"""Host-side logic of the library package (no GPU): direction tables and serving bookkeeping."""
import numpy as np


def test_product_cl_rule_moments():
    """The library's host-side CL rule (used to build direction tables) integrates the sphere's
    low moments exactly: sum w = 1, sum w vx^2 = sum w vy^2 = 1/3, odd moments vanish."""
    from paper_2402_10488_amd import quadrature as pq
    vx, vy, w = pq.chebyshev_legendre(12, 4)
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs(np.dot(w, vx * vx) - 1.0 / 3.0) < 1e-15
    assert abs(np.dot(w, vy * vy) - 1.0 / 3.0) < 1e-15
    assert abs(np.dot(w, vx)) < 1e-15 and abs(np.dot(w, vx * vy)) < 1e-15
    # N_vz-point Gauss-Legendre in v_z: sum w vz^4 = 1/5 (in-plane: sum w (vx^2+vy^2)^2 = 8/15)
    assert abs(np.dot(w, (vx * vx + vy * vy) ** 2) - 8.0 / 15.0) < 1e-14


def test_product_chebyshev_rule():
    from paper_2402_10488_amd import quadrature as pq
    vx, vy, w = pq.chebyshev_circle(16)
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs(np.dot(w, vx * vx) - 0.5) < 1e-15          # in-plane rule: sum w vx^2 = 1/2
    assert np.all(np.abs(vx) > 1e-3) and np.all(np.abs(vy) > 1e-3)   # no axis-aligned direction
    # N_phi / 4 directions per quadrant
    q = (vx < 0).astype(int) + 2 * (vy < 0).astype(int)
    assert np.bincount(q, minlength=4).tolist() == [4, 4, 4, 4]


def test_memory_budget_accounting():
    from paper_2402_10488_amd.serving import MemoryBudget
    m = MemoryBudget(100)
    assert m.try_reserve(60) and not m.try_reserve(50) and m.try_reserve(40)
    assert m.peak == 100
    m.release(60)
    assert m.used == 40 and m.try_reserve(60) and m.peak == 100
