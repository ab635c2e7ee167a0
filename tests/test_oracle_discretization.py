"""Pins of the oracle's quadrature, DG operators and sweeps against facts the
paper and the mathematics fix (no GPU)."""
import numpy as np
import pytest

import rte_workloads as W
from oracle import dg, quadrature
from oracle.brute import BruteForce
from oracle.problem import discretize
from oracle.sisa import sisa, residual


# --------------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", [2, 8, 16])
def test_gauss_legendre_normalized_exactness(n):
    mu, w = quadrature.gauss_legendre(n)
    assert abs(w.sum() - 1.0) < 1e-15
    for k in range(2 * n):   # (1/2) int_{-1}^{1} x^k dx
        exact = 0.0 if k % 2 else 1.0 / (k + 1)
        assert abs(np.sum(w * mu ** k) - exact) < 1e-14


@pytest.mark.parametrize("n", [8, 12, 64])
def test_chebyshev_circle(n):
    vx, vy, w = quadrature.chebyshev_circle(n)
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs(np.sum(w * vx ** 2) - 0.5) < 1e-14 and abs(np.sum(w * vy ** 2) - 0.5) < 1e-14
    assert abs(np.sum(w * vx)) < 1e-15 and abs(np.sum(w * vx * vy)) < 1e-15
    # closed under v -> -v: phi_j + pi = phi_{j + n/2}
    assert np.allclose(vx[: n // 2], -vx[n // 2:], atol=1e-15)
    if n % 4 == 0:
        assert np.min(np.abs(vx)) > 0.0 and np.min(np.abs(vy)) > 0.0
        assert np.sum((vx > 0) & (vy > 0)) == n // 4
    # sum_{v.n>0} w v.n -> 1/pi for the circle
    assert abs(np.sum(w[vx > 0] * vx[vx > 0]) - 1.0 / np.pi) < 2.0 / n ** 2


def test_cl_rule_integrates_sphere_moments():
    vx, vy, vz, w = quadrature.chebyshev_legendre(30, 6)
    assert abs(w.sum() - 1.0) < 1e-14
    for v in (vx, vy, vz):
        assert abs(np.sum(w * v ** 2) - 1.0 / 3.0) < 1e-13


# ----------------------------------------------------------------- DG operators
def test_plane_operators_reproduce_constants():
    """A constant f is in the DG space: the inflow from a constant neighbour cancels
    the volume and outflow terms (divergence theorem), so (V + E) 1 = 0."""
    hx, hy = 0.3, 0.2
    vx, vy, w = quadrature.chebyshev_circle(12)
    V, Ex, Ey, bx, by = dg.plane_operators(hx, hy, vx, vy)
    one = np.array([np.sqrt(hx * hy), 0, 0, 0])
    for j in range(12):
        assert np.abs((V[j] + Ex[j] + Ey[j]) @ one).max() < 1e-13
        # a unit inflow load equals the coupling to a unit-constant neighbour
        assert np.abs(-Ex[j] @ one - bx[j]).max() < 1e-13
        assert np.abs(-Ey[j] @ one - by[j]).max() < 1e-13


def test_plane_operator_closed_form():
    """For v_x, v_y > 0 the x-part of V is (v_x/h_x) [[1, s3],[-s3, 3]] in the x-index
    (Legendre traces P(+1) = (1, s3), P(-1) = (1, -s3)), tensored with the identity."""
    s3 = np.sqrt(3.0)
    A = np.array([[1, s3], [-s3, 3]])
    hx, hy = 0.25, 0.5
    V, Ex, Ey, _, _ = dg.plane_operators(hx, hy, np.array([0.6]), np.array([0.8]))
    I = np.eye(2)
    expect = 0.6 / hx * np.kron(I, A) + 0.8 / hy * np.kron(A, I)   # k = a + 2b
    assert np.abs(V[0] - expect).max() < 1e-13
    Pm, Pp = np.array([1, -s3]), np.array([1, s3])
    ex = -0.6 / hx * np.kron(I, np.outer(Pm, Pp))
    assert np.abs(Ex[0] - ex).max() < 1e-13


# ------------------------------------------------------------------------ sweeps
def test_infinite_medium_plane():
    """f = G / sigma_a with matching inflow is reproduced exactly; one sweep from
    the exact guess returns it (n_sweep = 1)."""
    sa, G = 0.5, 0.8
    p = W.plane_uniform(7, 2.0, 1.5, G, g=G / sa, n_phi=12)
    d = discretize(p)
    rho0 = np.tile([G / sa * np.sqrt(d.hx * d.hy), 0, 0, 0], d.nc)
    r, _ = d.sweep(rho0)
    assert np.abs(r - rho0).max() < 1e-14 * np.abs(rho0).max()
    res = sisa(d, "si", eps=1e-12, rho0=rho0)
    assert res.n_sweep == 1


def test_infinite_medium_slab():
    s = W.slab_uniform(9, 1.3, 2.0, 1.5, 0.8, g_left=1.6, g_right=1.6, n_dir=8)
    d = discretize(s)
    rho0 = np.concatenate([[1.6 * np.sqrt(h), 0] for h in np.diff(s.edges)])
    r, _ = d.sweep(rho0)
    assert np.abs(r - rho0).max() < 1e-14 * np.abs(rho0).max()


def _absorber_errors(nc):
    sig, G, gl, gr, L = 1.7, 0.6, 1.0, 0.3, 2.0
    s = W.slab_uniform(nc, L, sig, 0.0, G, g_left=gl, g_right=gr, n_dir=8)
    d = discretize(s)
    res = sisa(d, "si", eps=1e-14, want_f=True)
    assert res.n_sweep == 2          # L = 0: the second sweep reproduces the first
    mu, w = d.mu, d.w

    def f_exact(x, m):
        if m > 0:
            e = np.exp(-sig * x / m)
            return gl * e + G / sig * (1 - e)
        e = np.exp(-sig * (L - x) / abs(m))
        return gr * e + G / sig * (1 - e)

    xs = np.linspace(0, L, 4001)[1:-1]
    rho_ex = sum(w[j] * f_exact(xs, mu[j]) for j in range(len(mu)))
    rho_h = dg.slab_eval(s.edges, res.rho.reshape(-1, 2), xs)
    l2 = np.sqrt(np.mean((rho_h - rho_ex) ** 2) * L)
    # outflow trace of the most grazing positive direction at x = L
    jpos = int(np.argmin(np.where(mu > 0, mu, np.inf)))
    f = res.f.reshape(d.nv, nc, 2)
    out = np.array([1.0, np.sqrt(3.0)]) @ f[jpos, -1] / np.sqrt(L / nc)
    return l2, abs(out - f_exact(L, mu[jpos]))


def test_pure_absorber_convergence_orders():
    """sigma_s = 0: exact exponential attenuation per direction.  rho converges at
    O(h^2) in L2; the outflow trace superconverges at O(h^3) (upwind DG, K=1)."""
    e1 = _absorber_errors(16)
    e2 = _absorber_errors(32)
    e3 = _absorber_errors(64)
    r_l2 = np.log2(e2[0] / e3[0])
    r_out = np.log2(e2[1] / e3[1])
    assert r_l2 > 1.8, (e1, e2, e3)
    assert r_out > 2.7, (e1, e2, e3)


def _manufactured_error(n):
    """f(x,v) = (1 + vx/2 + vy/3) sin(pi x) sin(pi y), zero inflow, direction-dependent source."""
    sig_t, sig_s = 2.0, 1.2
    p = W.plane_uniform(n, sig_t, sig_s, 0.0, n_phi=8)
    d = discretize(p)
    pi = np.pi
    q = np.stack([dg.plane_project(n, n, d.hx, d.hy,
                  lambda x, y, a=vx, b=vy: (1 + a / 2 + b / 3) * (
                      a * pi * np.cos(pi * x) * np.sin(pi * y) + b * pi * np.sin(pi * x) * np.cos(pi * y)
                      + sig_t * np.sin(pi * x) * np.sin(pi * y)) - sig_s * np.sin(pi * x) * np.sin(pi * y))
                  for vx, vy in zip(d.vx, d.vy)])
    rho = np.zeros(d.ndof)
    for _ in range(200):
        rs, _ = d.sweep(rho, q=q)
        if np.abs(rs - rho).max() < 1e-13:
            break
        rho = rs
    ex = dg.plane_project(n, n, d.hx, d.hy, lambda x, y: np.sin(pi * x) * np.sin(pi * y)).reshape(-1)
    return np.linalg.norm(rs - ex)


def test_manufactured_solution_order_plane():
    e = [_manufactured_error(n) for n in (8, 16, 32)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(rates > 1.8), e


def test_cell_balance_per_sweep():
    """Row (0,0) of every local system is the cell particle balance:
    outflow - inflow + sigma_t * cell integral = source integral."""
    p = W.random_plane(5, nx=6, ny=5, n_phi=8)
    d = discretize(p)
    rho = np.random.default_rng(1).uniform(0, 1, d.ndof)
    _, f = d.sweep(rho, want_f=True)
    f = f.reshape(d.nv, d.nc, 4)
    src = (d.apply_Ss(rho) + d.G)
    s3 = np.sqrt(3.0)
    for j in range(d.nv):
        F = f[j].reshape(d.ny, d.nx, 4)
        # edge-integrated traces: int over a vertical edge of f = hy * (f00 +/- s3 f10)/sqrt(hx hy)
        scale = 1.0 / np.sqrt(d.hx * d.hy)
        right = d.hy * scale * (F[..., 0] + s3 * F[..., 1])
        left = d.hy * scale * (F[..., 0] - s3 * F[..., 1])
        top = d.hx * scale * (F[..., 0] + s3 * F[..., 2])
        bot = d.hx * scale * (F[..., 0] - s3 * F[..., 2])
        vx, vy = d.vx[j], d.vy[j]
        g = d.g
        # upwind edge values
        if vx > 0:
            inx = np.concatenate([np.full((d.ny, 1), g[0] * d.hy), right[:, :-1]], axis=1)
            outx = right
        else:
            inx = np.concatenate([left[:, 1:], np.full((d.ny, 1), g[1] * d.hy)], axis=1)
            outx = left
        if vy > 0:
            iny = np.concatenate([np.full((1, d.nx), g[2] * d.hx), top[:-1, :]], axis=0)
            outy = top
        else:
            iny = np.concatenate([bot[1:, :], np.full((1, d.nx), g[3] * d.hx)], axis=0)
            outy = bot
        mass = F[..., 0] / scale       # int f over the cell
        bal = abs(vx) * (outx - inx) + abs(vy) * (outy - iny) + d.sigma_t.reshape(d.ny, d.nx) * mass
        rhs = src.reshape(d.ny, d.nx, 4)[..., 0] / scale
        assert np.abs(bal - rhs).max() < 1e-13 * max(1.0, np.abs(rhs).max())


@pytest.mark.parametrize("mode", ["si", "si_dsa"])
def test_si_matches_dense_solve_plane(mode):
    p = W.random_plane(1, nx=5, ny=4, n_phi=8)
    d = discretize(p)
    _, rho = BruteForce(d).solve()
    r = sisa(d, mode, eps=1e-14)
    assert r.converged
    assert np.abs(r.rho - rho).max() <= 1e-12 * np.abs(rho).max()


@pytest.mark.parametrize("mode", ["si", "si_dsa"])
def test_si_matches_dense_solve_slab(mode):
    s = W.random_slab(2, nc=8, n_dir=4)
    d = discretize(s)
    _, rho = BruteForce(d).solve()
    r = sisa(d, mode, eps=1e-14)
    assert np.abs(r.rho - rho).max() <= 1e-12 * np.abs(rho).max()


def test_ideal_correction_converges_in_two_sweeps():
    """Exactly solving the kinetic correction equation gives convergence in two sweeps (Sec. 2.3)."""
    for disc in (discretize(W.random_plane(2, nx=4, ny=4, n_phi=8)), discretize(W.random_slab(4))):
        bf = BruteForce(disc)
        r = sisa(disc, "exact", eps=1e-12, exact=bf)
        assert r.n_sweep == 2


def test_residual_after_convergence():
    d = discretize(W.c0_slab())
    r = sisa(d, "si_dsa", eps=1e-10)
    assert r.converged and r.n_sweep < 20
    assert residual(d, r.rho) < 1e-9 * np.abs(r.rho).max()


def test_point_symmetry_of_checkerboard():
    """The checkerboard medium and its central source are invariant under
    (x,y) -> (1-x,1-y) and the direction set is closed under v -> -v, so the cell
    means satisfy rho(x,y) = rho(1-x,1-y)."""
    p = W.c1_checkerboard(n=32, n_phi=16)
    d = discretize(p)
    r = sisa(d, "si_dsa", eps=1e-12)
    m = r.rho.reshape(32, 32, 4)[..., 0]
    assert np.abs(m - m[::-1, ::-1]).max() < 1e-11 * np.abs(m).max()

