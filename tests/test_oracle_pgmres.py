"""Pins of the oracle's DSA-preconditioned restarted GMRES (no GPU)."""
import numpy as np
import pytest

import rte_workloads as W
from oracle.brute import BruteForce
from oracle.pgmres import pgmres
from oracle.problem import discretize
from oracle.sisa import sisa


@pytest.mark.parametrize("geom", ["plane", "slab"])
def test_pgmres_reaches_the_dense_solution(geom):
    """(I + C Sigma_s)(I - L) rho = (I + C Sigma_s) b_bar has the discrete solution as its root."""
    if geom == "plane":
        d = discretize(W.random_plane(3, nx=5, ny=4, n_phi=8))
    else:
        d = discretize(W.random_slab(5, nc=8, n_dir=4))
    _, rho = BruteForce(d).solve()
    r = pgmres(d, tol=1e-14, m=25)
    assert r.converged
    assert np.abs(r.rho - rho).max() <= 1e-11 * np.abs(rho).max()


def test_unpreconditioned_gmres_terminates_within_the_dimension():
    """Without preconditioning GMRES on (I - L) finds the solution in at most N_DOF steps (one
    cycle long enough), and its residual estimates never increase."""
    d = discretize(W.random_plane(4, nx=3, ny=3, n_phi=8))       # N_DOF = 36
    _, rho = BruteForce(d).solve()
    r = pgmres(d, tol=1e-13, m=d.ndof + 1, precondition=False)
    assert r.converged
    assert r.iterations <= d.ndof
    assert np.all(np.diff(r.residuals) <= 1e-15)
    assert np.abs(r.rho - rho).max() <= 1e-10 * np.abs(rho).max()


def test_sweep_accounting_and_dsa_acceleration():
    """Thick scattering: DSA preconditioning cuts the GMRES steps, PGMRES needs no more sweeps than
    SI-DSA, and a solve converging in its first cycle costs steps + 3 sweeps (right-hand side,
    initial residual, final check)."""
    p = W.plane_uniform(10, sigma_t=10.0, sigma_s=9.9, G=1.0, n_phi=8, L=1.0)
    d = discretize(p)
    plain = pgmres(d, tol=1e-10, m=60, precondition=False)
    pre = pgmres(d, tol=1e-10, m=25)
    assert pre.converged and plain.converged
    assert pre.iterations < plain.iterations
    assert pre.n_sweep == pre.iterations + 3
    si = sisa(d, "si_dsa", eps=1e-10)
    assert pre.n_sweep <= si.n_sweep


def test_restart_still_converges():
    """A short restart length reaches the same solution through several cycles."""
    d = discretize(W.random_plane(6, nx=4, ny=4, n_phi=8))
    _, rho = BruteForce(d).solve()
    r = pgmres(d, tol=1e-12, m=3)
    assert r.converged
    assert np.abs(r.rho - rho).max() <= 1e-10 * np.abs(rho).max()
