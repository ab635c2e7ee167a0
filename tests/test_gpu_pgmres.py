"""DSA-preconditioned restarted GMRES on the GPU vs the oracle's (GPU)."""
import numpy as np
import pytest

import rte_workloads as W
from oracle.pgmres import pgmres
from oracle.problem import discretize
from tests.gpu_common import host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2402_10488_amd import problems, rte
    return rte, problems


def _check(res, rho, discs, tol, m=25, precondition=True, counts_exact=True):
    for b, d in enumerate(discs):
        ref = pgmres(d, tol=tol, m=m, precondition=precondition)
        assert ref.converged and res.inst_status[b] == 0
        if counts_exact:
            assert res.iterations[b] == ref.iterations, (b, res.iterations[b], ref.iterations)
            assert res.n_sweep[b] == ref.n_sweep, (b, res.n_sweep[b], ref.n_sweep)
        else:
            assert abs(int(res.iterations[b]) - ref.iterations) <= 1
        assert rel_err(rho[b], ref.rho) < 50 * tol, (b, rel_err(rho[b], ref.rho))


@pytest.mark.parametrize("case", ["lattice", "cl_homogeneous"])
def test_pgmres_plane_matches_oracle(R, case):
    import torch
    rte, problems = R
    if case == "lattice":
        plane = W.c2_lattice([20000, 20001, 20002], n=12, n_phi=8)
    else:
        plane = W.homogeneous_medium([0.92, 1.08], n=10, quad=("cl", (8, 2)))
    P = problems.plane_problem(plane)
    say(f"pgmres plane {case}")
    rho = torch.zeros((plane.B, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.pgmres_solve(P, rho, tol=1e-10, restart=25, cg_rtol=1e-13)
    _check(res, host(rho), [discretize(plane, b) for b in range(plane.B)], 1e-10)


def test_pgmres_slab_batch_matches_oracle(R):
    import torch
    rte, problems = R
    base = W.random_slab(1, nc=30, n_dir=8)
    batch = []
    for k in range(4):
        s = W.random_slab(70 + k, nc=30, n_dir=8)
        s.edges = base.edges
        batch.append(s)
    P = problems.slab_problem(batch)
    say("pgmres slab batch")
    rho = torch.zeros((len(batch), P.ndof), dtype=torch.float64, device="cuda")
    res = rte.pgmres_solve(P, rho, tol=1e-11, restart=25)
    _check(res, host(rho), [discretize(s) for s in batch], 1e-11)


def test_gmres_restarts_and_no_preconditioner(R):
    import torch
    rte, problems = R
    plane = W.random_plane(12, nx=6, ny=5, n_phi=8, B=2)
    P = problems.plane_problem(plane)
    discs = [discretize(plane, b) for b in range(plane.B)]
    say("pgmres restart 3")
    rho = torch.zeros((plane.B, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.pgmres_solve(P, rho, tol=1e-10, restart=3, cg_rtol=1e-13)
    assert res.cycles > 1
    _check(res, host(rho), discs, 1e-10, m=3, counts_exact=False)
    say("gmres without preconditioner")
    rho.zero_()
    res = rte.pgmres_solve(P, rho, tol=1e-10, restart=60, precondition=False)
    _check(res, host(rho), discs, 1e-10, m=60, precondition=False, counts_exact=False)


def test_pgmres_from_rom_initial_guess(R):
    """PGMRES-ROMIG: the parametric ROM's initial guess shortens the Krylov solve (Sec. 3.1)."""
    import torch
    rte, problems = R
    from paper_2402_10488_amd import offline
    train = W.c2_lattice([41000 + i for i in range(8)], n=12, n_phi=8)
    say("pgmres-romig: rom")
    ra = offline.build_parametric_rom(train, r=8, eps_train=1e-12, cg_rtol=1e-13)
    test = W.c2_lattice([20005, 20006], n=12, n_phi=8)
    P = problems.plane_problem(test)
    Rm = rte.Rom(P, ra.U_rho, ra.U_iso, ra.A0, ra.A, ra.eps_pod, ra.eps_train, ra.b_inflow)
    rho = torch.zeros((test.B, P.ndof), dtype=torch.float64, device="cuda")
    cold = rte.pgmres_solve(P, rho.clone(), tol=1e-10, cg_rtol=1e-13)
    say("pgmres-romig: solve")
    rte.rom_initial_guess(P, Rm, problems.plane_psi(test), rho)
    warm = rte.pgmres_solve(P, rho, tol=1e-10, cg_rtol=1e-13)
    assert np.all(warm.inst_status == 0)
    assert np.all(warm.iterations < cold.iterations)
    for b in range(test.B):
        ref = pgmres(discretize(test, b), tol=1e-10)
        assert rel_err(host(rho)[b], ref.rho) < 1e-8
