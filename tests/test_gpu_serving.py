"""Serving: resumable slot sessions and the continuous-batching loop (GPU).

A request's result must be the same whether it is solved alone or admitted into a batch that
other requests join and leave; with the same slot-pool capacity (hence the same sweep schedule)
the per-slot arithmetic is identical, so the comparison is bitwise.
"""
import numpy as np
import pytest

import rte_workloads as W
from oracle.problem import discretize
from oracle.sisa import sisa
from tests.gpu_common import host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2402_10488_amd import problems, rte, serving
    return rte, problems, serving


def _run_session(S, max_rounds=1000):
    for _ in range(max_rounds):
        if not S.iterate(1).any():
            return
    raise AssertionError("session did not finish")


def test_session_matches_batch_solve(R):
    import torch
    rte, problems, _ = R
    plane = W.c2_lattice([20000 + i for i in range(4)], n=16, n_phi=8, left_inflow=True)
    P = problems.plane_problem(plane)
    say("session vs batch solve (si_dsa fp64)")
    rho = torch.zeros((4, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.sisa_solve(P, rho, mode="si_dsa", eps=1e-8, precision="fp64", cg_rtol=1e-12)
    S = rte.Session(P, "si_dsa", eps=1e-8, precision="fp64", cg_rtol=1e-12)
    S.admit([0, 1, 2, 3])
    _run_session(S)
    assert np.array_equal(S.n_sweep, res.n_sweep)
    assert np.all(S.status == 0)
    assert np.array_equal(host(S.rho), host(rho))


def test_staggered_admission_follows_alg1_per_slot(R):
    import torch
    rte, problems, _ = R
    plane = W.c2_lattice([20010, 20011, 20012], n=16, n_phi=8, left_inflow=True)
    P = problems.plane_problem(plane)
    say("staggered admission (si_dsa fp64)")
    rho = torch.zeros((3, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.sisa_solve(P, rho, mode="si_dsa", eps=1e-8, precision="fp64", cg_rtol=1e-12)
    S = rte.Session(P, "si_dsa", eps=1e-8, precision="fp64", cg_rtol=1e-12)
    S.admit([1])
    S.iterate(3)
    S.admit([2])
    S.iterate(2)
    S.admit([0])
    _run_session(S)
    assert np.array_equal(S.n_sweep, res.n_sweep)
    assert np.array_equal(host(S.rho), host(rho))
    # a finished slot can be refilled: slot 1 solves instance 0's problem again
    P.sigma_t[1] = P.sigma_t[0]
    P.sigma_s[1] = P.sigma_s[0]
    P.G[1] = P.G[0]
    P.inflow[1] = P.inflow[0]
    S.rho[1] = 0.0
    S.admit([1])
    _run_session(S)
    assert S.n_sweep[1] == res.n_sweep[0]
    assert np.array_equal(host(S.rho[1]), host(rho[0]))


def _requests(serving, specs):
    return [serving.lattice_request(i, t, n, nphi, seed) for i, (t, n, nphi, seed) in enumerate(specs)]


def _pools(serving, keys, capacity, mode, precision, roms=None):
    return {k: serving.KeyPool(k[0], k[1], capacity, mode, (roms or {}).get(k),
                               precision=precision, eps=1e-8 if precision == "fp64" else 1e-6,
                               cg_rtol=1e-12, keep_rho=True) for k in keys}


def test_served_alone_equals_mixed_and_oracle(R):
    rte, problems, serving = R
    keys = [(16, 8), (8, 16)]
    specs = [(0.000, 16, 8, 101), (0.001, 8, 16, 102), (0.002, 16, 8, 103), (0.003, 16, 8, 104),
             (0.004, 8, 16, 105), (0.005, 16, 8, 106), (0.006, 8, 16, 107)]
    reqs = _requests(serving, specs)
    say("serving mix (si_dsa fp64, capacity 2)")
    srv = serving.Server(_pools(serving, keys, 2, "si_dsa", "fp64"), budget_bytes=1 << 40)
    mixed = srv.run(reqs)
    assert [r.rid for r in mixed] == list(range(len(reqs)))
    for r in mixed:
        assert r.status == 0
    for q in (reqs[2], reqs[4]):
        say(f"serving alone rid={q.rid}")
        alone = serving.Server(_pools(serving, keys, 2, "si_dsa", "fp64"), 1 << 40).run(
            [serving.Request(0, 0.0, q.n, q.n_phi, q.sigma_t, q.sigma_s, q.G, q.g, q.psi)])[0]
        m = mixed[q.rid]
        assert alone.n_sweep == m.n_sweep
        assert np.array_equal(alone.rho, m.rho)
        # and the served result is the oracle's (FP64 SI-DSA, direct diffusion solve)
        pl = W.c2_lattice([specs[q.rid][3]], n=q.n, n_phi=q.n_phi, left_inflow=True)
        ref = sisa(discretize(pl, 0), "si_dsa", eps=1e-8)
        assert m.n_sweep == ref.n_sweep
        assert rel_err(m.rho, ref.rho) < 1e-10


def test_memory_budget_limits_residency(R):
    rte, problems, serving = R
    keys = [(16, 8)]
    pools = _pools(serving, keys, 4, "si_dsa", "fp64")
    one = pools[keys[0]].slot_bytes
    srv = serving.Server(pools, budget_bytes=one + one // 2)      # room for one request only
    reqs = _requests(serving, [(0.0, 16, 8, 201), (0.0, 16, 8, 202), (0.0, 16, 8, 203)])
    say("serving under a one-request memory budget")
    out = srv.run(reqs)
    assert srv.budget.peak == one
    # with one resident request at a time, each starts after the previous one finished
    order = sorted(out, key=lambda r: r.admitted)
    for a, b in zip(order, order[1:]):
        assert b.admitted >= a.finished - 1e-9
    assert all(r.status == 0 for r in out)


def test_served_romsad_alone_equals_mixed(R):
    rte, problems, serving = R
    from paper_2402_10488_amd import offline
    key = (16, 8)
    train = W.c2_lattice([41000 + i for i in range(6)], n=16, n_phi=8, left_inflow=True)
    say("offline rom for serving key (16, 8)")
    rom = offline.build_correction_rom(train, r=10, window=3, eps_train=1e-10)
    specs = [(0.0, 16, 8, 301), (0.0005, 16, 8, 302), (0.001, 16, 8, 303), (0.0015, 16, 8, 304)]
    reqs = _requests(serving, specs)
    say("serving romsad mix (mixed precision, capacity 3)")
    mixed = serving.Server(_pools(serving, [key], 3, "romsad", "mixed", {key: rom}), 1 << 40).run(reqs)
    q = reqs[3]
    alone = serving.Server(_pools(serving, [key], 3, "romsad", "mixed", {key: rom}), 1 << 40).run(
        [serving.Request(0, 0.0, q.n, q.n_phi, q.sigma_t, q.sigma_s, q.G, q.g, q.psi)])[0]
    assert alone.n_sweep == mixed[3].n_sweep
    assert np.array_equal(alone.rho, mixed[3].rho)
    assert all(r.status == 0 for r in mixed)
