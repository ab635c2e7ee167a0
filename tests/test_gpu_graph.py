"""The outer iteration of Alg. 1 / Alg. 2 as one HIP graph launch (rte_solve_opts.graph_cg_iters)
against the kernel-by-kernel driver: the same kernels in the same order, so densities, sweep
counts, change histories and correction kinds must be identical bit for bit, whichever launches
the host polls after (GPU)."""
import numpy as np
import pytest

import rte_workloads as W
from oracle import rom as orom
from oracle.problem import discretize
from oracle.sisa import sisa
from tests.gpu_common import host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2402_10488_amd import rte, problems
    return rte, problems


def _run(rte, P, mode, eps, **kw):
    import torch
    rho = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
    ws = kw.pop("ws", None)
    res = rte.sisa_solve(P, rho, mode=mode, eps=eps, ws=ws, **kw)
    return host(rho), res


def _same(a, b):
    (ra, sa), (rb, sb) = a, b
    assert sa.status == sb.status
    assert np.array_equal(sa.n_sweep, sb.n_sweep)
    assert np.array_equal(sa.kind, sb.kind)
    assert np.array_equal(sa.change, sb.change)
    assert np.array_equal(ra, rb)
    assert sa.cg_iterations == sb.cg_iterations


@pytest.fixture(scope="module")
def lattice_rom():
    train = W.c2_lattice([30000 + i for i in range(6)], n=16, n_phi=16)
    discs = [discretize(train, b) for b in range(train.B)]
    return orom.build_correction_rom(discs, orom.plane_affine(discs[0]), orom.plane_psi, window=3,
                                     r=12, eps_train=1e-10)


@pytest.mark.parametrize("mode", ["si", "si_dsa"])
@pytest.mark.parametrize("poll", [1, 3])
def test_graph_equals_eager_plane(R, mode, poll):
    rte, problems = R
    plane = W.random_plane(8, nx=19, ny=14, n_phi=12, B=3, Lx=2.0, Ly=1.5)
    P = problems.plane_problem(plane)
    say(f"graph vs eager plane {mode} poll {poll}")
    kw = dict(max_iter=4000, cg_rtol=1e-13, precision="mixed", poll_every=poll)
    eager = _run(rte, P, mode, 1e-6, **kw)
    graph = _run(rte, P, mode, 1e-6, graph_cg_iters=40, **kw)
    _same(eager, graph)
    # the cached graph on a second call, and the oracle's counts
    _same(eager, _run(rte, P, mode, 1e-6, graph_cg_iters=40, **kw))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_equals_eager_romsad_and_oracle(R, lattice_rom, precision):
    rte, problems = R
    test = W.c2_lattice([20000 + i for i in range(6)], n=16, n_phi=16)
    P = problems.plane_problem(test)
    rom = lattice_rom
    Rm = rte.Rom(P, rom.dU_rho, rom.dU_iso, rom.A0, np.stack(rom.At + rom.As), rom.eps_pod,
                 rom.eps_train)
    psi = problems.plane_psi(test)
    eps = 1e-8 if precision == "fp64" else 1e-6
    say(f"graph vs eager romsad {precision}")
    kw = dict(rom=Rm, psi=psi, theta=5, max_iter=400, cg_rtol=1e-13, precision=precision,
              poll_every=2)
    eager = _run(rte, P, "romsad", eps, **kw)
    graph = _run(rte, P, "romsad", eps, graph_cg_iters=40, **kw)
    _same(eager, graph)
    rho, res = graph
    for b in range(test.B):
        ref = sisa(discretize(test, b), "romsad", eps=eps, rom=rom, theta=5)
        assert res.n_sweep[b] == ref.n_sweep
        assert list(res.kind[b, :res.n_sweep[b] - 1]) == ref.kinds
        assert rel_err(rho[b], ref.rho) < (1e-12 if precision == "fp64" else 1e-5)


def test_graph_equals_eager_slab(R):
    rte, problems = R
    base = W.random_slab(1, nc=40, n_dir=8)
    batch = []
    for k in range(4):
        s = W.random_slab(60 + k, nc=40, n_dir=8)
        s.edges = base.edges
        batch.append(s)
    P = problems.slab_problem(batch)
    say("graph vs eager slab si_dsa")
    kw = dict(max_iter=3000)
    _same(_run(rte, P, "si_dsa", 1e-11, **kw), _run(rte, P, "si_dsa", 1e-11, graph_cg_iters=8, **kw))


def test_graph_is_recaptured_for_new_arguments(R):
    """Every call gets a new density buffer (a new capture whenever its address differs from the
    cached graph's) and a changed poll interval reuses the capture: results stay equal to the
    kernel-by-kernel driver's."""
    rte, problems = R
    plane = W.c2_lattice([20000 + i for i in range(3)], n=24, n_phi=16)
    P = problems.plane_problem(plane)
    say("graph recapture on new arguments")
    ws = P.workspace("si_dsa", None, "mixed", 200)
    kw = dict(max_iter=200, cg_rtol=1e-6, precision="mixed", ws=ws)
    eager = _run(rte, P, "si_dsa", 1e-6, **kw)
    for _ in range(3):
        _same(eager, _run(rte, P, "si_dsa", 1e-6, graph_cg_iters=20, **kw))
    _same(eager, _run(rte, P, "si_dsa", 1e-6, graph_cg_iters=20, poll_every=5, **kw))


def test_graph_depth_below_need_reports_cg_failure(R):
    """With a one-iteration CG in the graph and a tight CG tolerance the diffusion solves cannot
    converge: the solve returns RTE_ECG (after filling its statistics)."""
    rte, problems = R
    plane = W.c2_lattice([20000, 20001], n=24, n_phi=16)
    P = problems.plane_problem(plane)
    say("graph depth 1: CG failure reported")
    rho, res = _run(rte, P, "si_dsa", 1e-8, max_iter=300, cg_rtol=1e-12, graph_cg_iters=1,
                    raise_on_error=False)
    assert res.status == rte.RTE_ECG
    assert np.all(res.n_sweep > 0)


def test_graph_session_equals_eager_session(R):
    """rte_sisa_iterate in graph mode: slots admitted at different times, one iteration per call,
    equal bit for bit to the kernel-by-kernel session."""
    import torch
    rte, problems = R
    plane = W.c2_lattice([20000 + i for i in range(4)], n=16, n_phi=16)
    out = []
    for depth in (0, 30):
        P = problems.plane_problem(plane)
        say(f"session graph depth {depth}")
        S = rte.Session(P, mode="si_dsa", eps=1e-6, max_iter=200, cg_rtol=1e-8,
                        precision="mixed", graph_cg_iters=depth)
        S.admit([0, 1])
        S.iterate(3)
        S.admit([2, 3])
        for _ in range(200):
            if not S.iterate(1).any():
                break
        out.append((host(S.rho), S.n_sweep.copy()))
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][0], out[1][0])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_preconditioner_graphs_kept_across_calls(R, precision):
    """The multigrid preconditioner's graphs are captured once per (handle, workspace carve-up)
    and replayed by later calls.  Repeated solves on one workspace, a solve on a second one (a
    new capture) and a return to the first (another) give bitwise-equal results, and so does a
    fresh handle."""
    rte, problems = R
    plane = W.c2_lattice([20000 + i for i in range(3)], n=48, n_phi=16, left_inflow=True)
    P = problems.plane_problem(plane)
    kw = dict(precision=precision, cg_rtol=1e-6, max_iter=300)
    ws1 = P.workspace("si_dsa", None, precision, 300)
    ws2 = P.workspace("si_dsa", None, precision, 300)
    ref = _run(rte, problems.plane_problem(plane), "si_dsa", 1e-8, **kw)
    for k, ws in enumerate([ws1, ws1, ws2, ws1, ws1]):
        say(f"preconditioner graphs {precision}: call {k}")
        _same(_run(rte, P, "si_dsa", 1e-8, ws=ws, **kw), ref)
