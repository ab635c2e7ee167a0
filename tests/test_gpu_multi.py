"""Several batches solved together on their own streams (rte_sisa_solve_multi): a batch split
into sub-batches gives every instance exactly the result of the whole batch solved at once, when
the sub-batches use the whole batch's sweep schedule (GPU)."""
import numpy as np
import pytest

import rte_workloads as W
from tests.gpu_common import host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2402_10488_amd import offline, problems, rte
    return rte, problems, offline


@pytest.mark.parametrize("mode,precision,parts", [("si_dsa", "fp64", (5, 7)),
                                                  ("romsad", "mixed", (4, 4, 4)),
                                                  ("romsad", "fp64", (12,))])
def test_split_batch_equals_whole_batch(R, mode, precision, parts):
    import torch
    rte, problems, offline = R
    n, nphi = 24, 16
    plane = W.c2_lattice([20000 + i for i in range(sum(parts))], n=n, n_phi=nphi, left_inflow=True)
    arrays = None
    if mode == "romsad":
        say("rom for the split test")
        arrays = offline.build_correction_rom(W.c2_lattice([30000 + i for i in range(6)], n=n,
                                                           n_phi=nphi, left_inflow=True),
                                              r=8, window=3, eps_train=1e-10)

    def setup(pl):
        P = problems.plane_problem(pl, dg=2, wpb=2)
        Rm = (rte.Rom(P, arrays.U_rho, arrays.U_iso, arrays.A0, arrays.A, arrays.eps_pod,
                      arrays.eps_train) if arrays is not None else None)
        psi = problems.plane_psi(pl) if arrays is not None else None
        rho = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
        return P, Rm, psi, rho

    kw = dict(mode=mode, eps=1e-6 if precision == "mixed" else 1e-9, precision=precision,
              cg_rtol=1e-6, theta=5)
    P, Rm, psi, rho = setup(plane)
    say(f"whole batch {mode} {precision}")
    whole = rte.sisa_solve(P, rho, rom=Rm, psi=psi, **kw)
    rho_whole = host(rho)
    subs, lo = [], 0
    for k in parts:
        subs.append(setup(plane.subset(range(lo, lo + k))))
        lo += k
    streams = [torch.cuda.Stream() for _ in parts]
    say(f"{len(parts)} sub-batches {parts} together")
    res = rte.sisa_solve_multi([s[0] for s in subs], [s[3] for s in subs], streams,
                               roms=[s[1] for s in subs], psis=[s[2] for s in subs], **kw)
    torch.cuda.synchronize()
    lo = 0
    for (Ps, _, _, rho_s), r, k in zip(subs, res, parts):
        assert r.status == 0 and np.all(r.inst_status == 0)
        assert np.array_equal(r.n_sweep, whole.n_sweep[lo:lo + k])
        assert np.array_equal(host(rho_s), rho_whole[lo:lo + k])
        if mode == "romsad":
            assert np.array_equal(r.kind, whole.kind[lo:lo + k])
        lo += k
