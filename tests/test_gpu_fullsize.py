"""The configurations at full size, in the launch configuration the benchmark times (GPU).

The oracle computes sampled instances one by one where it can; otherwise properties that hold at
any size are checked (convergence to the same discrete solution by different methods, the point
symmetry of a symmetric medium)."""
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
    from paper_2402_10488_amd import offline, problems, rte
    return rte, problems, offline


@pytest.fixture(scope="module")
def c2(R):
    """The 256 x 128^2 x 64 batch solved by SI-DSA in mixed precision at 1e-6."""
    import torch
    rte, problems, _ = R
    plane = W.c2_batch(256, 128, 64)
    P = problems.plane_problem(plane)
    say(f"c2 full batch si_dsa mixed, tuning {P.tuning()}")
    rho = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.sisa_solve(P, rho, mode="si_dsa", eps=1e-6, precision="mixed", cg_rtol=1e-10)
    return plane, P, host(rho), res


def test_c2_full_batch_sampled_against_oracle(c2):
    plane, P, rho, res = c2
    assert res.status == 0
    for b in (0, 137, 255):
        say(f"  oracle instance {b}")
        ref = sisa(discretize(plane, b), "si_dsa", eps=1e-6)
        assert res.n_sweep[b] == ref.n_sweep, (b, res.n_sweep[b], ref.n_sweep)
        assert rel_err(rho[b], ref.rho) < 1e-5


def test_c2_full_batch_romsad_reaches_the_same_solutions(R, c2):
    """ROMSAD with a GPU-built rank-20 ROM (32 training solves, window 3) converges, instance by
    instance, to the SI-DSA solution within the stop tolerance."""
    import torch
    rte, problems, offline = R
    plane, P, rho_dsa, res_dsa = c2
    say("c2 rom build (32 training solves)")
    ra = offline.build_correction_rom(W.c2_training(32, 128, 64), r=20, window=3, eps_train=1e-10)
    Rm = rte.Rom(P, ra.U_rho, ra.U_iso, ra.A0, ra.A, ra.eps_pod, ra.eps_train)
    say("c2 full batch romsad mixed")
    rho = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.sisa_solve(P, rho, mode="romsad", rom=Rm, psi=problems.plane_psi(plane), eps=1e-6,
                         theta=5, precision="mixed", cg_rtol=1e-10)
    assert res.status == 0
    rho = host(rho)
    err = np.abs(rho - rho_dsa).max(axis=1) / np.abs(rho_dsa).max(axis=1)
    assert err.max() < 2e-5, err.max()
    # every instance took ROMSA at least once (kind 2), so the switch of Alg. 2 ran
    assert np.all((res.kind == 2).any(axis=1))


def test_c4_full_size_point_symmetry(R):
    """512^2 cells, 256 directions, the multiscale checkerboard: the medium, the source and the
    direction set are symmetric under (x, y) -> (1 - x, 1 - y), so is the converged density
    (cell means equal, first moments opposite)."""
    import torch
    rte, problems, _ = R
    plane = W.c4_multiscale()
    P = problems.plane_problem(plane)
    say(f"c4 full size si_dsa mixed, tuning {P.tuning()}")
    rho = torch.zeros((1, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.sisa_solve(P, rho, mode="si_dsa", eps=1e-6, precision="mixed", cg_rtol=1e-10,
                         max_iter=500)
    assert res.status == 0
    r = host(rho)[0].reshape(512, 512, 4)
    flip = r[::-1, ::-1]
    scale = np.abs(r[..., 0]).max()
    assert np.abs(r[..., 0] - flip[..., 0]).max() < 1e-5 * scale
    assert np.abs(r[..., 1] + flip[..., 1]).max() < 1e-5 * scale
    assert np.abs(r[..., 2] + flip[..., 2]).max() < 1e-5 * scale
