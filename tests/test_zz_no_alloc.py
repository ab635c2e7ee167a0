"""rte_sweep_noalloc (the sweep on the library's own per-device scratch array) against rte_sweep
with a caller workspace: the same kernels run, so angular flux and densities must be identical
bit for bit.  Two calls in a row, the second on a smaller problem, so the second reads an array
that still holds the first call's larger contents (GPU)."""
import numpy as np
import pytest

import rte_workloads as W
from tests.gpu_common import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2402_10488_amd import rte, problems
    return rte, problems


def _inputs(R, seed, nx, ny, n_phi, B):
    rte, problems = R
    plane = W.random_plane(seed, nx=nx, ny=ny, n_phi=n_phi, B=B, nbx=3, nby=2, Lx=1.0, Ly=0.8)
    P = problems.plane_problem(plane)
    rho = np.random.default_rng(seed + 1).uniform(0.0, 1.0, (B, P.ndof)) / np.sqrt(nx * ny)
    return P, dev(rho)


def _both(R, P, rho, precision):
    import torch
    rte, _ = R
    dt = torch.float64 if precision == "fp64" else torch.float32
    out = []
    for noalloc in (False, True):
        f = torch.full(rte.f_shape(P), float("nan"), dtype=dt, device="cuda")
        rs = torch.full((P.B, P.ndof), float("nan"), dtype=torch.float64, device="cuda")
        if noalloc:
            rte.sweep_noalloc(P, rho, f_out=f, rho_star_out=rs, precision=precision)
        else:
            rte.sweep(P, rho, f_out=f, rho_star_out=rs, precision=precision)
        out.append((host(f), host(rs)))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_sweep_equals_workspace_sweep_twice(R, precision):
    rte, _ = R
    # first call: 3 instances of 130 x 70 cells (three 64-row bands, the last ragged), 24 dirs
    P1, rho1 = _inputs(R, 500, 130, 70, 24, 3)
    assert P1.workspace_bytes("si", None, precision) <= rte.NOALLOC_SCRATCH_BYTES
    say(f"noalloc sweep call 1: 130x70 B=3 24 dirs {precision}")
    (fa, ra), (fb, rb) = _both(R, P1, rho1, precision)
    assert np.all(np.isfinite(fa)) and np.all(np.isfinite(ra))
    assert np.array_equal(fa, fb) and np.array_equal(ra, rb)
    # second call, smaller: 1 instance of 20 x 33 cells, 8 directions
    P2, rho2 = _inputs(R, 501, 20, 33, 8, 1)
    say(f"noalloc sweep call 2: 20x33 B=1 8 dirs {precision}")
    (fa, ra), (fb, rb) = _both(R, P2, rho2, precision)
    assert np.all(np.isfinite(fa)) and np.all(np.isfinite(ra))
    assert np.array_equal(fa, fb) and np.array_equal(ra, rb)
    # densities only (no f) on the small problem after the large one
    import torch
    rs1 = torch.zeros((P2.B, P2.ndof), dtype=torch.float64, device="cuda")
    rs2 = torch.zeros_like(rs1)
    rte.sweep(P2, rho2, rho_star_out=rs1, precision=precision)
    rte.sweep_noalloc(P2, rho2, rho_star_out=rs2, precision=precision)
    assert np.array_equal(host(rs1), host(rs2))


def test_noalloc_sweep_rejects_problems_beyond_its_scratch(R):
    """A batch whose sweep needs more than the scratch array is refused before any device work."""
    import torch
    rte, problems = R
    plane = W.c2_batch(8, 128, 64)
    P = problems.plane_problem(plane)
    assert P.workspace_bytes("si", None, "fp64") > rte.NOALLOC_SCRATCH_BYTES
    rho = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
    rs = torch.zeros_like(rho)
    say("noalloc sweep: oversized batch must be refused")
    with pytest.raises(rte.RteError) as e:
        rte.sweep_noalloc(P, rho, rho_star_out=rs)
    assert e.value.status == rte.RTE_ENOMEM
