"""Bands in flight (rte_problem_create_sched): a 2D sweep workgroup running several mesh bands at
once does the same cells, solves and sums in the same order as one running them one after
another, so sweeps and solves are bitwise equal for every number of bands (GPU).  The schedule of
one band in flight is compared with the oracle elsewhere."""
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
    from paper_2402_10488_amd import problems, rte
    return rte, problems


# (nx, ny, directions, batch, dg, wpb): a full two-band mesh, ragged band counts (130 and 300
# rows), a mesh narrower than a band (nx < 64, so a band's pipeline is padded to 64 columns),
# one wide instance with 8 bands
CASES = [(128, 128, 64, 3, 4, 4), (200, 130, 16, 2, 2, 2), (40, 256, 8, 2, 1, 4),
         (512, 300, 16, 1, 1, 4), (96, 520, 24, 1, 2, 1)]


@pytest.mark.parametrize("nx,ny,nphi,B,dg,wpb", CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sweep_bitwise_for_every_band_count(R, nx, ny, nphi, B, dg, wpb, precision):
    import torch
    rte, problems = R
    plane = W.random_plane(70 + nx, nx=nx, ny=ny, n_phi=nphi, B=B, nbx=5, nby=3)
    rng = np.random.default_rng(nx + ny)
    out = {}
    for bands in (1, 2, 4):
        P = problems.plane_problem(plane, dg=dg, wpb=wpb, bands=bands)
        rho = torch.as_tensor(rng.uniform(0, 1, (B, P.ndof)) if bands == 1 else out[1][2],
                              device="cuda")
        fdt = torch.float32 if precision == "mixed" else torch.float64
        f = torch.zeros(rte.f_shape(P), dtype=fdt, device="cuda")
        rs = torch.zeros((B, P.ndof), dtype=torch.float64, device="cuda")
        rs2 = torch.zeros_like(rs)
        say(f"{nx}x{ny} {nphi} dirs B={B} ({dg},{wpb}) bands {bands} {precision}")
        rte.sweep(P, rho, rho_star_out=rs, precision=precision)          # rho-form
        rte.sweep(P, rho, f_out=f, rho_star_out=rs2, precision=precision)  # with f
        f_only = torch.zeros_like(f)
        rte.sweep(P, rho, f_out=f_only, precision=precision)             # f, no partial sums
        out[bands] = (host(rs), host(f), host(rho), host(rs2), host(f_only))
    for bands in (2, 4):
        assert np.array_equal(out[bands][0], out[1][0])
        assert np.array_equal(out[bands][1], out[1][1])
        assert np.array_equal(out[bands][3], out[1][3])
        assert np.array_equal(out[bands][4], out[1][1])


@pytest.mark.parametrize("mode,precision", [("si_dsa", "fp64"), ("romsad", "mixed")])
def test_solve_bitwise_for_every_band_count(R, mode, precision):
    import torch
    rte, problems = R
    from paper_2402_10488_amd import offline
    n, nphi = 136, 16
    plane = W.c2_lattice([20000 + i for i in range(3)], n=n, n_phi=nphi, left_inflow=True)
    arrays = None
    if mode == "romsad":
        say("rom for the bands solve test")
        arrays = offline.build_correction_rom(W.c2_lattice([30000 + i for i in range(4)], n=n,
                                                           n_phi=nphi, left_inflow=True),
                                              r=6, window=3, eps_train=1e-10)
    res = {}
    for bands in (1, 2, 4):
        P = problems.plane_problem(plane, dg=2, wpb=2, bands=bands)
        Rm = (rte.Rom(P, arrays.U_rho, arrays.U_iso, arrays.A0, arrays.A, arrays.eps_pod,
                      arrays.eps_train) if arrays is not None else None)
        psi = problems.plane_psi(plane) if arrays is not None else None
        rho = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
        say(f"solve {mode} {precision} bands {bands} (schedule {P.tuning()})")
        r = rte.sisa_solve(P, rho, mode=mode, rom=Rm, psi=psi, eps=1e-6 if precision == "mixed"
                           else 1e-9, precision=precision, cg_rtol=1e-6)
        res[bands] = (r, host(rho))
    for bands in (2, 4):
        assert np.array_equal(res[bands][0].n_sweep, res[1][0].n_sweep)
        assert np.array_equal(res[bands][0].kind, res[1][0].kind)
        assert np.array_equal(res[bands][1], res[1][1])


def test_automatic_band_count(R):
    """The automatic schedule runs one band for a batch that fills the chip, two below 4096
    wavefronts of work and four (of two-wavefront workgroups) below 1024."""
    rte, problems = R
    for B, nphi, want in ((256, 64, (4, 4, 1)), (32, 64, (1, 4, 2)), (1, 64, (1, 2, 4))):
        plane = W.random_plane(5 + B, nx=128, ny=128, n_phi=nphi, B=B, nbx=4, nby=4)
        P = problems.plane_problem(plane)
        t = P.tuning()
        say(f"automatic schedule B={B}: {t}")
        assert (t["dg"], t["wpb"], t["bands"]) == want
