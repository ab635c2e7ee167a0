"""Parity of every library entry point with the CPU oracle on the same seeded inputs (GPU)."""
import numpy as np
import pytest

import rte_workloads as W
from oracle import dsa as odsa, rom as orom
from oracle.problem import discretize
from tests.gpu_common import dev, f_library, f_natural, host, rel_err, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-6
# The FP32 angular flux element by element, relative to its largest value: FP32 rounding gathers
# along upwind paths of up to 200 cells here; measured at most 2.42e-6 (5 x 200 cells), asserted
# at twice that.  Densities stay within TOL32 (measured at most 1.4e-6).
TOL32_F = 5e-6


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2402_10488_amd import rte, problems
    return rte, problems


def _rand_rho(d, seed):
    return np.random.default_rng(seed).uniform(0.0, 1.0, d.ndof) * np.sqrt(d.hx * d.hy)


SWEEP_CASES = [
    # (nx, ny, n_phi, B, dg, wpb)
    (13, 9, 8, 3, 0, 0),
    (70, 130, 12, 2, 1, 1),       # 3 bands, ragged last band, nx > 64, 3 directions / quadrant
    (70, 130, 12, 2, 2, 4),
    (70, 130, 12, 2, 4, 2),
    (33, 65, 64, 1, 8, 4),        # 8 directions per lane, nx < 64 (pipeline stride 64)
    (64, 64, 32, 2, 8, 4),
    (1, 1, 4, 1, 0, 0),           # single cell
    (5, 200, 8, 1, 2, 3),         # nx < 64: padded pipeline stride
]


@pytest.mark.parametrize("nx,ny,nphi,B,dg,wpb", SWEEP_CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sweep2d_matches_oracle(R, nx, ny, nphi, B, dg, wpb, precision):
    import torch
    rte, problems = R
    plane = W.random_plane(100 + nx + ny, nx=nx, ny=ny, n_phi=nphi, B=B, nbx=3, nby=2,
                           Lx=1.3, Ly=0.7)
    say(f"sweep2d {nx}x{ny} nphi={nphi} B={B} dg={dg} wpb={wpb} {precision}")
    P = problems.plane_problem(plane, dg=dg, wpb=wpb)
    discs = [discretize(plane, b) for b in range(B)]
    rho_in = np.stack([_rand_rho(d, 7 + b) for b, d in enumerate(discs)])
    f_dtype = torch.float64 if precision == "fp64" else torch.float32
    fd = torch.zeros(rte.f_shape(P), dtype=f_dtype, device="cuda")
    rs = torch.zeros((B, P.ndof), dtype=torch.float64, device="cuda")
    rte.sweep(P, dev(rho_in), f_out=fd, rho_star_out=rs, precision=precision)
    tol = TOL64 if precision == "fp64" else TOL32
    tol_f = TOL64 if precision == "fp64" else TOL32_F
    rs, f = host(rs), host(fd)
    f_or_all = []
    for b, d in enumerate(discs):
        r_or, f_or = d.sweep(rho_in[b], want_f=True)
        f_or_all.append(f_or)
        assert rel_err(rs[b], r_or) < tol, (b, rel_err(rs[b], r_or))
        fb = f_natural(f[b], P)
        assert rel_err(fb, f_or) < tol_f, (b, rel_err(fb, f_or))
    # the library's own conversion to natural order moves values exactly
    fn = host(rte.f_natural(P, fd, precision))
    assert np.array_equal(fn, np.stack([f_natural(f[b], P) for b in range(B)]))
    # f alone (no partial densities formed): the same values
    fd2 = torch.zeros_like(fd)
    rte.sweep(P, dev(rho_in), f_out=fd2, precision=precision)
    assert np.array_equal(host(fd2), f)
    # quadrature reduction of the oracle's angular flux in the library layout
    if precision == "fp64":
        out = torch.zeros((B, P.ndof), dtype=torch.float64, device="cuda")
        rte.scalar_flux(P, dev(np.stack([f_library(f_or_all[b], P) for b in range(B)])), out)
        ref = np.stack([d.w @ f_or_all[b] for b, d in enumerate(discs)])
        assert rel_err(host(out), ref) < 1e-14
    # zero inflow variant (boundary condition of the kinetic correction equation)
    rte.sweep(P, dev(rho_in), rho_star_out=(rs2 := torch.zeros_like(torch.as_tensor(rs, device="cuda"))),
              zero_inflow=True, precision=precision)
    rs2 = host(rs2)
    for b, d in enumerate(discs):
        r_or, _ = d.sweep(rho_in[b], zero_bc=True)
        assert rel_err(rs2[b], r_or) < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sweep1d_and_scalar_flux(R, precision):
    import torch
    rte, problems = R
    slabs = [W.random_slab(s, nc=37, n_dir=16) for s in (1, 1, 1)]
    # same mesh for the batch: vary only the materials
    base = slabs[0]
    batch = []
    for k in range(3):
        s = W.random_slab(10 + k, nc=37, n_dir=16)
        s.edges = base.edges
        batch.append(s)
    say(f"sweep1d {precision}")
    P = problems.slab_problem(batch)
    discs = [discretize(s) for s in batch]
    rho_in = np.stack([np.random.default_rng(b).uniform(0, 1, d.ndof) for b, d in enumerate(discs)])
    f_dtype = torch.float64 if precision == "fp64" else torch.float32
    f = torch.zeros(rte.f_shape(P), dtype=f_dtype, device="cuda")
    rs = torch.zeros((3, P.ndof), dtype=torch.float64, device="cuda")
    rte.sweep(P, dev(rho_in), f_out=f, rho_star_out=rs, precision=precision)
    tol = TOL64 if precision == "fp64" else TOL32
    rs_h, f_h = host(rs), host(f)
    for b, d in enumerate(discs):
        r_or, f_or = d.sweep(rho_in[b], want_f=True)
        assert rel_err(rs_h[b], r_or) < tol
        assert rel_err(f_natural(f_h[b], P), f_or) < tol
    # scalar flux of the oracle's angular flux
    f_or = np.stack([d.sweep(rho_in[b], want_f=True)[1] for b, d in enumerate(discs)])
    out = torch.zeros((3, P.ndof), dtype=torch.float64, device="cuda")
    say("scalar_flux fp64")
    f_lib = np.stack([f_library(f_or[b], P) for b in range(3)])
    rte.scalar_flux(P, dev(f_lib), out)
    ref = np.stack([d.w @ f_or[b] for b, d in enumerate(discs)])
    assert rel_err(host(out), ref) < 1e-14


def test_dsa1d_matches_appendix_b(R):
    import torch
    rte, problems = R
    batch = []
    base = W.random_slab(3, nc=29, n_dir=8)
    for k in range(4):
        s = W.random_slab(20 + k, nc=29, n_dir=8)
        s.edges = base.edges
        batch.append(s)
    say("dsa1d")
    P = problems.slab_problem(batch)
    discs = [discretize(s) for s in batch]
    rng = np.random.default_rng(5)
    rs = rng.uniform(0, 1, (4, P.ndof))
    rp = rng.uniform(0, 1, (4, P.ndof))
    delta = torch.zeros((4, P.ndof), dtype=torch.float64, device="cuda")
    rte.dsa_correct(P, dev(rs), dev(rp), delta)
    delta = host(delta)
    for b, d in enumerate(discs):
        ref = odsa.ConsistentDSA1D(d).correct(d.apply_Ss(rs[b] - rp[b]))
        assert rel_err(delta[b], ref) < 1e-12


# 11x7, 16x16, 64x48, 32x32, 47x47 and 100x16 run the operator on 16x16 tiles (the tile count
# equals the CG's block count; 47x47 and 100x16 have ragged tiles), 40x33 one cell per thread
@pytest.mark.parametrize("nx,ny,L,mg", [(11, 7, 1.0, True), (40, 33, 10.0, True),
                                        (16, 16, 0.05, True), (64, 48, 3.0, True),
                                        (32, 32, 30.0, True), (40, 33, 10.0, False),
                                        (16, 16, 0.05, False), (47, 47, 2.0, True),
                                        (100, 16, 5.0, True)])
def test_dsa2d_matches_mip_direct_solve(R, nx, ny, L, mg):
    import torch
    rte, problems = R
    plane = W.random_plane(40 + nx, nx=nx, ny=ny, n_phi=8, B=3, Lx=L, Ly=0.8 * L)
    say(f"dsa2d {nx}x{ny} L={L} multigrid={mg}")
    P = problems.plane_problem(plane)
    P.dsa_multigrid(mg)
    discs = [discretize(plane, b) for b in range(3)]
    rng = np.random.default_rng(9)
    rs = rng.uniform(0, 1, (3, P.ndof))
    rp = rng.uniform(0, 1, (3, P.ndof))
    delta = torch.zeros((3, P.ndof), dtype=torch.float64, device="cuda")
    iters = torch.zeros(3, dtype=torch.int32, device="cuda")
    rte.dsa_correct(P, dev(rs), dev(rp), delta, cg_rtol=1e-14, cg_maxit=20000, iters_out=iters,
                    ws=P.workspace("si_dsa"))
    delta = host(delta)
    it = host(iters)
    say(f"  cg iterations {it}")
    assert np.all(it > 0)
    for b, d in enumerate(discs):
        ref = odsa.MIPDSA2D(d).correct(d.apply_Ss(rs[b] - rp[b]))
        assert rel_err(delta[b], ref) < 1e-10, rel_err(delta[b], ref)


@pytest.fixture(scope="module")
def small_rom():
    train = W.c2_lattice([30000 + i for i in range(5)], n=12, n_phi=8)
    discs = [discretize(train, b) for b in range(train.B)]
    rom = orom.build_correction_rom(discs, orom.plane_affine(discs[0]), orom.plane_psi, window=3,
                                    r=9, eps_train=1e-12)
    return rom


def _rom_arrays(rom):
    return rom.dU_rho, rom.dU_iso, rom.A0, np.stack(rom.At + rom.As)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_rom_correct_matches_oracle(R, small_rom, precision):
    import torch
    rte, problems = R
    test = W.c2_lattice([20000 + i for i in range(19)], n=12, n_phi=8)
    say(f"rom_correct {precision}")
    P = problems.plane_problem(test)
    U_rho, U_iso, A0, A = _rom_arrays(small_rom)
    Rm = rte.Rom(P, U_rho, U_iso, A0, A, small_rom.eps_pod, small_rom.eps_train)
    psi = problems.plane_psi(test)
    rng = np.random.default_rng(3)
    rs = rng.uniform(0, 1, (test.B, P.ndof))
    rp = rs + 1e-3 * rng.normal(size=rs.shape)
    delta = torch.zeros((test.B, P.ndof), dtype=torch.float64, device="cuda")
    status = torch.full((test.B,), -1, dtype=torch.int32, device="cuda")
    rte.rom_correct(P, Rm, psi, dev(rs), dev(rp), delta, status_out=status, precision=precision)
    delta, status = host(delta), host(status)
    assert np.all(status == 0)
    tol = TOL64 if precision == "fp64" else TOL32
    for b in range(test.B):
        d = discretize(test, b)
        ref = small_rom.correct(d, d.apply_Ss(rs[b] - rp[b]))
        assert rel_err(delta[b], ref) < tol, (b, rel_err(delta[b], ref))


def test_rom_singular_system_reported(R, small_rom):
    import torch
    rte, problems = R
    test = W.c2_lattice([20000, 20001], n=12, n_phi=8)
    P = problems.plane_problem(test)
    U_rho, U_iso, A0, A = _rom_arrays(small_rom)
    say("rom singular")
    Rm = rte.Rom(P, U_rho, U_iso, np.zeros_like(A0), np.zeros_like(A), 1e-3, 1e-10)
    delta = torch.full((2, P.ndof), 7.0, dtype=torch.float64, device="cuda")
    status = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    z = torch.zeros((2, P.ndof), dtype=torch.float64, device="cuda")
    rte.rom_correct(P, Rm, problems.plane_psi(test), z + 1.0, z, delta, status_out=status)
    assert np.all(host(status) == 1)
    assert np.all(host(delta) == 7.0)      # untouched


def test_invalid_arguments_rejected(R):
    import torch
    rte, problems = R
    plane = W.random_plane(1, nx=4, ny=3, n_phi=8)
    P = problems.plane_problem(plane)
    ws = P.workspace()
    bad = dev(plane.sigma_s) * 0 + 5.0     # sigma_s > sigma_t somewhere
    Q = rte.Problem(2, 4, 3, *problems.quadrature.chebyshev_circle(8)[::2], dev(plane.sigma_t), bad,
                    dev(plane.G), dev(plane.g), dirs_y=problems.quadrature.chebyshev_circle(8)[1])
    with pytest.raises(rte.RteError):
        Q.check(ws)
    P.check(ws)
    tiny = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(rte.RteError) as e:
        rte.sweep(P, torch.zeros(P.ndof, dtype=torch.float64, device="cuda"),
                  rho_star_out=torch.zeros(P.ndof, dtype=torch.float64, device="cuda"), ws=tiny)
    assert e.value.status == rte.RTE_ENOMEM


def test_cg_limit_reports_ecg(R):
    """A diffusion CG that reaches its iteration limit is reported (RTE_ECG) by the correction
    call and by the solve, whose instances all still stop (here at max_iter)."""
    import torch
    rte, problems = R
    plane = W.random_plane(41, nx=16, ny=16, n_phi=8, B=2, Lx=10.0, Ly=10.0)
    say("cg limit: dsa_correct with cg_maxit = 1")
    P = problems.plane_problem(plane)
    rng = np.random.default_rng(2)
    rs, rp = dev(rng.uniform(0, 1, (2, P.ndof))), dev(rng.uniform(0, 1, (2, P.ndof)))
    delta = torch.zeros((2, P.ndof), dtype=torch.float64, device="cuda")
    with pytest.raises(rte.RteError) as e:
        rte.dsa_correct(P, rs, rp, delta, cg_rtol=1e-14, cg_maxit=1)
    assert e.value.status == rte.RTE_ECG
    rte.dsa_correct(P, rs, rp, delta, cg_rtol=1e-14, cg_maxit=5000)      # converges: no error
    say("cg limit: sisa_solve with cg_maxit = 1")
    rho = torch.zeros((2, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.sisa_solve(P, rho, mode="si_dsa", eps=1e-10, cg_rtol=1e-14, cg_maxit=1, max_iter=6,
                         raise_on_error=False)
    assert res.status == rte.RTE_ECG, res.status


def _media_with_materials(plane, counts, seed):
    """The plane with instance b's sigma_t made of counts[b] distinct values (None: one value per
    cell), sigma_s kept at the same fraction of sigma_t."""
    import dataclasses
    rng = np.random.default_rng(seed)
    st, ss = plane.sigma_t.copy(), plane.sigma_s.copy()
    for b, n in enumerate(counts):
        frac = ss[b] / st[b]
        if n is None:
            st[b] = rng.uniform(0.5, 20.0, st[b].shape)
        else:
            levels = rng.uniform(0.5, 20.0, n)
            ids = np.arange(st[b].size) % n
            rng.shuffle(ids)
            st[b] = levels[ids].reshape(st[b].shape)
        ss[b] = frac * st[b]
    return dataclasses.replace(plane, sigma_t=st, sigma_s=ss)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sweep2d_material_tables_beside_per_cell_instances(R, precision):
    """An instance whose sigma_t takes at most 16 values is swept from its material table, one
    with more (17, or a value per cell) by the per-cell kernel, in the same launch: every
    instance against the oracle, element by element (eq. (transport_sweep))."""
    import torch
    rte, problems = R
    counts = [1, 16, 17, None, 5]
    base = W.random_plane(321, nx=37, ny=70, n_phi=16, B=len(counts), nbx=3, nby=2)
    plane = _media_with_materials(base, counts, 5)
    for b, n in enumerate(counts):
        assert len(np.unique(plane.sigma_t[b])) == (n if n is not None else plane.sigma_t[b].size)
    say(f"sweep2d material tables {counts} {precision}")
    P = problems.plane_problem(plane)
    discs = [discretize(plane, b) for b in range(P.B)]
    rho_in = np.stack([_rand_rho(d, 11 + b) for b, d in enumerate(discs)])
    f_dtype = torch.float64 if precision == "fp64" else torch.float32
    fd = torch.zeros(rte.f_shape(P), dtype=f_dtype, device="cuda")
    rs = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
    rte.sweep(P, dev(rho_in), f_out=fd, rho_star_out=rs, precision=precision)
    rs, f = host(rs), host(fd)
    tol = TOL64 if precision == "fp64" else TOL32
    tol_f = TOL64 if precision == "fp64" else TOL32_F
    for b, d in enumerate(discs):
        r_or, f_or = d.sweep(rho_in[b], want_f=True)
        assert rel_err(rs[b], r_or) < tol, (b, counts[b], rel_err(rs[b], r_or))
        assert rel_err(f_natural(f[b], P), f_or) < tol_f, (b, counts[b])
