"""The paper's pin-cell (Sec. 4.3.3) and variable-scattering (Sec. 4.3.4) families on the GPU
against the oracle, at small sizes: SI-DSA, ROMSAD with the oracle's correction ROM, the ROM
initial guess (ROMIG) with the oracle's parametric ROM followed by SI-DSA, and
DSA-preconditioned GMRES.  Equal sweep counts (and correction kinds) and densities within 1e-12
(FP64) or 1e-5 (mixed precision) (GPU)."""
import numpy as np
import pytest

import rte_workloads as W
from oracle import rom as orom
from oracle.pgmres import pgmres
from oracle.problem import discretize
from oracle.sisa import sisa
from tests.gpu_common import first_divergence, host, rel_err, say

pytestmark = pytest.mark.gpu

QUAD = ("cl", (8, 2))
N = 16


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2402_10488_amd import problems, rte
    return rte, problems


def _family(name):
    if name == "pin_cell":
        train = W.pin_cell(W.pin_cell_training()[::3], n=N, quad=QUAD)
        test = W.pin_cell(W.pin_cell_test(3), n=N, quad=QUAD)
    else:
        train = W.variable_scattering(W.variable_scattering_training()[::7], n=N, quad=QUAD)
        test = W.variable_scattering(W.variable_scattering_test(3), n=N, quad=QUAD)
    return train, test


@pytest.fixture(scope="module", params=["pin_cell", "variable_scattering"])
def fam(request):
    train, test = _family(request.param)
    discs = [discretize(train, b) for b in range(train.B)]
    say(f"{request.param}: oracle ROMs from {train.B} training solves")
    crom = orom.build_correction_rom(discs, orom.plane_affine(discs[0]), orom.plane_psi, window=3,
                                     eps_pod=1e-9, eps_train=1e-12)
    prom = orom.build_parametric_rom(discs, orom.plane_affine(discs[0]), orom.plane_psi,
                                     eps_pod=1e-9, eps_train=1e-12)
    return request.param, test, crom, prom


def test_family_si_dsa(R, fam):
    import torch
    rte, problems = R
    name, test, _, _ = fam
    P = problems.plane_problem(test)
    say(f"{name}: si_dsa fp64")
    rho = torch.zeros((test.B, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.sisa_solve(P, rho, mode="si_dsa", eps=1e-10, precision="fp64", cg_rtol=1e-13,
                         max_iter=500)
    rho = host(rho)
    for b in range(test.B):
        ref = sisa(discretize(test, b), "si_dsa", eps=1e-10)
        assert res.n_sweep[b] == ref.n_sweep, (b, res.n_sweep[b], ref.n_sweep)
        assert rel_err(rho[b], ref.rho) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_family_romsad(R, fam, precision):
    import torch
    rte, problems = R
    name, test, rom, _ = fam
    P = problems.plane_problem(test)
    Rm = rte.Rom(P, rom.dU_rho, rom.dU_iso, rom.A0, np.stack(rom.At + rom.As), rom.eps_pod,
                 rom.eps_train)
    eps = 1e-10 if precision == "fp64" else 1e-6
    say(f"{name}: romsad {precision} (r_c = {rom.r})")
    rho = torch.zeros((test.B, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.sisa_solve(P, rho, mode="romsad", rom=Rm, psi=problems.plane_psi(test), eps=eps,
                         theta=5, precision=precision, cg_rtol=1e-13, max_iter=500)
    rho = host(rho)
    eps_romsad = 0.1 * max(rom.eps_train, rom.eps_pod)
    for b in range(test.B):
        d = discretize(test, b)
        ref = sisa(d, "romsad", eps=eps, rom=rom, theta=5)
        if precision == "mixed":
            # A mixed-precision trajectory may leave the FP64 oracle's only where a decision
            # straddles its threshold within the precision to which the FP32 sweep measures the
            # relative change e_l.  e_l ~ 1e-6 is the difference of two swept densities that each
            # carry FP32 rounding of a few 1e-7 of themselves; between sweeps of nearly the same
            # input those errors cancel (1e-3 of e_l in the full-size batch), but right after a
            # ROMSA correction has changed the input they do not, and e_l is known to some tens
            # of percent (measured: the pin cell's instance 1 after its correction, GPU e_2 15%
            # below the oracle's).  Accepted: the oracle's e_l within 30% of the threshold; the
            # density must still be within 1e-5.
            assert rel_err(rho[b], ref.rho) < 1e-5
            div = first_divergence(res, b, ref.n_sweep, ref.kinds)
            if div is not None:
                l, what = div
                thr = eps if what == "stop" else eps_romsad
                e_or, e_gpu = ref.changes[l - 1], float(res.change[b, l - 1])
                say(f"  instance {b}: {what} decision after sweep {l} differs: oracle e_l "
                    f"{e_or:.6e}, GPU e_l {e_gpu:.6e}, threshold {thr:.3e}")
                assert abs(e_or - thr) <= 0.3 * thr, (b, l, what, e_or, e_gpu, thr)
        else:
            assert res.n_sweep[b] == ref.n_sweep, (b, res.n_sweep[b], ref.n_sweep)
            assert list(res.kind[b, :res.n_sweep[b] - 1]) == ref.kinds
            assert rel_err(rho[b], ref.rho) < 1e-12


def test_family_romig_then_si_dsa(R, fam):
    import torch
    rte, problems = R
    name, test, _, prom = fam
    P = problems.plane_problem(test)
    d0 = discretize(test, 0)
    U = prom.U.reshape(d0.nv, d0.ndof, -1)
    Rm = rte.Rom(P, prom.U_rho, U.sum(axis=0), prom.A0, np.stack(prom.At + prom.As), 1e-9, 1e-12)
    say(f"{name}: romig (r_p = {prom.U.shape[1]}) + si_dsa fp64")
    rho = torch.zeros((test.B, P.ndof), dtype=torch.float64, device="cuda")
    rte.rom_initial_guess(P, Rm, problems.plane_psi(test), rho)
    guess = host(rho)
    res = rte.sisa_solve(P, rho, mode="si_dsa", eps=1e-10, precision="fp64", cg_rtol=1e-13,
                         max_iter=500)
    rho = host(rho)
    for b in range(test.B):
        d = discretize(test, b)
        g_or = prom.initial_guess(d)
        assert rel_err(guess[b], g_or) < 1e-10
        ref = sisa(d, "si_dsa", eps=1e-10, rho0=g_or)
        assert res.n_sweep[b] == ref.n_sweep, (b, res.n_sweep[b], ref.n_sweep)
        assert rel_err(rho[b], ref.rho) < 1e-12


def test_family_pgmres(R, fam):
    import torch
    rte, problems = R
    name, test, _, _ = fam
    P = problems.plane_problem(test)
    say(f"{name}: pgmres fp64")
    rho = torch.zeros((test.B, P.ndof), dtype=torch.float64, device="cuda")
    res = rte.pgmres_solve(P, rho, tol=1e-10, restart=25, cg_rtol=1e-13)
    rho = host(rho)
    for b in range(test.B):
        ref = pgmres(discretize(test, b), tol=1e-10, m=25)
        assert ref.converged and res.inst_status[b] == 0
        assert res.iterations[b] == ref.iterations and res.n_sweep[b] == ref.n_sweep
        assert rel_err(rho[b], ref.rho) < 5e-9
