"""GPU offline POD construction vs the oracle's (GPU)."""
import numpy as np
import pytest

import rte_workloads as W
from oracle import rom as orom
from oracle.problem import discretize
from tests.gpu_common import dev, host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2402_10488_amd import offline, problems, rte
    return rte, problems, offline


def test_streaming_operator_matches_oracle(R):
    rte, problems, offline = R
    plane = W.random_plane(4, nx=11, ny=7, n_phi=12, B=1, Lx=1.3, Ly=0.9)
    say("apply_streaming")
    P = problems.plane_problem(plane)
    d = discretize(plane, 0)
    x = np.random.default_rng(2).normal(size=(3, d.nv, d.ndof))
    y = host(offline.apply_streaming(P, dev(x)))
    for v in range(3):
        ref = d.apply_D(x[v])
        assert rel_err(y[v], ref) < 1e-13


def test_gram_and_combine(R):
    import torch
    rte, problems, offline = R
    rng = np.random.default_rng(7)
    X = rng.normal(size=(37, 10007))
    Y = rng.normal(size=(21, 10007))
    say("gram")
    G = host(offline.gram(dev(X), dev(Y)))
    assert rel_err(G, X @ Y.T) < 1e-13
    cls = rng.integers(0, 3, 10007 // 4 + 1).astype(np.int32)
    Gc = host(offline.gram(dev(X), dev(Y), torch.as_tensor(cls, device="cuda"), 4, len(cls), 1))
    mask = cls[np.arange(10007) // 4] == 1
    assert rel_err(Gc, (X * mask) @ Y.T) < 1e-13
    Wm = rng.normal(size=(37, 5))
    say("combine")
    out = host(offline.combine(dev(X), dev(Wm)))
    assert rel_err(out, Wm.T @ X) < 1e-13


def test_symmetric_eigensolver(R):
    rte, problems, offline = R
    rng = np.random.default_rng(3)
    for n in (1, 7, 96):
        M = rng.normal(size=(n, n))
        S = M @ M.T + np.diag(np.logspace(-6, 2, n))
        say(f"sym_eig n={n}")
        ev, V = offline.sym_eig(dev(S))
        ev, V = host(ev), host(V)
        ref = np.linalg.eigvalsh(S)
        assert rel_err(np.sort(ev), ref) < 1e-12
        assert np.abs(V.T @ V - np.eye(n)).max() < 1e-12
        assert rel_err(S @ V, V * ev) < 1e-11


def test_pod_weights_and_small_products(R):
    """Ranking, truncation by eq. (pod_truncation), W = V S^-1 and the reduced products, against
    numpy on the same eigenpairs (ties included)."""
    rte, problems, offline = R
    rng = np.random.default_rng(11)
    n = 40
    ev = np.concatenate([np.logspace(4, -20, n - 4), [5.0, 5.0, 0.0, -1e-18]])
    rng.shuffle(ev)
    V, _ = np.linalg.qr(rng.normal(size=(n, n)))
    order = np.argsort(-ev, kind="stable")
    sv_ref = np.sqrt(np.clip(ev[order], 0.0, None))
    nz = int(np.sum(sv_ref > sv_ref[0] * 1e-13))
    for r_fix, eps_pod in ((0, 1e-6), (0, 1e-12), (7, 0.0), (n, 0.0)):
        say(f"pod_weights r={r_fix} eps={eps_pod}")
        sv, Wd, r, eps_eff = offline.pod_weights(dev(ev), dev(V), r_fix, eps_pod)
        if r_fix:
            r_ref = min(r_fix, nz)
        else:
            ratio = np.cumsum(sv_ref) / np.sum(sv_ref)
            r_ref = min(int(np.argmax(ratio >= 1.0 - eps_pod) + 1), nz)
        assert r == r_ref
        assert rel_err(sv, sv_ref) < 1e-15
        assert abs(eps_eff - max(0.0, 1.0 - sv_ref[:r].sum() / sv_ref.sum())) < 1e-14
        assert rel_err(host(Wd), V[:, order[:r]] / sv_ref[:r]) < 1e-15
    A = rng.normal(size=(33, 9))
    B = rng.normal(size=(33, 5))
    C = rng.normal(size=(9, 33))
    say("small_gemm")
    assert rel_err(host(offline.small_gemm(dev(A), dev(B), trans_a=True)), A.T @ B) < 1e-14
    assert rel_err(host(offline.small_gemm(dev(C), dev(B), alpha=-2.0)), -2.0 * C @ B) < 1e-14
    assert np.array_equal(host(offline.small_gemm(dev(C), alpha=-1.0)), -C)
    assert np.array_equal(host(offline.small_gemm(dev(A), trans_a=True)), A.T)


def test_offline_rom_matches_oracle_rom(R):
    """Same training set, window and rank: same singular values and the same ROMSA correction
    (a basis-independent output of the reduced model)."""
    import torch
    rte, problems, offline = R
    train = W.c2_lattice([30000 + i for i in range(5)], n=12, n_phi=8)
    say("offline rom build")
    ra = offline.build_correction_rom(train, r=9, window=3, eps_train=1e-12, cg_rtol=1e-13)
    discs = [discretize(train, b) for b in range(train.B)]
    ro = orom.build_correction_rom(discs, orom.plane_affine(discs[0]), orom.plane_psi, window=3,
                                   r=9, eps_train=1e-12)
    assert rel_err(ra.sv[:9], ro.sv[:9]) < 1e-8
    assert abs(ra.eps_pod - ro.eps_pod) < 1e-8
    test = W.c2_lattice([20000 + i for i in range(4)], n=12, n_phi=8)
    P = problems.plane_problem(test)
    Rm = rte.Rom(P, ra.U_rho, ra.U_iso, ra.A0, ra.A, ra.eps_pod, ra.eps_train)
    rng = np.random.default_rng(11)
    rs = rng.uniform(0, 1, (test.B, P.ndof))
    rp = rs + 1e-3 * rng.normal(size=rs.shape)
    delta = torch.zeros((test.B, P.ndof), dtype=torch.float64, device="cuda")
    rte.rom_correct(P, Rm, problems.plane_psi(test), dev(rs), dev(rp), delta)
    delta = host(delta)
    for b in range(test.B):
        d = discretize(test, b)
        ref = ro.correct(d, d.apply_Ss(rs[b] - rp[b]))
        assert rel_err(delta[b], ref) < 1e-7, rel_err(delta[b], ref)


def test_offline_rom_fp32_snapshots_and_chunks(R):
    """FP32 snapshot storage, training solved in chunks: the singular values and the ROMSA
    correction stay within FP32 storage rounding of the oracle's."""
    import torch
    rte, problems, offline = R
    train = W.c2_lattice([30000 + i for i in range(5)], n=12, n_phi=8)
    say("offline rom build, fp32 snapshots, chunks of 2")
    ra = offline.build_correction_rom(train, r=9, window=3, eps_train=1e-12, cg_rtol=1e-13,
                                      snapshot_dtype="fp32", chunk=2, slice_cols=4)
    discs = [discretize(train, b) for b in range(train.B)]
    ro = orom.build_correction_rom(discs, orom.plane_affine(discs[0]), orom.plane_psi, window=3,
                                   r=9, eps_train=1e-12)
    assert rel_err(ra.sv[:6], ro.sv[:6]) < 1e-6
    test = W.c2_lattice([20000 + i for i in range(3)], n=12, n_phi=8)
    P = problems.plane_problem(test)
    Rm = rte.Rom(P, ra.U_rho, ra.U_iso, ra.A0, ra.A, ra.eps_pod, ra.eps_train)
    rng = np.random.default_rng(11)
    rs = rng.uniform(0, 1, (test.B, P.ndof))
    rp = rs + 1e-3 * rng.normal(size=rs.shape)
    delta = torch.zeros((test.B, P.ndof), dtype=torch.float64, device="cuda")
    rte.rom_correct(P, Rm, problems.plane_psi(test), dev(rs), dev(rp), delta)
    delta = host(delta)
    for b in range(test.B):
        d = discretize(test, b)
        ref = ro.correct(d, d.apply_Ss(rs[b] - rp[b]))
        assert rel_err(delta[b], ref) < 1e-4, rel_err(delta[b], ref)
