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


def test_cholesky_and_jacobi_svd_kernels(R):
    """rte_chol_upper (plain and shifted) and rte_svd_jacobi against their definitions and numpy,
    on matrices with singular values down to 1e-13 of the largest."""
    import torch
    rte, problems, offline = R
    rng = np.random.default_rng(17)
    for n in (1, 5, 24, 61):
        M = rng.normal(size=(n, n))
        G = M @ M.T + n * np.eye(n)
        say(f"chol_upper n={n}")
        Rd, Td, info, dev_ = offline.chol_upper(dev(G))
        Rh, Th = host(Rd), host(Td)
        assert info == 0
        assert abs(dev_ - np.abs(G - np.eye(n)).max()) <= 1e-15 * np.abs(G).max()
        assert np.array_equal(np.triu(Rh), Rh) and np.array_equal(np.triu(Th), Th)
        assert rel_err(Rh.T @ Rh, G) < 1e-14
        assert rel_err(Rh, np.linalg.cholesky(G).T) < 1e-13
        assert np.abs(Rh @ Th - np.eye(n)).max() < 1e-13
        # the shifted factorization: G + s I with s = 11 (m n + n (n + 1)) u trace(G)
        m = 1000
        s_ = 11.0 * (m * n + n * (n + 1)) * 2.0 ** -53 * np.trace(G)
        Rs, _, info, _ = offline.chol_upper(dev(G), shift_rows=m)
        Rs = host(Rs)
        assert info == 0 and rel_err(Rs.T @ Rs, G + s_ * np.eye(n)) < 1e-14
    # a pivot that is not positive is reported, not hidden
    _, _, info, _ = offline.chol_upper(dev(np.diag([1.0, -1.0, 2.0])))
    assert info == 2
    for n in (1, 6, 33, 64):
        U0, _ = np.linalg.qr(rng.normal(size=(n, n)))
        V0, _ = np.linalg.qr(rng.normal(size=(n, n)))
        sig = np.logspace(0, -13, n)
        A = np.triu((U0 * sig) @ V0.T) if n > 1 else np.array([[3.0]])
        say(f"svd_jacobi n={n}")
        lam, V, US = offline.svd_jacobi(dev(A))
        lam, V, US = host(lam), host(V), host(US)
        ref = np.linalg.svd(A, compute_uv=False)
        s_gpu = np.sort(np.sqrt(lam))[::-1]
        assert np.all(np.abs(s_gpu - ref) <= 1e-14 * ref[0] + 1e-10 * ref)
        assert np.abs(V.T @ V - np.eye(n)).max() < 1e-13
        assert rel_err(US, A @ V) < 1e-13
        C = US.T @ US                                    # orthogonal columns of A V
        off = np.abs(C - np.diag(np.diag(C)))
        assert np.all(off <= 1e-14 * np.sqrt(np.outer(np.diag(C), np.diag(C))) + 1e-30)


def test_pod_qr_route_small_singular_values(R):
    """The QR route of the POD on columns with singular values down to 1e-12 of the largest:
    singular values and the basis against numpy's SVD (the Gram route cannot resolve them).
    (pod_weights keeps singular values above 1e-13 of the largest.)"""
    import torch
    rte, problems, offline = R
    rng = np.random.default_rng(23)
    n, L = 40, 30011
    U0, _ = np.linalg.qr(rng.normal(size=(L, n)))
    V0, _ = np.linalg.qr(rng.normal(size=(n, n)))
    sig = np.logspace(0, -12, n)
    F = (U0 * sig) @ V0.T
    say("pod_qr")
    sv, Wq, r, eps_eff, Q = offline.pod_qr([dev(F.T)], r=n)
    assert r == n
    assert np.all(np.abs(sv - sig) <= 2e-15 * sig[0] + 1e-8 * sig)
    Ub = host(offline.combine(Q, Wq))                   # [r, L], rows = basis vectors
    assert np.abs(Ub @ Ub.T - np.eye(n)).max() < 1e-12
    # each basis vector is the matching left singular vector, up to sign
    dots = np.abs(np.sum(Ub * U0.T, axis=1))
    assert np.all(np.abs(dots[:30] - 1.0) < 1e-9)
    # the Gram route on the same columns loses the tail
    X = dev(F.T)
    ev, Vg = offline.sym_eig(offline.gram(X, X))
    sv_g, _, _, _ = offline.pod_weights(ev, Vg, n, 0.0)
    say(f"  worst relative error of sv below 1e-9: QR {np.max(np.abs(sv - sig)[sig < 1e-9] / sig[sig < 1e-9]):.1e}, "
        f"Gram {np.max(np.abs(sv_g - sig)[sig < 1e-9] / sig[sig < 1e-9]):.1e}")


@pytest.mark.parametrize("pod", ["qr", "gram"])
def test_offline_rom_matches_oracle_rom(R, pod):
    """Same training set, window and rank: same singular values and the same ROMSA correction
    (a basis-independent output of the reduced model), by both POD routes."""
    import torch
    rte, problems, offline = R
    train = W.c2_lattice([30000 + i for i in range(5)], n=12, n_phi=8)
    say(f"offline rom build ({pod})")
    ra = offline.build_correction_rom(train, r=9, window=3, eps_train=1e-12, cg_rtol=1e-13,
                                      pod=pod)
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


def test_offline_rom_qr_route_at_the_papers_truncation(R):
    """The homogeneous-medium family (Sec. 4.3.1) at 16^2 with CL(8, 2), its 21 training values,
    window 3, truncated at eps_POD = 1e-9 as in the paper: the kept singular values reach 5e-9 of
    the largest and the first dropped ones lie below, where the Gram matrix no longer resolves
    them.  The library's QR route gives the oracle's rank and singular values (the oracle takes
    LAPACK's SVD) and a ROM whose ROMSA corrections equal the oracle ROM's (measured 3.8e-8)."""
    import torch
    rte, problems, offline = R
    quad = ("cl", (8, 2))
    train = W.homogeneous_medium(W.homogeneous_training(), 16, quad)
    say("offline rom build, homogeneous family, eps_pod 1e-9")
    ra = offline.build_correction_rom(train, r=None, eps_pod=1e-9, window=3, eps_train=1e-12,
                                      cg_rtol=1e-13)
    discs = [discretize(train, b) for b in range(train.B)]
    ro = orom.build_correction_rom(discs, orom.plane_affine(discs[0]), orom.plane_psi, window=3,
                                   eps_pod=1e-9, eps_train=1e-12)
    k = ro.r
    r_gpu = ra.U_rho.shape[1]
    say(f"  rank {r_gpu} (oracle {k}), sv[r-1]/sv[0] {ro.sv[k - 1] / ro.sv[0]:.1e}")
    assert r_gpu == k
    sv_a, sv_o = np.asarray(ra.sv)[:k + 2], np.asarray(ro.sv)[:k + 2]
    assert np.all(np.abs(sv_a - sv_o) <= 1e-13 * sv_o[0] + 1e-8 * sv_o)
    test = W.homogeneous_medium(W.homogeneous_test(3), 16, quad)
    P = problems.plane_problem(test)
    Rm = rte.Rom(P, ra.U_rho, ra.U_iso, ra.A0, ra.A, ra.eps_pod, ra.eps_train)
    rng = np.random.default_rng(13)
    rs = rng.uniform(0, 1, (test.B, P.ndof))
    rp = rs + 1e-3 * rng.normal(size=rs.shape)
    delta = torch.zeros((test.B, P.ndof), dtype=torch.float64, device="cuda")
    rte.rom_correct(P, Rm, problems.plane_psi(test), dev(rs), dev(rp), delta, precision="fp64")
    delta = host(delta)
    errs = []
    for b in range(test.B):
        d = discretize(test, b)
        errs.append(rel_err(delta[b], ro.correct(d, d.apply_Ss(rs[b] - rp[b]))))
    say(f"  ROMSA correction vs the oracle ROM's: max {max(errs):.1e}")
    assert max(errs) < 1e-6


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
