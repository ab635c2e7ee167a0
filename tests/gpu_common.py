"""Shared helpers of the GPU parity tests: device upload of inputs and oracle runs."""
import os
import sys

import numpy as np


_capman = None


def set_capture_manager(capman):
    global _capman
    _capman = capman


def say(*a):
    """Print and flush the case name before a GPU step (so a fault names its case).  Under
    pytest the line bypasses output capture, so a long test shows its progress as it runs."""
    if _capman is not None:
        with _capman.global_and_fixture_disabled():
            print(*a, flush=True)
    else:
        print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a, b):
    """max |a - b| / max |b|.  With RTE_ERRLOG set, every value is appended to that file as a
    JSON line with the running test's id, so one run records the measured error of each check."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = max(np.abs(b).max(), 1e-300)
    e = float(np.abs(a - b).max() / den)
    log = os.environ.get("RTE_ERRLOG")
    if log:
        import json
        with open(log, "a") as fh:
            fh.write(json.dumps({"test": os.environ.get("PYTEST_CURRENT_TEST", "?"), "err": e}) + "\n")
    return e


def sweep_positions(nx, ny, vx, vy):
    """[n_dir, ncell] storage position of every natural cell in the library's 2D angular flux,
    written from the layout stated in the public header (band order of reflected coordinates)."""

    def T(d, m, M):
        e = d - M
        return np.where(d <= m, d * (d + 1) // 2,
                        np.where(d <= M, m * (m + 1) // 2 + (d - m) * m,
                                 m * (m + 1) // 2 + (M - m) * m + e * (m - 1) - e * (e - 1) // 2))

    y, x = np.divmod(np.arange(nx * ny, dtype=np.int64), nx)
    out = np.empty((len(vx), nx * ny), dtype=np.int64)
    for j, (a, b) in enumerate(zip(vx, vy)):
        xr = nx - 1 - x if a < 0 else x
        yr = ny - 1 - y if b < 0 else y
        k, r = np.divmod(yr, 64)
        h = np.minimum(64, ny - 64 * k)
        m, M = np.minimum(nx, h), np.maximum(nx, h)
        d = xr + r
        out[j] = 64 * nx * k + T(d, m, M) + r - np.maximum(0, d - nx + 1)
    return out


def f_natural(f_lib, P):
    """One instance's library angular flux -> the oracle's [n_dir][N_DOF] (natural order)."""
    f_lib = np.asarray(f_lib)
    if P.dim == 1:
        return np.ascontiguousarray(np.transpose(f_lib, (1, 0, 2))).reshape(P.n_dir, P.ndof)
    pos = sweep_positions(P.nx, P.ny, P._dx, P._dy)
    out = np.take_along_axis(f_lib, pos[:, :, None], axis=1)
    return out.reshape(P.n_dir, P.ndof)


def f_library(f_nat, P):
    """The oracle's [n_dir][N_DOF] -> one instance's library angular flux."""
    f3 = np.asarray(f_nat).reshape(P.n_dir, P.ncell, P.K)
    if P.dim == 1:
        return np.ascontiguousarray(np.transpose(f3, (1, 0, 2)))
    pos = sweep_positions(P.nx, P.ny, P._dx, P._dy)
    out = np.empty_like(f3)
    np.put_along_axis(out, pos[:, :, None], f3, axis=1)
    return out


def first_divergence(res, b, ns, kinds):
    """(l, kind) of the first iteration at which the GPU's trajectory of instance b leaves the
    oracle's: 'stop' (one stops at sweep l, the other does not) or 'switch' (Alg. 2 chose
    differently after sweep l); None if sweep counts and correction kinds are equal."""
    ng = int(res.n_sweep[b])
    gk = list(res.kind[b, :ng - 1])
    for l in range(1, min(ng, ns) + 1):
        g_stop, o_stop = l == ng, l == ns
        if g_stop != o_stop:
            return l, "stop"
        if g_stop:
            return None
        if gk[l - 1] != kinds[l - 1]:
            return l, "switch"
    return None
