"""Host-side argument checks of the C ABI (CPU only: every call here is rejected before any
device work, as the public header promises for argument errors)."""
import ctypes

import numpy as np
import pytest

from paper_2402_10488_amd import rte

lib = rte.lib
_vp = ctypes.c_void_p
FAKE = _vp(0x1000)          # a non-null "device pointer": never dereferenced on these paths


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _create(dim=2, nx=4, ny=3, batch=1, vx=(0.5, -0.5), vy=(0.5, 0.5), w=(0.5, 0.5),
            widths=None, lx=1.0, ly=1.0, dg=0, wpb=0, bands=0):
    keep = []
    _, pvx = _arr(vx); keep.append(_)
    _, pvy = _arr(vy); keep.append(_)
    _, pw = _arr(w); keep.append(_)
    pwd = None
    if widths is not None:
        _, pwd = _arr(widths); keep.append(_)
    d = rte.ProblemDesc(dim, nx, ny, batch, len(vx), lx, ly, pwd, pvx,
                        pvy if dim == 2 else None, pw, FAKE, FAKE, FAKE, FAKE)
    h = ctypes.c_void_p()
    rc = lib.rte_problem_create_sched(ctypes.byref(d), dg, wpb, bands, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("kw", [
    dict(dim=3),
    dict(nx=0),
    dict(batch=0),
    dict(w=(0.6, 0.6)),                                  # weights must sum to 1
    dict(w=(1.5, -0.5)),                                 # and be positive
    dict(vx=(0.0, -0.5), vy=(0.0, 0.5)),                 # no direction with vx = vy = 0
    dict(vx=(np.nan, -0.5)),
    dict(lx=0.0),
    dict(dg=16),                                         # 1, 2, 4 or 8 directions per lane
    dict(dg=3),
    dict(wpb=5),
    dict(bands=-1),                                      # 0 (automatic) to 16 bands in flight
    dict(bands=17),
    dict(dim=1, ny=2, widths=[0.25] * 4),                # a slab has one row
    dict(dim=1, ny=1, widths=[0.25, 0.0, 0.25, 0.5]),    # cell widths must be positive
    dict(dim=1, ny=1, widths=None),
])
def test_problem_create_rejects_invalid_descriptions(kw):
    rc, h = _create(**kw)
    assert rc == rte.RTE_EINVAL
    assert not h.value


def test_problem_create_rejects_null_arguments():
    h = ctypes.c_void_p()
    assert lib.rte_problem_create_tuned(None, 0, 0, ctypes.byref(h)) == rte.RTE_EINVAL
    assert lib.rte_problem_create_sched(None, 0, 0, 0, ctypes.byref(h)) == rte.RTE_EINVAL
    assert lib.rte_problem_bands(None, ctypes.byref(ctypes.c_int())) == rte.RTE_EINVAL


def test_entry_points_reject_a_null_problem():
    opts = rte.SolveOpts(1e-6, 10, 1, 0, -1.0, 1e-10, 100, 0, 1)
    n = ctypes.c_size_t()
    assert lib.rte_workspace_size(None, 0, None, 0, 1, ctypes.byref(n)) == rte.RTE_EINVAL
    assert lib.rte_sweep(None, FAKE, FAKE, FAKE, 0, 0, FAKE, 1024, None) == rte.RTE_EINVAL
    assert lib.rte_scalar_flux(None, FAKE, FAKE, 0, None) == rte.RTE_EINVAL
    assert lib.rte_f_natural(None, FAKE, FAKE, 0, None) == rte.RTE_EINVAL
    assert lib.rte_dsa_correct(None, FAKE, FAKE, FAKE, 1e-10, 100, None, FAKE, 1024,
                               None) == rte.RTE_EINVAL
    assert lib.rte_sisa_solve(None, 1, None, None, ctypes.byref(opts), FAKE, None, None, FAKE,
                              1024, None) == rte.RTE_EINVAL


def test_offline_building_blocks_check_their_arguments():
    from paper_2402_10488_amd import offline  # noqa: F401  (sets the argument types)
    G = FAKE
    # null operand, empty shapes, unknown precision code
    assert lib.rte_gram(None, 0, 4, FAKE, 0, 4, 16, None, 4, 1, 0, G, FAKE, 1 << 20,
                        None) == rte.RTE_EINVAL
    assert lib.rte_gram(FAKE, 0, 0, FAKE, 0, 4, 16, None, 4, 1, 0, G, FAKE, 1 << 20,
                        None) == rte.RTE_EINVAL
    assert lib.rte_gram(FAKE, 7, 4, FAKE, 0, 4, 16, None, 4, 1, 0, G, FAKE, 1 << 20,
                        None) == rte.RTE_EINVAL
    assert lib.rte_sym_eig(FAKE, 300, FAKE, FAKE, None) == rte.RTE_EINVAL    # n <= 256
    assert lib.rte_sym_eig(FAKE, 0, FAKE, FAKE, None) == rte.RTE_EINVAL
    assert lib.rte_combine(FAKE, 0, 16, FAKE, 2, FAKE, None) == rte.RTE_EINVAL
    for fn in (lib.rte_apply_streaming, lib.rte_direction_sum, lib.rte_inflow_loads):
        assert fn.argtypes is not None
    assert lib.rte_apply_streaming(None, FAKE, 0, 1, FAKE, None) == rte.RTE_EINVAL
    assert lib.rte_inflow_loads(None, FAKE, 0, 1, FAKE, None) == rte.RTE_EINVAL
    assert lib.rte_direction_sum(None, FAKE, 0, 1, 1, FAKE, None) == rte.RTE_EINVAL
    assert lib.rte_pod_snapshots(None, FAKE, None, FAKE, 1, 0, None) == rte.RTE_EINVAL


def test_status_strings_and_profile_ids():
    for code in range(8):
        assert lib.rte_strerror(code)
    t, c = ctypes.c_double(), ctypes.c_longlong()
    assert lib.rte_profile_read(99, ctypes.byref(t), ctypes.byref(c)) == rte.RTE_EINVAL


def test_last_device_error_is_empty_when_no_hip_call_failed():
    """Argument errors are not device errors: after any number of rejected calls the HIP error
    detail stays empty (the binding appends it to RTE_EDEVICE messages only)."""
    rc, _ = _create(nx=0)
    assert rc == rte.RTE_EINVAL
    assert lib.rte_last_device_error() == b""
    assert "HIP" not in str(rte.RteError(rte.RTE_EINVAL, "x"))


def test_multi_batch_solve_checks_its_arguments():
    """rte_sisa_solve_multi rejects a bad count, missing arrays or entries, and batches that share
    a handle, a density array or workspace bytes, before any device work."""
    o = rte.SolveOpts(1e-6, 10, 1, 5, -1.0, 1e-3, 100, 0, 4, 0)
    P2 = _vp * 2
    sizes = (ctypes.c_size_t * 2)(1 << 20, 1 << 20)
    streams = P2(None, None)
    a, b = _vp(0x1000), _vp(0x2000)
    ws_apart = P2(_vp(0x100000), _vp(0x300000))

    def call(n, probs, rho, ws, sz=sizes):
        return lib.rte_sisa_solve_multi(n, probs, 1, None, None, ctypes.byref(o), rho, None, None,
                                        ws, sz, streams, None)

    assert call(0, P2(a, b), P2(a, b), ws_apart) == rte.RTE_EINVAL
    assert call(17, P2(a, b), P2(a, b), ws_apart) == rte.RTE_EINVAL
    assert call(2, None, P2(a, b), ws_apart) == rte.RTE_EINVAL
    assert call(2, P2(a, None), P2(a, b), ws_apart) == rte.RTE_EINVAL
    assert call(2, P2(a, a), P2(a, b), ws_apart) == rte.RTE_EINVAL            # shared handle
    assert call(2, P2(a, b), P2(a, a), ws_apart) == rte.RTE_EINVAL            # shared densities
    overlap = P2(_vp(0x100000), _vp(0x180000))                                 # 1 MiB apart by half
    assert call(2, P2(a, b), P2(a, b), overlap) == rte.RTE_EINVAL
    assert lib.rte_sisa_solve_multi(2, P2(a, b), 1, None, None, None, P2(a, b), None, None,
                                    ws_apart, sizes, streams, None) == rte.RTE_EINVAL
