"""Oracle: ctypes binding of the plain C FP64 sweeps in oracle/csweep.c.

Test infrastructure only -- never imported by the product path.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csweep.c")
_LIB = os.path.join(_HERE, "liboracle_sweep.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile csweep.c with gcc (-O2, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.oracle_sweep1d.restype = ctypes.c_int
        L.oracle_sweep1d.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D, _D, _D,
                                     ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_sweep2d.restype = ctypes.c_int
        L.oracle_sweep2d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int] + [_D] * 14
        L.oracle_apply_D2d.restype = None
        L.oracle_apply_D2d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int] + [_D] * 7
        L.oracle_apply_D1d.restype = None
        L.oracle_apply_D1d.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _c(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def sweep1d(mu, w, K, E, bl, src, g_left, g_right, q=None, want_f=False):
    nv, nc = K.shape[0], K.shape[1]
    mu, w, K, E, bl, src, q = map(_c, (mu, w, K, E, bl, src, q))
    rho = np.zeros((nc, 2))
    f = np.zeros((nv, nc, 2)) if want_f else None
    rc = lib().oracle_sweep1d(nc, nv, _p(mu), _p(w), _p(K), _p(E), _p(bl), _p(src), _p(q),
                              float(g_left), float(g_right), _p(f), _p(rho))
    if rc:
        raise RuntimeError(f"oracle_sweep1d failed ({rc})")
    return rho, f


def sweep2d(nx, ny, vx, vy, w, V, Ex, Ey, bx, by, sigma_t, src, g, q=None, want_f=False):
    nv = len(vx)
    args = list(map(_c, (vx, vy, w, V, Ex, Ey, bx, by, sigma_t, src, q, g)))
    rho = np.zeros((nx * ny, 4))
    f = np.zeros((nv, nx * ny, 4)) if want_f else None
    vx, vy, w, V, Ex, Ey, bx, by, sigma_t, src, q, g = args
    rc = lib().oracle_sweep2d(nx, ny, nv, _p(vx), _p(vy), _p(w), _p(V), _p(Ex), _p(Ey), _p(bx),
                              _p(by), _p(sigma_t), _p(src), _p(q), _p(g), _p(f), _p(rho))
    if rc:
        raise RuntimeError(f"oracle_sweep2d failed ({rc})")
    return rho, f


def apply_D2d(nx, ny, vx, vy, V, Ex, Ey, x):
    x = _c(x)
    y = np.empty_like(x)
    vx, vy, V, Ex, Ey = map(_c, (vx, vy, V, Ex, Ey))
    lib().oracle_apply_D2d(nx, ny, len(vx), _p(vx), _p(vy), _p(V), _p(Ex), _p(Ey), _p(x), _p(y))
    return y


def apply_D1d(mu, V, E, x):
    x = _c(x)
    y = np.empty_like(x)
    mu, V, E = map(_c, (mu, V, E))
    lib().oracle_apply_D1d(V.shape[1], len(mu), _p(mu), _p(V), _p(E), _p(x), _p(y))
    return y
