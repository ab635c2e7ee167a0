"""Normalized angular rules of Sec. 2.1 (weights sum to one).

Host-side set-up of the direction tables handed to the library.
"""
import numpy as np


def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes on [-1,1] with weights halved (rho = 1/2 int f dxi)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return np.asarray(x, np.float64), np.asarray(w, np.float64) * 0.5


def chebyshev_circle(n_phi: int):
    """Angles (2j - 1) pi / N_phi, j = 1..N_phi, each of weight 1/N_phi -> (vx, vy, w)."""
    phi = (2.0 * np.arange(1, n_phi + 1) - 1.0) * np.pi / n_phi
    return np.cos(phi), np.sin(phi), np.full(n_phi, 1.0 / n_phi)


def chebyshev_legendre(n_phi: int, n_vz: int):
    """CL(N_phi, N_vz) rule on the sphere (Sec. 2.1): the tensor product of the N_phi-point
    Chebyshev rule in the azimuth and the N_vz-point Gauss-Legendre rule in v_z, weights
    multiplied.  For X-Y geometry only the in-plane components matter:
    (vx, vy) = sqrt(1 - vz^2) (cos phi, sin phi).  Ordered with the azimuth fastest.
    Returns (vx, vy, w)."""
    cx, cy, cw = chebyshev_circle(n_phi)
    z, zw = gauss_legendre(n_vz)
    s = np.sqrt(1.0 - z * z)
    vx = (s[:, None] * cx[None, :]).reshape(-1)
    vy = (s[:, None] * cy[None, :]).reshape(-1)
    w = (zw[:, None] * cw[None, :]).reshape(-1)
    return vx, vy, w


def plane_rule(quad):
    """Direction table (vx, vy, w) of a 2D problem's quadrature description:
    ("cheb", N_phi) or ("cl", (N_phi, N_vz))."""
    kind, n = quad
    if kind == "cheb":
        return chebyshev_circle(n)
    if kind == "cl":
        return chebyshev_legendre(*n)
    raise ValueError(f"unknown quadrature {quad!r}")
