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
