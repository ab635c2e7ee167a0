"""Oracle: normalized angular quadrature rules (paper Sec. 2.1).

Test infrastructure only -- never imported by the product path.

The paper normalizes every rule so that the weights sum to one and
rho = sum_j w_j f_j approximates the normalized angular integral.
"""
import numpy as np


def gauss_legendre(n: int):
    """Normalized n-point Gauss-Legendre rule on [-1,1] (slab directions, Sec. 2.1).

    Nodes are numpy's textbook Gauss-Legendre nodes; weights are halved so
    that they sum to 1 (rho = 1/2 int f dxi).  Returns (mu[n], w[n]) with mu
    ascending.
    """
    x, w = np.polynomial.legendre.leggauss(n)
    return x.astype(np.float64), (w / 2.0).astype(np.float64)


def chebyshev_circle(n_phi: int):
    """Normalized N_phi-point Chebyshev rule on the unit circle (Sec. 2.1):
    phi_j = 2 j pi / N_phi - pi / N_phi, weight 1/N_phi, j = 1..N_phi.
    Returns (vx[n], vy[n], w[n])."""
    j = np.arange(1, n_phi + 1, dtype=np.float64)
    phi = 2.0 * j * np.pi / n_phi - np.pi / n_phi
    return np.cos(phi), np.sin(phi), np.full(n_phi, 1.0 / n_phi)


def chebyshev_legendre(n_phi: int, n_vz: int):
    """CL(N_phi, N_vz) tensor rule on S^2 (Sec. 2.1), ordered j = (j2-1) N_phi + j1.
    Returns (vx, vy, vz, w)."""
    cx, cy, cw = chebyshev_circle(n_phi)
    z, zw = gauss_legendre(n_vz)
    vx, vy, vz, w = [], [], [], []
    for j2 in range(n_vz):
        s = np.sqrt(1.0 - z[j2] ** 2)
        vx.append(cx * s)
        vy.append(cy * s)
        vz.append(np.full(n_phi, z[j2]))
        w.append(cw * zw[j2])
    return (np.concatenate(vx), np.concatenate(vy), np.concatenate(vz), np.concatenate(w))
