"""Oracle: diffusion synthetic acceleration operators (paper Sec. 2.3, eq.
(diffusion_correction); consistent slab DSA of Appendix B).

Test infrastructure only -- never imported by the product path.

Slab (``ConsistentDSA1D``): the D^+ and D^- operators of Appendix B are
assembled term by term from their definitions (volume integral, interior
edge products, boundary edge products, with inflow edges excluded), then
D_C = (D^+ + D^-)/2, D_J = D^+ - D^-, and the coupled system of
eq. (dsa_rho) and eq. (dsa_J) for (delta rho, delta J) is solved directly.

Plane (``MIPDSA2D``): the paper does not print its 2D diffusion
discretization (it cites a consistent DSA solved by AMG).  The reading used
here is the symmetric interior-penalty DG diffusion form of modified
interior-penalty (MIP) type on the same Q1 space:

  a(u,w) = sum_T int_T (D grad u . grad w + sigma_a u w)
         + sum_{interior e} int_e ( kappa_e [u][w] - {D d_n u}[w] - [u]{D d_n w} )
         + sum_{boundary e} int_e ( kappa_e u w - 1/2 D d_n u w - 1/2 u D d_n w )

with D = diag(sum_j w_j vx_j^2, sum_j w_j vy_j^2) / sigma_t (eq.
(diffusion_correction) with 1/sigma_t), [u] = u^- - u^+ and n pointing from
- to +, {q} the edge average, and
  kappa_e = max(kappa_min, kappa_IP),
  kappa_min = sum_{v_j . n > 0} w_j v_j . n        (from the direction set),
  kappa_IP  = (C/2) (D^-_n / h^-_perp + D^+_n / h^+_perp)  interior,
              C D_n / h_perp                            boundary,   C = 4.
The system is factorized once (sparse LU) and solved directly.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dg

MIP_C = 4.0


# ---------------------------------------------------------------------------
# Slab: Appendix B
# ---------------------------------------------------------------------------
def slab_Dpm(edges):
    """D^+ and D^- of Appendix B (sparse N_DOF x N_DOF, N_DOF = 2 nc)."""
    edges = np.asarray(edges, dtype=np.float64)
    nc = len(edges) - 1
    n = 2 * nc
    vol = np.zeros((n, n))
    for c in range(nc):
        xl, xr = edges[c], edges[c + 1]
        h = xr - xl
        xq = 0.5 * (xl + xr) + 0.5 * h * dg._GX
        val, der = dg._phi1d(xl, xr, xq)
        # - int d_x phi_k phi_l
        vol[2 * c:2 * c + 2, 2 * c:2 * c + 2] -= np.einsum("kq,lq,q->kl", der, val, 0.5 * h * dg._GW)

    def trace_minus(e):   # values of the two basis functions of the cell left of edge e at x_e
        return dg._phi1d(edges[e - 1], edges[e], edges[e])[0]

    def trace_plus(e):    # values of the two basis functions of the cell right of edge e at x_e
        return dg._phi1d(edges[e], edges[e + 1], edges[e])[0]

    Dp = vol.copy()
    Dm = vol.copy()
    # D^+: + sum_{i=1}^{Nx-1} phi_l(x+_{i+1/2}) phi_k(x-_{i+1/2})   (interior edges e = 1..nc-1)
    for e in range(1, nc):
        pm, pp = trace_minus(e), trace_plus(e)
        Dp[2 * (e - 1):2 * e, 2 * e:2 * e + 2] += np.outer(pm, pp)       # k in left cell, l in right cell
    # D^+: - sum_{i=1}^{Nx} phi_l(x+_{i-1/2}) phi_k(x+_{i-1/2})     (left edges of all cells, e = 0..nc-1)
    for e in range(0, nc):
        pp = trace_plus(e)
        Dp[2 * e:2 * e + 2, 2 * e:2 * e + 2] -= np.outer(pp, pp)
    # D^-: + sum_{i=1}^{Nx} phi_l(x-_{i+1/2}) phi_k(x-_{i+1/2})     (right edges of all cells, e = 1..nc)
    for e in range(1, nc + 1):
        pm = trace_minus(e)
        Dm[2 * (e - 1):2 * e, 2 * (e - 1):2 * e] += np.outer(pm, pm)
    # D^-: - sum_{i=2}^{Nx} phi_l(x-_{i-1/2}) phi_k(x+_{i-1/2})     (interior edges e = 1..nc-1)
    for e in range(1, nc):
        pm, pp = trace_minus(e), trace_plus(e)
        Dm[2 * e:2 * e + 2, 2 * (e - 1):2 * e] -= np.outer(pp, pm)       # k in right cell, l in left cell
    return sp.csr_matrix(Dp), sp.csr_matrix(Dm)


class ConsistentDSA1D:
    """Appendix B consistent DSA for the slab, solved directly."""

    def __init__(self, disc):
        self.disc = disc
        Dp, Dm = slab_Dpm(disc.edges)
        self.Dp, self.Dm = Dp, Dm
        self.DC = 0.5 * (Dp + Dm)
        self.DJ = Dp - Dm
        mu, w = disc.mu, disc.w
        self.c1 = float(np.sum(w[mu > 0] * mu[mu > 0]))
        self.c2 = float(np.sum(w * mu ** 2))
        self.c3 = float(np.sum(w[mu > 0] * mu[mu > 0] ** 3))
        St, Ss = disc.sigma_blocks()
        Sa = St - Ss
        top = sp.hstack([Sa - self.c1 * self.DJ, self.DC])
        bot = sp.hstack([self.c2 * self.DC, St - 3.0 * self.c3 * self.DJ])
        self.M = sp.vstack([top, bot]).tocsc()
        self.lu = spla.splu(self.M)
        self.n = disc.ndof

    def correct(self, rhs):
        """delta rho solving eq. (dsa_rho)-(dsa_J) for the source rhs = Sigma_s (rho^* - rho)."""
        b = np.concatenate([rhs.reshape(-1), np.zeros(self.n)])
        x = self.lu.solve(b)
        return x[:self.n]


# ---------------------------------------------------------------------------
# Plane: MIP diffusion form
# ---------------------------------------------------------------------------
def _edge_points(h):
    return 0.5 * h * (1 + dg._GX), 0.5 * h * dg._GW


class MIPDSA2D:
    """Symmetric interior-penalty diffusion correction on the Q1 DG space."""

    def __init__(self, disc, C: float = MIP_C):
        self.disc = disc
        nx, ny, hx, hy = disc.nx, disc.ny, disc.hx, disc.hy
        vx, vy, w = disc.vx, disc.vy, disc.w
        if np.any(disc.sigma_t <= 0):
            raise ValueError("diffusion correction needs sigma_t > 0 in every cell")
        cxx = float(np.sum(w * vx ** 2))
        cyy = float(np.sum(w * vy ** 2))
        self.Dx = cxx / disc.sigma_t        # per cell
        self.Dy = cyy / disc.sigma_t
        self.kmin_x = float(np.sum(w[vx > 0] * vx[vx > 0]))
        self.kmin_y = float(np.sum(w[vy > 0] * vy[vy > 0]))
        self.C = C
        self.A = self._assemble(nx, ny, hx, hy, disc.sigma_a).tocsc()
        self.lu = spla.splu(self.A)

    def _assemble(self, nx, ny, hx, hy, sa):
        X, Y, W = dg._vol_points(hx, hy)
        val, gx, gy = dg._phi2d(0.0, 0.0, hx, hy, X, Y)
        Kxx = np.einsum("kq,lq,q->kl", gx, gx, W)
        Kyy = np.einsum("kq,lq,q->kl", gy, gy, W)
        Mm = np.einsum("kq,lq,q->kl", val, val, W)
        rows, cols, vals = [], [], []

        def add(ca, cb, M):
            for k in range(4):
                for l in range(4):
                    rows.append(4 * ca + k)
                    cols.append(4 * cb + l)
                    vals.append(M[k, l])

        Dx, Dy = self.Dx, self.Dy
        for c in range(nx * ny):
            add(c, c, Dx[c] * Kxx + Dy[c] * Kyy + sa[c] * Mm)

        # reference edge quantities for a vertical edge at x = hx between cell L=[0,hx] and R=[hx,2hx]
        ey, wy = _edge_points(hy)
        pL, gxL, _ = dg._phi2d(0.0, 0.0, hx, hy, np.full_like(ey, hx), ey)
        pR, gxR, _ = dg._phi2d(hx, 0.0, hx, hy, np.full_like(ey, hx), ey)
        # horizontal edge at y = hy between cell D=[0,hy] (below, -) and U=[hy,2hy] (above, +)
        ex, wx = _edge_points(hx)
        pD, _, gyD = dg._phi2d(0.0, 0.0, hx, hy, ex, np.full_like(ex, hy))
        pU, _, gyU = dg._phi2d(0.0, hy, hx, hy, ex, np.full_like(ex, hy))

        def interior(cm, cp, Pm, Pp, Gm, Gp, wq, Dm_n, Dp_n, kap):
            # sides: s=+1 for the '-' cell, -1 for the '+' cell; Gs = normal derivative (n from - to +)
            sides = [(cm, Pm, Gm, 1.0, Dm_n), (cp, Pp, Gp, -1.0, Dp_n)]
            for ca, Pa, Ga, sa_, Da in sides:        # test function w = phi_k of cell a
                for cb, Pb, Gb, sb, Db in sides:     # trial function u = phi_l of cell b
                    jj = np.einsum("kq,lq,q->kl", sa_ * Pa, sb * Pb, wq)          # [u][w]
                    avg_u = np.einsum("kq,lq,q->kl", sa_ * Pa, 0.5 * Db * Gb, wq)  # {D d_n u}[w]
                    avg_w = np.einsum("kq,lq,q->kl", 0.5 * Da * Ga, sb * Pb, wq)   # [u]{D d_n w}
                    add(ca, cb, kap * jj - avg_u - avg_w)

        def boundary(c, P, Gn, wq, Dn, kap):
            M = (kap * np.einsum("kq,lq,q->kl", P, P, wq)
                 - 0.5 * Dn * np.einsum("kq,lq,q->kl", P, Gn, wq)
                 - 0.5 * Dn * np.einsum("kq,lq,q->kl", Gn, P, wq))
            add(c, c, M)

        C = self.C
        for j in range(ny):
            for i in range(nx):
                c = j * nx + i
                if i + 1 < nx:      # vertical interior edge between (i,j) and (i+1,j)
                    r = c + 1
                    kap = max(self.kmin_x, 0.5 * C * (Dx[c] / hx + Dx[r] / hx))
                    interior(c, r, pL, pR, gxL, gxR, wy, Dx[c], Dx[r], kap)
                if j + 1 < ny:      # horizontal interior edge between (i,j) and (i,j+1)
                    u = c + nx
                    kap = max(self.kmin_y, 0.5 * C * (Dy[c] / hy + Dy[u] / hy))
                    interior(c, u, pD, pU, gyD, gyU, wx, Dy[c], Dy[u], kap)
        # boundary edges: outward normals, each cell's own traces
        pl, gxl, _ = dg._phi2d(0.0, 0.0, hx, hy, np.zeros_like(ey), ey)
        pr, gxr, _ = dg._phi2d(0.0, 0.0, hx, hy, np.full_like(ey, hx), ey)
        pb, _, gyb = dg._phi2d(0.0, 0.0, hx, hy, ex, np.zeros_like(ex))
        pt, _, gyt = dg._phi2d(0.0, 0.0, hx, hy, ex, np.full_like(ex, hy))
        for j in range(ny):
            for side, i, P, Gn in ((0, 0, pl, -gxl), (1, nx - 1, pr, gxr)):
                c = j * nx + i
                boundary(c, P, Gn, wy, Dx[c], max(self.kmin_x, C * Dx[c] / hx))
        for i in range(nx):
            for side, j, P, Gn in ((2, 0, pb, -gyb), (3, ny - 1, pt, gyt)):
                c = j * nx + i
                boundary(c, P, Gn, wx, Dy[c], max(self.kmin_y, C * Dy[c] / hy))
        n = 4 * nx * ny
        return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))

    def correct(self, rhs):
        """delta rho = A^{-1} rhs for rhs = Sigma_s (rho^* - rho) (coefficients in the orthonormal basis)."""
        return self.lu.solve(np.asarray(rhs, dtype=np.float64).reshape(-1))


def make_dsa(disc):
    return ConsistentDSA1D(disc) if disc.dim == 1 else MIPDSA2D(disc)
