"""Oracle: upwind DG element operators (paper Sec. 2.2, eq. (DG), eq. (upwind),
eq. (dg_matrix_vec)), evaluated by Gauss quadrature of the orthonormal basis.

Test infrastructure only -- never imported by the product path.

Every integral below is the integral written in eq. (DG) / the definitions
under eq. (dg_matrix_vec), evaluated numerically with a Gauss rule that is
exact for the polynomial degree involved.  Nothing is hand-simplified.

Basis (orthonormal, as eq. (dg_matrix_vec) requires): on a cell with
reference coordinates t in [-1,1] per axis, L_0 = 1, L_1 = sqrt(3) t, and
phi_ab = L_a(xi) L_b(eta) / sqrt(hx hy) in 2D (local dof k = a + 2 b),
phi_a = L_a(t) / sqrt(h) in 1D.

Sign convention of the sweep equation used by the oracle sweeps:
    (V_j + Sigma_t) f_c = s_c - sum_{upwind neighbours N} E_j f_N + loads,
where V_j holds the volume term and the outflow-edge flux terms, E_j the
inflow-edge flux term coupling to the upwind neighbour's coefficients (the
upwind flux of eq. (upwind) takes the neighbour's trace on inflow edges),
and the boundary load is -int_e g phi (v.n) on inflow boundary edges.
"""
import numpy as np
import scipy.sparse as sp

_GX, _GW = np.polynomial.legendre.leggauss(4)   # exact to degree 7 on [-1,1]


def _leg(t):
    """Orthonormal-on-[-1,1] (w.r.t. dt/2) Legendre values and t-derivatives, degrees 0,1."""
    t = np.asarray(t, dtype=np.float64)
    val = np.stack([np.ones_like(t), np.sqrt(3.0) * t])
    der = np.stack([np.zeros_like(t), np.sqrt(3.0) * np.ones_like(t)])
    return val, der


# ---------------------------------------------------------------------------
# 1D
# ---------------------------------------------------------------------------
def _phi1d(xl, xr, x):
    """phi_a(x) and d phi_a/dx on cell [xl, xr] (zero outside is not needed)."""
    h = xr - xl
    t = (2.0 * np.asarray(x, dtype=np.float64) - xl - xr) / h
    v, d = _leg(t)
    return v / np.sqrt(h), d * (2.0 / h) / np.sqrt(h)


def slab_operators(edges, mu):
    """Per-direction, per-cell operators of the slab sweep.

    Returns V [nv, nc, 2, 2], E [nv, nc, 2, 2] (coupling to the upwind
    neighbour; zero for the boundary cell) and bload [nv, 2] (the load of a
    unit inflow on the inflow boundary cell).
    """
    edges = np.asarray(edges, dtype=np.float64)
    nc = len(edges) - 1
    nv = len(mu)
    V = np.zeros((nv, nc, 2, 2))
    E = np.zeros((nv, nc, 2, 2))
    bload = np.zeros((nv, 2))
    for j, m in enumerate(mu):
        for c in range(nc):
            xl, xr = edges[c], edges[c + 1]
            h = xr - xl
            xq = 0.5 * (xl + xr) + 0.5 * h * _GX
            val, der = _phi1d(xl, xr, xq)
            # volume term: - int (v . grad phi_k) phi_l
            V[j, c] -= m * np.einsum("kq,lq,q->kl", der, val, 0.5 * h * _GW)
            x_out, n_out, x_in, n_in = (xr, 1.0, xl, -1.0) if m > 0 else (xl, -1.0, xr, 1.0)
            po, _ = _phi1d(xl, xr, x_out)
            V[j, c] += m * n_out * np.outer(po, po)
            pi_, _ = _phi1d(xl, xr, x_in)
            nb = c - 1 if m > 0 else c + 1
            if 0 <= nb < nc:
                pn, _ = _phi1d(edges[nb], edges[nb + 1], x_in)
                E[j, c] = m * n_in * np.outer(pi_, pn)
            else:
                bload[j] = -m * n_in * pi_
    return V, E, bload


def slab_mass_weighted(edges, values):
    """Per-cell 2x2 matrices int sigma(x) phi_k phi_l for piecewise-linear
    sigma given by its (left, right) values per cell -> [nc, 2, 2]."""
    edges = np.asarray(edges, dtype=np.float64)
    nc = len(edges) - 1
    out = np.zeros((nc, 2, 2))
    for c in range(nc):
        xl, xr = edges[c], edges[c + 1]
        h = xr - xl
        xq = 0.5 * (xl + xr) + 0.5 * h * _GX
        sig = values[c, 0] + (values[c, 1] - values[c, 0]) * (xq - xl) / h
        val, _ = _phi1d(xl, xr, xq)
        out[c] = np.einsum("kq,lq,q->kl", val, val, sig * 0.5 * h * _GW)
    return out


def slab_load(edges, values):
    """Per-cell load vectors int G(x) phi_k for piecewise-linear G -> [nc, 2]."""
    edges = np.asarray(edges, dtype=np.float64)
    nc = len(edges) - 1
    out = np.zeros((nc, 2))
    for c in range(nc):
        xl, xr = edges[c], edges[c + 1]
        h = xr - xl
        xq = 0.5 * (xl + xr) + 0.5 * h * _GX
        G = values[c, 0] + (values[c, 1] - values[c, 0]) * (xq - xl) / h
        val, _ = _phi1d(xl, xr, xq)
        out[c] = val @ (G * 0.5 * h * _GW)
    return out


def slab_eval(edges, coef, x):
    """Evaluate a DG function with coefficients coef [nc, 2] at points x."""
    edges = np.asarray(edges)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    c = np.clip(np.searchsorted(edges, x, side="right") - 1, 0, len(edges) - 2)
    out = np.empty_like(x)
    for i, (ci, xi) in enumerate(zip(c, x)):
        v, _ = _phi1d(edges[ci], edges[ci + 1], xi)
        out[i] = v @ coef[ci]
    return out


# ---------------------------------------------------------------------------
# 2D uniform Cartesian mesh
# ---------------------------------------------------------------------------
def _phi2d(x0, y0, hx, hy, x, y):
    """phi_ab and its gradient for the cell [x0,x0+hx] x [y0,y0+hy] at points (x, y).
    Returns val [4, nq], gx [4, nq], gy [4, nq] with k = a + 2 b."""
    xi = (2.0 * (np.asarray(x, dtype=np.float64) - x0) - hx) / hx
    eta = (2.0 * (np.asarray(y, dtype=np.float64) - y0) - hy) / hy
    lx, dx = _leg(xi)
    ly, dy = _leg(eta)
    s = 1.0 / np.sqrt(hx * hy)
    val = np.stack([lx[a] * ly[b] for b in range(2) for a in range(2)]) * s
    gx = np.stack([dx[a] * (2.0 / hx) * ly[b] for b in range(2) for a in range(2)]) * s
    gy = np.stack([lx[a] * dy[b] * (2.0 / hy) for b in range(2) for a in range(2)]) * s
    return val, gx, gy


def _vol_points(hx, hy):
    X, Y = np.meshgrid(0.5 * hx * (1 + _GX), 0.5 * hy * (1 + _GX), indexing="ij")
    W = np.outer(_GW, _GW) * 0.25 * hx * hy
    return X.ravel(), Y.ravel(), W.ravel()


def plane_operators(hx, hy, vx, vy):
    """Per-direction operators of the 2D sweep on a uniform mesh.

    Returns V [nv,4,4], Ex [nv,4,4], Ey [nv,4,4], bx [nv,4], by [nv,4]:
    Ex couples to the x-upwind neighbour (left if vx>0, right if vx<0), Ey to
    the y-upwind neighbour; bx / by are the loads of a unit isotropic inflow on
    the x- / y-inflow boundary edge of a boundary cell.
    """
    nv = len(vx)
    V = np.zeros((nv, 4, 4))
    Ex = np.zeros((nv, 4, 4))
    Ey = np.zeros((nv, 4, 4))
    bx = np.zeros((nv, 4))
    by = np.zeros((nv, 4))
    X, Y, W = _vol_points(hx, hy)
    val, gx, gy = _phi2d(0.0, 0.0, hx, hy, X, Y)
    ex = 0.5 * hx * (1 + _GX)    # points along a horizontal edge
    ey = 0.5 * hy * (1 + _GX)    # points along a vertical edge
    wx = 0.5 * hx * _GW
    wy = 0.5 * hy * _GW
    for j in range(nv):
        v = np.array([vx[j], vy[j]])
        # volume: - int (v . grad phi_k) phi_l
        V[j] -= np.einsum("kq,lq,q->kl", v[0] * gx + v[1] * gy, val, W)
        # four edges: (points x, points y, weights, outward normal, neighbour origin)
        edges = [
            (np.zeros_like(ey), ey, wy, (-1.0, 0.0), (-hx, 0.0)),   # left   x=0
            (np.full_like(ey, hx), ey, wy, (1.0, 0.0), (hx, 0.0)),  # right  x=hx
            (ex, np.zeros_like(ex), wx, (0.0, -1.0), (0.0, -hy)),   # bottom y=0
            (ex, np.full_like(ex, hy), wx, (0.0, 1.0), (0.0, hy)),  # top    y=hy
        ]
        for px, py, pw, n, org in edges:
            vn = v[0] * n[0] + v[1] * n[1]
            pc, _, _ = _phi2d(0.0, 0.0, hx, hy, px, py)
            if vn > 0:      # outflow: upwind value is the cell's own trace
                V[j] += vn * np.einsum("kq,lq,q->kl", pc, pc, pw)
            elif vn < 0:    # inflow: upwind value is the neighbour's trace
                pn, _, _ = _phi2d(org[0], org[1], hx, hy, px, py)
                M = vn * np.einsum("kq,lq,q->kl", pc, pn, pw)
                load = -vn * (pc @ pw)
                if n[0] != 0.0:
                    Ex[j] = M
                    bx[j] = load
                else:
                    Ey[j] = M
                    by[j] = load
    return V, Ex, Ey, bx, by


def plane_cell_load(hx, hy):
    """int phi_k over a cell for a unit constant -> [4]."""
    X, Y, W = _vol_points(hx, hy)
    val, _, _ = _phi2d(0.0, 0.0, hx, hy, X, Y)
    return val @ W


def plane_eval_cell(hx, hy, coef, xl, yl):
    """Evaluate one cell's DG function (coef [4]) at local points (xl, yl) in [0,hx]x[0,hy]."""
    val, _, _ = _phi2d(0.0, 0.0, hx, hy, xl, yl)
    return coef @ val


def plane_project(nx, ny, hx, hy, fun):
    """L2 projection of fun(x, y) onto the DG Q1 space -> [ny*nx, 4]."""
    X, Y, W = _vol_points(hx, hy)
    val, _, _ = _phi2d(0.0, 0.0, hx, hy, X, Y)
    out = np.zeros((ny * nx, 4))
    for jj in range(ny):
        for ii in range(nx):
            out[jj * nx + ii] = val @ (fun(ii * hx + X, jj * hy + Y) * W)
    return out


# ---------------------------------------------------------------------------
# Global sparse assembly of eq. (dg_matrix_vec) (small meshes: pins, brute force)
# ---------------------------------------------------------------------------
def plane_global_D(nx, ny, V, Ex, Ey, vx, vy):
    """Global D_j (sparse, N_DOF x N_DOF) for every direction: the cell's own
    block V_j and the coupling E_j to each interior upwind neighbour; inflow
    boundary edges contribute no matrix entry (their term is the load)."""
    out = []
    for j in range(len(vx)):
        rows, cols, vals = [], [], []
        for jj in range(ny):
            for ii in range(nx):
                c = jj * nx + ii
                blocks = [(c, V[j])]
                iu = ii - 1 if vx[j] > 0 else ii + 1
                if vx[j] != 0 and 0 <= iu < nx:
                    blocks.append((jj * nx + iu, Ex[j]))
                ju = jj - 1 if vy[j] > 0 else jj + 1
                if vy[j] != 0 and 0 <= ju < ny:
                    blocks.append((ju * nx + ii, Ey[j]))
                for cc, M in blocks:
                    for k in range(4):
                        for l in range(4):
                            rows.append(4 * c + k)
                            cols.append(4 * cc + l)
                            vals.append(M[k, l])
        out.append(sp.csr_matrix((vals, (rows, cols)), shape=(4 * nx * ny, 4 * nx * ny)))
    return out


def plane_bc_load(nx, ny, bx, by, vx, vy, g):
    """g_j^(bc) of eq. (dg_matrix_vec) for isotropic side values g = (x=0, x=L, y=0, y=L)
    -> [nv, N_DOF]."""
    nv = len(vx)
    out = np.zeros((nv, nx * ny, 4))
    for j in range(nv):
        if vx[j] > 0:
            out[j, np.arange(ny) * nx + 0] += g[0] * bx[j]
        elif vx[j] < 0:
            out[j, np.arange(ny) * nx + nx - 1] += g[1] * bx[j]
        if vy[j] > 0:
            out[j, np.arange(nx)] += g[2] * by[j]
        elif vy[j] < 0:
            out[j, (ny - 1) * nx + np.arange(nx)] += g[3] * by[j]
    return out.reshape(nv, -1)


def slab_global_D(edges, V, E, mu):
    """Global D_j (sparse) for the slab, as plane_global_D."""
    nc = len(edges) - 1
    out = []
    for j in range(len(mu)):
        rows, cols, vals = [], [], []
        for c in range(nc):
            blocks = [(c, V[j, c])]
            nb = c - 1 if mu[j] > 0 else c + 1
            if 0 <= nb < nc:
                blocks.append((nb, E[j, c]))
            for cc, M in blocks:
                for k in range(2):
                    for l in range(2):
                        rows.append(2 * c + k)
                        cols.append(2 * cc + l)
                        vals.append(M[k, l])
        out.append(sp.csr_matrix((vals, (rows, cols)), shape=(2 * nc, 2 * nc)))
    return out
