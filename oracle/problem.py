"""Oracle: discretized single-instance problems (paper Sec. 2.1-2.2).

Test infrastructure only -- never imported by the product path.

``SlabDisc`` / ``PlaneDisc`` hold the S_N upwind-DG discretization of one
problem instance in the notation of eq. (dg_matrix_vec): direction set
{(v_j, w_j)}, local operators of D_j, the diagonal blocks of Sigma_t and
Sigma_s, the load G and the inflow loads g_j^(bc).  ``sweep(rho)`` applies
eq. (transport_sweep) for all directions and returns
rho^* = sum_j w_j f_j (and optionally f).
"""
import numpy as np

from . import dg, quadrature, sweep as csweep


class SlabDisc:
    """Slab, P1 upwind DG, normalized Gauss-Legendre directions (Sec. 4.2)."""
    dim = 1

    def __init__(self, slab, quad=None):
        kind, n = quad or slab.quad
        assert kind == "gl"
        self.slab = slab
        self.edges = np.asarray(slab.edges, dtype=np.float64)
        self.nc = len(self.edges) - 1
        self.ndof = 2 * self.nc
        self.mu, self.w = quadrature.gauss_legendre(n)
        self.nv = len(self.mu)
        self.V, self.E, self.bl = dg.slab_operators(self.edges, self.mu)
        self.St = dg.slab_mass_weighted(self.edges, slab.sigma_t)     # [nc,2,2]
        self.Ss = dg.slab_mass_weighted(self.edges, slab.sigma_s)
        self.Sa = self.St - self.Ss
        self.K = self.V + self.St[None]
        self.G = dg.slab_load(self.edges, slab.G)                     # [nc,2]
        self.g_left, self.g_right = slab.g_left, slab.g_right

    # Sigma applied blockwise to a coefficient vector [nc,2]
    def apply_Ss(self, rho):
        return np.einsum("ckl,cl->ck", self.Ss, rho.reshape(self.nc, 2))

    def apply_St(self, rho):
        return np.einsum("ckl,cl->ck", self.St, rho.reshape(self.nc, 2))

    def sweep(self, rho, src=None, q=None, zero_bc=False, want_f=False):
        """One transport sweep with source Sigma_s rho + G (or an explicit ``src``)."""
        if src is None:
            src = self.apply_Ss(rho) + self.G
        gl, gr = (0.0, 0.0) if zero_bc else (self.g_left, self.g_right)
        r, f = csweep.sweep1d(self.mu, self.w, self.K, self.E, self.bl, src.reshape(self.nc, 2),
                              gl, gr, q=q, want_f=want_f)
        return r.reshape(-1), (None if f is None else f.reshape(self.nv, -1))

    def apply_D(self, x):
        """D_j x_j for x [nv, N_DOF]."""
        return csweep.apply_D1d(self.mu, self.V, self.E, x.reshape(self.nv, self.nc, 2)).reshape(self.nv, -1)

    def bc_load(self):
        """g_j^(bc) for every direction -> [nv, N_DOF]."""
        out = np.zeros((self.nv, self.nc, 2))
        for j, m in enumerate(self.mu):
            if m > 0:
                out[j, 0] += self.g_left * self.bl[j]
            else:
                out[j, -1] += self.g_right * self.bl[j]
        return out.reshape(self.nv, -1)

    def global_D(self):
        return dg.slab_global_D(self.edges, self.V, self.E, self.mu)

    def sigma_blocks(self):
        """Sigma_t and Sigma_s as sparse block-diagonal N_DOF x N_DOF matrices."""
        import scipy.sparse as sp
        return sp.block_diag(list(self.St)).tocsr(), sp.block_diag(list(self.Ss)).tocsr()

    def Gvec(self):
        return self.G.reshape(-1)


class PlaneDisc:
    """One instance of a 2D problem: Q1 upwind DG on a uniform mesh,
    normalized Chebyshev rule on the unit circle (Sec. 2.1)."""
    dim = 2

    def __init__(self, plane, b: int = 0, quad=None, dirs=None):
        kind, n = quad or plane.quad
        self.plane = plane
        self.nx, self.ny = plane.nx, plane.ny
        self.hx, self.hy = plane.hx, plane.hy
        self.nc = self.nx * self.ny
        self.ndof = 4 * self.nc
        if dirs is not None:
            self.vx, self.vy, self.w = (np.asarray(a, dtype=np.float64) for a in dirs)
        elif kind == "cheb":
            self.vx, self.vy, self.w = quadrature.chebyshev_circle(n)
        elif kind == "cl":
            # CL(N_phi, N_vz) on the sphere (Sec. 2.1); X-Y geometry sees (vx, vy) only
            self.vx, self.vy, _, self.w = quadrature.chebyshev_legendre(*n)
        else:
            raise ValueError(kind)
        self.nv = len(self.vx)
        self.V, self.Ex, self.Ey, self.bx, self.by = dg.plane_operators(self.hx, self.hy, self.vx, self.vy)
        M = np.zeros((4, 4))
        # cell mass matrix int phi_k phi_l (identity for the orthonormal basis, computed)
        X, Y, W = dg._vol_points(self.hx, self.hy)
        val, _, _ = dg._phi2d(0.0, 0.0, self.hx, self.hy, X, Y)
        M = np.einsum("kq,lq,q->kl", val, val, W)
        self.mass = M
        self.sigma_t = plane.sigma_t[b].reshape(-1).astype(np.float64)
        self.sigma_s = plane.sigma_s[b].reshape(-1).astype(np.float64)
        self.sigma_a = self.sigma_t - self.sigma_s
        load = dg.plane_cell_load(self.hx, self.hy)
        self.G = plane.G[b].reshape(-1)[:, None] * load[None, :]        # [nc,4]
        self.g = np.asarray(plane.g[b], dtype=np.float64)
        self.block = plane.block.reshape(-1)
        self.block_fields = getattr(plane, "block_fields", None)
        self.block_sigma_t = plane.block_sigma_t[b]
        self.block_sigma_s = plane.block_sigma_s[b]
        # the sweep's local matrix is V_j + sigma_t * mass; the C code adds sigma_t on the
        # diagonal, which requires the computed mass matrix to be the identity.
        assert np.allclose(M, np.eye(4), atol=1e-14)

    def apply_Ss(self, rho):
        return self.sigma_s[:, None] * rho.reshape(self.nc, 4)

    def apply_St(self, rho):
        return self.sigma_t[:, None] * rho.reshape(self.nc, 4)

    def sweep(self, rho, src=None, q=None, zero_bc=False, want_f=False):
        if src is None:
            src = self.apply_Ss(rho) + self.G
        g = np.zeros(4) if zero_bc else self.g
        r, f = csweep.sweep2d(self.nx, self.ny, self.vx, self.vy, self.w, self.V, self.Ex, self.Ey,
                              self.bx, self.by, self.sigma_t, src.reshape(self.nc, 4), g, q=q,
                              want_f=want_f)
        return r.reshape(-1), (None if f is None else f.reshape(self.nv, -1))

    def apply_D(self, x):
        return csweep.apply_D2d(self.nx, self.ny, self.vx, self.vy, self.V, self.Ex, self.Ey,
                                x.reshape(self.nv, self.nc, 4)).reshape(self.nv, -1)

    def bc_load(self):
        return dg.plane_bc_load(self.nx, self.ny, self.bx, self.by, self.vx, self.vy, self.g)

    def global_D(self):
        return dg.plane_global_D(self.nx, self.ny, self.V, self.Ex, self.Ey, self.vx, self.vy)

    def sigma_blocks(self):
        import scipy.sparse as sp
        return (sp.diags(np.repeat(self.sigma_t, 4)).tocsr(), sp.diags(np.repeat(self.sigma_s, 4)).tocsr())

    def Gvec(self):
        return self.G.reshape(-1)


def discretize(problem, b: int = 0, **kw):
    """SlabDisc for a slab description, PlaneDisc for instance ``b`` of a plane description."""
    if hasattr(problem, "edges"):
        return SlabDisc(problem, **kw)
    return PlaneDisc(problem, b, **kw)
