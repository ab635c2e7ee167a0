"""Oracle: brute-force global solves of eq. (one_equation) (paper Sec. 2.2) and the
ideal kinetic correction of eq. (one_equation_correction) (Sec. 2.3).

Test infrastructure only -- never imported by the product path.  Tiny meshes only.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class BruteForce:
    def __init__(self, disc):
        self.disc = disc
        Ds = disc.global_D()
        St, Ss = disc.sigma_blocks()
        nv = disc.nv
        w = disc.w
        blocks = [[None] * nv for _ in range(nv)]
        for j in range(nv):
            for k in range(nv):
                M = -w[k] * Ss
                if j == k:
                    M = Ds[j] + St + M
                blocks[j][k] = M
        self.A = sp.bmat(blocks).tocsc()
        self.lu = spla.splu(self.A)
        self.b = (disc.Gvec()[None, :] + disc.bc_load()).reshape(-1)

    def solve(self):
        """Exact discrete solution: (f [nv, N_DOF], rho = sum_j w_j f_j)."""
        f = self.lu.solve(self.b).reshape(self.disc.nv, -1)
        return f, self.disc.w @ f

    def correction(self, rho_star, rho_prev):
        """Ideal correction: solve A delta f = delta b, delta b = repeat(Sigma_s (rho^* - rho))."""
        src = self.disc.apply_Ss(rho_star - rho_prev).reshape(-1)
        db = np.tile(src, self.disc.nv)
        df = self.lu.solve(db).reshape(self.disc.nv, -1)
        return self.disc.w @ df
