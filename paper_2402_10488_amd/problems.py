"""Upload problem descriptions (rte_workloads) to the device and wrap them as library handles."""
import numpy as np

from . import quadrature
from .rte import Problem


def _dev(a, device="cuda"):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device).contiguous()


def plane_problem(plane, device="cuda", dg=0, wpb=0, bands=0) -> Problem:
    """Problem handle for every instance of a 2D description (materials uploaded to ``device``)."""
    vx, vy, w = quadrature.plane_rule(plane.quad)
    return Problem(2, plane.nx, plane.ny, vx, w, _dev(plane.sigma_t, device), _dev(plane.sigma_s, device),
                   _dev(plane.G, device), _dev(plane.g, device), dirs_y=vy, lx=plane.Lx, ly=plane.Ly,
                   dg=dg, wpb=wpb, bands=bands)


def slab_problem(slabs, device="cuda") -> Problem:
    """Problem handle for a batch of slabs sharing cells and directions (cell-constant materials)."""
    if not isinstance(slabs, (list, tuple)):
        slabs = [slabs]
    s0 = slabs[0]
    for s in slabs:
        if not s.cell_constant:
            raise ValueError("the device library takes cell-constant materials")
        assert np.array_equal(s.edges, s0.edges) and s.quad == s0.quad
    kind, n = s0.quad
    assert kind == "gl"
    mu, w = quadrature.gauss_legendre(n)
    st = np.stack([s.sigma_t[:, 0] for s in slabs])[:, None, :]
    ss = np.stack([s.sigma_s[:, 0] for s in slabs])[:, None, :]
    G = np.stack([s.G[:, 0] for s in slabs])[:, None, :]
    g = np.array([[s.g_left, s.g_right, 0.0, 0.0] for s in slabs])
    return Problem(1, s0.nc, 1, mu, w, _dev(st, device), _dev(ss, device), _dev(G, device),
                   _dev(g, device), widths=np.diff(s0.edges))


def plane_psi(plane, device="cuda"):
    """Affine parameters of a block lattice: (sigma_t per block, sigma_s per block) [B, 2 nb]."""
    return _dev(np.concatenate([plane.block_sigma_t, plane.block_sigma_s], axis=1), device)
