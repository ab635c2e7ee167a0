"""Seeded synthetic inputs for the S_N upwind-DG transport problems.

This module only *describes* problems: meshes, per-cell material values,
isotropic sources, inflow values, quadrature names, parameter samples and
request streams.  It holds none of the method's arithmetic (no quadrature
nodes, no DG operators, no sweeps, no corrections), so both the CPU oracle
and the GPU library can take their inputs from here without sharing any
computation.

All randomness is numpy's PCG64 (``numpy.random.default_rng(seed)``); every
seed is part of the returned description.

Problem statement followed (paper Sec. 2, eq. (rte) and the slab form
eq. (slab_geometry)): sigma_t >= sigma_s >= 0, isotropic source G,
isotropic inflow g on the inflow part of the boundary.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Slab", "Plane", "slab_uniform", "c0_slab", "cross_regime", "two_material",
    "window_demo", "plane_uniform", "c1_checkerboard", "c2_lattice", "c2_batch",
    "c2_training", "c3_requests", "c4_multiscale", "c4_training", "random_plane",
    "homogeneous_medium", "lattice_medium", "pin_cell", "variable_scattering",
    "homogeneous_training", "homogeneous_test", "lattice_training", "lattice_test",
    "pin_cell_training", "pin_cell_test", "variable_scattering_training",
    "variable_scattering_test", "random_slab", "Request",
]


# ---------------------------------------------------------------------------
# 1D slab
# ---------------------------------------------------------------------------
@dataclass
class Slab:
    """1D slab problem (paper eq. (slab_geometry)).

    Materials are piecewise linear per cell: ``sigma_t[c] = (value at left
    edge, value at right edge)``; cell-constant problems repeat the value.
    ``g_left`` is the inflow for xi > 0 at x = edges[0]; ``g_right`` for
    xi < 0 at x = edges[-1].  ``quad`` names the angular rule.
    """
    edges: np.ndarray            # [nc+1]
    sigma_t: np.ndarray          # [nc, 2]
    sigma_s: np.ndarray          # [nc, 2]
    G: np.ndarray                # [nc, 2]
    g_left: float = 0.0
    g_right: float = 0.0
    quad: Tuple[str, int] = ("gl", 16)
    name: str = "slab"

    @property
    def nc(self) -> int:
        return len(self.edges) - 1

    @property
    def cell_constant(self) -> bool:
        return all(np.array_equal(a[:, 0], a[:, 1]) for a in (self.sigma_t, self.sigma_s, self.G))


def _pl(values_left, values_right=None):
    values_left = np.asarray(values_left, dtype=np.float64)
    if values_right is None:
        values_right = values_left
    return np.stack([values_left, np.asarray(values_right, dtype=np.float64)], axis=1)


def slab_uniform(nc: int, length: float, sigma_t: float, sigma_s: float, G: float,
                 g_left: float = 0.0, g_right: float = 0.0, n_dir: int = 16,
                 x0: float = 0.0, name: str = "slab") -> Slab:
    """Homogeneous slab on [x0, x0+length] with ``nc`` uniform cells."""
    edges = x0 + np.linspace(0.0, length, nc + 1)
    one = np.ones(nc)
    return Slab(edges, _pl(sigma_t * one), _pl(sigma_s * one), _pl(G * one),
                g_left, g_right, ("gl", n_dir), name)


def c0_slab() -> Slab:
    """Slab x in [0,1], 64 uniform cells, sigma_t=1, sigma_s=0.5, G=1, vacuum, 16 GL directions."""
    return slab_uniform(64, 1.0, 1.0, 0.5, 1.0, 0.0, 0.0, 16, name="c0_slab_64xS16")


def cross_regime(mu_s: float, nc: int = 400) -> Slab:
    """Paper Sec. 4.2.1 cross-regime problem: [0,10], G=0.01, sigma_a=0,
    sigma_s(x) = 0.1 + mu_s x (linear inside each cell), vacuum, S16."""
    edges = np.linspace(0.0, 10.0, nc + 1)
    sl = 0.1 + mu_s * edges[:-1]
    sr = 0.1 + mu_s * edges[1:]
    g = 0.01 * np.ones(nc)
    return Slab(edges, _pl(sl, sr), _pl(sl, sr), _pl(g), 0.0, 0.0, ("gl", 16),
                name=f"cross_regime_mu{mu_s:g}")


def cross_regime_training() -> List[float]:
    """Paper Sec. 4.2.1 training set: mu_s = 10 + j/4, j = 0..40."""
    return [10.0 + 0.25 * j for j in range(41)]


def two_material(mu_a: float, mu_s: float) -> Slab:
    """Paper Sec. 4.2.2 two-material problem on [0,11]: absorber (mu_a, 0) on [0,1]
    with dx=1/100, scatterer (0, mu_s) on [1,11] with dx=1/10, f(0,xi>0)=5, G=0."""
    e1 = np.linspace(0.0, 1.0, 101)
    e2 = np.linspace(1.0, 11.0, 101)[1:]
    edges = np.concatenate([e1, e2])
    nc = len(edges) - 1
    st = np.where(np.arange(nc) < 100, mu_a, mu_s).astype(np.float64)
    ss = np.where(np.arange(nc) < 100, 0.0, mu_s).astype(np.float64)
    return Slab(edges, _pl(st), _pl(ss), _pl(np.zeros(nc)), 5.0, 0.0, ("gl", 16),
                name=f"two_material_{mu_a:g}_{mu_s:g}")


def two_material_training() -> List[Tuple[float, float]]:
    """Paper Sec. 4.2.2 training set: mu_a = 0.5 + 0.1 m (m<=10), mu_s = 10 + n (n<=40)."""
    return [(0.5 + 0.1 * m, 10.0 + n) for m in range(11) for n in range(41)]


def window_demo() -> Slab:
    """Paper Sec. 3.2.1 window-size example: [0,10], G=0.01, sigma_t=sigma_s=1, 400 cells."""
    return slab_uniform(400, 10.0, 1.0, 1.0, 0.01, name="window_demo")


def random_slab(seed: int, nc: int = 12, n_dir: int = 8, nonuniform: bool = True) -> Slab:
    """Small random cell-constant slab for parity tests (ragged, non-uniform mesh)."""
    rng = np.random.default_rng(seed)
    if nonuniform:
        widths = rng.uniform(0.05, 0.3, nc)
    else:
        widths = np.full(nc, 1.0 / nc)
    edges = np.concatenate([[0.0], np.cumsum(widths)])
    ss = rng.uniform(0.0, 5.0, nc)
    sa = rng.uniform(0.05, 2.0, nc)
    G = rng.uniform(0.0, 2.0, nc)
    return Slab(edges, _pl(ss + sa), _pl(ss), _pl(G), float(rng.uniform(0, 1)),
                float(rng.uniform(0, 1)), ("gl", n_dir), name=f"random_slab_{seed}")


# ---------------------------------------------------------------------------
# 2D X-Y geometry on a uniform Cartesian mesh
# ---------------------------------------------------------------------------
@dataclass
class Plane:
    """2D problem on [0,Lx] x [0,Ly] with a uniform nx x ny mesh.

    Arrays carry a leading batch axis B (one entry per parametric instance):
    ``sigma_t``, ``sigma_s``, ``G`` are [B, ny, nx] cell-constant values;
    ``g`` is [B, 4] isotropic inflow on the sides (x=0, x=Lx, y=0, y=Ly).
    ``block`` maps every cell to a material block id ([ny, nx], shared by the
    batch) and ``block_sigma_t``/``block_sigma_s`` are the per-instance block
    values [B, nblocks] the cell arrays were filled from (affine parameters).
    ``quad = ("cheb", N_phi)`` is the normalized Chebyshev rule on the unit circle,
    ``("cl", (N_phi, N_vz))`` the Chebyshev-Legendre rule on the sphere.
    ``block_fields`` ([nblocks, ny, nx], optional) replaces the block indicators by cell fields:
    then sigma = sum_k block_sigma[:, k] * block_fields[k] (a medium affine in its parameters
    whose terms are not piecewise constant), and ``block`` is not a material map.
    """
    nx: int
    ny: int
    Lx: float
    Ly: float
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    G: np.ndarray
    g: np.ndarray
    block: np.ndarray
    block_sigma_t: np.ndarray
    block_sigma_s: np.ndarray
    quad: Tuple = ("cheb", 64)
    name: str = "plane"
    seeds: Tuple[int, ...] = field(default_factory=tuple)
    block_fields: Optional[np.ndarray] = None

    @property
    def B(self) -> int:
        return self.sigma_t.shape[0]

    @property
    def hx(self) -> float:
        return self.Lx / self.nx

    @property
    def hy(self) -> float:
        return self.Ly / self.ny

    def instance(self, b: int) -> "Plane":
        s = slice(b, b + 1)
        return Plane(self.nx, self.ny, self.Lx, self.Ly, self.sigma_t[s], self.sigma_s[s],
                     self.G[s], self.g[s], self.block, self.block_sigma_t[s],
                     self.block_sigma_s[s], self.quad, f"{self.name}[{b}]",
                     self.seeds[b:b + 1] if self.seeds else (), self.block_fields)

    def subset(self, idx: Sequence[int]) -> "Plane":
        idx = list(idx)
        return Plane(self.nx, self.ny, self.Lx, self.Ly, self.sigma_t[idx], self.sigma_s[idx],
                     self.G[idx], self.g[idx], self.block, self.block_sigma_t[idx],
                     self.block_sigma_s[idx], self.quad, self.name,
                     tuple(self.seeds[i] for i in idx) if self.seeds else (), self.block_fields)


def _checker_blocks(nx: int, ny: int, nbx: int, nby: int) -> np.ndarray:
    """Block id of every cell for an nbx x nby lattice of equal blocks."""
    bx = (np.arange(nx) * nbx) // nx
    by = (np.arange(ny) * nby) // ny
    return (by[:, None] * nbx + bx[None, :]).astype(np.int32)


def _fill(block: np.ndarray, per_block: np.ndarray) -> np.ndarray:
    """Cell array [B, ny, nx] from per-block values [B, nblocks]."""
    return per_block[:, block]


def plane_uniform(n: int, sigma_t: float, sigma_s: float, G: float, g: float = 0.0,
                  n_phi: int = 16, L: float = 1.0, B: int = 1, name: str = "plane") -> Plane:
    """Homogeneous square with isotropic inflow g on all four sides."""
    block = np.zeros((n, n), np.int32)
    bst = np.full((B, 1), sigma_t)
    bss = np.full((B, 1), sigma_s)
    Gc = np.full((B, n, n), G, dtype=np.float64)
    return Plane(n, n, L, L, _fill(block, bst), _fill(block, bss), Gc,
                 np.full((B, 4), g, dtype=np.float64), block, bst, bss, ("cheb", n_phi), name)


def _central_source(n: int, lo: float = 0.375, hi: float = 0.625) -> np.ndarray:
    """G = 1 on the cells whose centres lie in [lo, hi]^2 of the unit square."""
    xc = (np.arange(n) + 0.5) / n
    inside = (xc > lo) & (xc < hi)
    return (inside[:, None] & inside[None, :]).astype(np.float64)


def homogeneous_medium(mu_s: Sequence[float], n: int = 80, quad=("cl", (30, 6))) -> Plane:
    """Stand-in for the paper's homogeneous-medium family (Sec. 4.3.1): [0,1]^2, vacuum,
    sigma_a = 0, sigma_s = mu_s, G = exp(-100 |x - (0.5, 0.5)|^2) taken at the cell centres
    (the library uses cell-constant data), one instance per mu_s."""
    B = len(mu_s)
    block = np.zeros((n, n), np.int32)
    bss = np.asarray(mu_s, np.float64)[:, None]
    xc = (np.arange(n) + 0.5) / n
    Gc = np.exp(-100.0 * ((xc[None, :] - 0.5) ** 2 + (xc[:, None] - 0.5) ** 2))
    G = np.broadcast_to(Gc, (B, n, n)).copy()
    return Plane(n, n, 1.0, 1.0, _fill(block, bss), _fill(block, bss), G, np.zeros((B, 4)),
                 block, bss.copy(), bss.copy(), quad, f"homogeneous_{n}x{n}_B{B}")


def lattice_medium(params: Sequence[Tuple[float, float]], n: int = 50,
                   quad=("cl", (40, 6))) -> Plane:
    """Stand-in for the paper's lattice family (Sec. 4.3.2): [0,5]^2 split into 5 x 5 unit
    blocks; absorbing blocks (sigma_a, sigma_s) = (mu_a, 0) where bx + by is odd, scattering
    blocks (0, mu_s) elsewhere; G = 1 on the centre block |x - 2.5|, |y - 2.5| < 0.5; vacuum.
    (The paper's figure fixes its own absorber pattern; this checkerboard is the reading used.)"""
    B = len(params)
    block = _checker_blocks(n, n, 5, 5)
    absorb = np.array([((b % 5) + (b // 5)) % 2 == 1 for b in range(25)])
    mu_a = np.array([p[0] for p in params], np.float64)[:, None]
    mu_s = np.array([p[1] for p in params], np.float64)[:, None]
    bst = np.where(absorb[None, :], mu_a, mu_s)
    bss = np.where(absorb[None, :], 0.0, mu_s)
    Gb = np.zeros((B, 25))
    Gb[:, 12] = 1.0
    return Plane(n, n, 5.0, 5.0, _fill(block, bst), _fill(block, bss), _fill(block, Gb),
                 np.zeros((B, 4)), block, bst, bss, quad, f"lattice_{n}x{n}_B{B}")


def homogeneous_training() -> List[float]:
    """Sec. 4.3.1: mu_s = 0.9 + m / 200, m = 0..20."""
    return [0.9 + m / 200.0 for m in range(21)]


def homogeneous_test(n_test: int = 10, seed: int = 60000) -> List[float]:
    """Test draws mu_s ~ U[0.9, 1.1] (Sec. 4.3.1 samples 10; its values are not published)."""
    return [float(v) for v in np.random.default_rng(seed).uniform(0.9, 1.1, n_test)]


def lattice_training() -> List[Tuple[float, float]]:
    """Sec. 4.3.2: (mu_a, mu_s) = (95 + i, 0.5 + 0.1 j), i, j = 0..10 (121 pairs)."""
    return [(95.0 + i, 0.5 + 0.1 * j) for i in range(11) for j in range(11)]


def lattice_test(n_test: int = 10, seed: int = 60100) -> List[Tuple[float, float]]:
    """Test draws (mu_a, mu_s) ~ U[95, 105] x U[0.5, 1.5]."""
    r = np.random.default_rng(seed)
    return [(float(a), float(b)) for a, b in zip(r.uniform(95, 105, n_test), r.uniform(0.5, 1.5, n_test))]


def _centres(n: int, lo: float, hi: float) -> np.ndarray:
    return lo + (np.arange(n) + 0.5) * (hi - lo) / n


def pin_cell(params: Sequence[Tuple[float, float]], n: int = 80, quad=("cl", (30, 6))) -> Plane:
    """Stand-in for the paper's pin-cell family (Sec. 4.3.3) on [-1, 1]^2 (stored as [0, 2]^2),
    vacuum inflow: in the pin |x|, |y| <= 0.5 (cells whose centre lies there) sigma_a = mu_a,
    sigma_s = mu_s; outside sigma_a = 0, sigma_s = 100; G = exp(-100 (x^2 + y^2)) at the cell
    centres (the library takes cell-constant data).  Block 0 is the pin, block 1 the rest; one
    instance per (mu_a, mu_s)."""
    B = len(params)
    xc = _centres(n, -1.0, 1.0)
    inside = np.abs(xc) <= 0.5
    block = np.where(inside[:, None] & inside[None, :], 0, 1).astype(np.int32)
    mu_a = np.array([p[0] for p in params], np.float64)
    mu_s = np.array([p[1] for p in params], np.float64)
    bst = np.stack([mu_a + mu_s, np.full(B, 100.0)], axis=1)
    bss = np.stack([mu_s, np.full(B, 100.0)], axis=1)
    Gc = np.exp(-100.0 * (xc[None, :] ** 2 + xc[:, None] ** 2))
    G = np.broadcast_to(Gc, (B, n, n)).copy()
    return Plane(n, n, 2.0, 2.0, _fill(block, bst), _fill(block, bss), G, np.zeros((B, 4)),
                 block, bst, bss, quad, f"pin_cell_{n}x{n}_B{B}")


def pin_cell_training() -> List[Tuple[float, float]]:
    """Sec. 4.3.3: (mu_a, mu_s) = (0.05 i, 0.05 j), i, j = 1..5 (25 pairs)."""
    return [(0.05 * i, 0.05 * j) for i in range(1, 6) for j in range(1, 6)]


def pin_cell_test(n_test: int = 10, seed: int = 60200) -> List[Tuple[float, float]]:
    """Test draws (mu_a, mu_s) ~ U[0.05, 0.5]^2."""
    r = np.random.default_rng(seed)
    return [(float(a), float(b)) for a, b in zip(r.uniform(0.05, 0.5, n_test),
                                                 r.uniform(0.05, 0.5, n_test))]


def variable_scattering(mu_s: Sequence[float], n: int = 80, quad=("cl", (30, 6))) -> Plane:
    """Stand-in for the paper's variable-scattering family (Sec. 4.3.4) on [-1, 1]^2 (stored as
    [0, 2]^2), vacuum inflow, sigma_a = 0 and sigma_s = mu_s s(r) + 0.1 with
    s(r) = r^4 (2 - r^2)^2 for r <= 1 and 1 beyond, G = (10 / pi) exp(-100 r^2); s and G at the
    cell centres.  The medium is affine in mu_s with two cell fields, s and 1
    (block_fields), whose coefficients are (mu_s, 0.1) for sigma_t and for sigma_s."""
    B = len(mu_s)
    xc = _centres(n, -1.0, 1.0)
    r2 = xc[None, :] ** 2 + xc[:, None] ** 2
    r = np.sqrt(r2)
    shape = np.where(r <= 1.0, r2 ** 2 * (2.0 - r2) ** 2, 1.0)
    fields = np.stack([shape, np.ones((n, n))])
    coef = np.stack([np.asarray(mu_s, np.float64), np.full(B, 0.1)], axis=1)    # [B, 2]
    sig = np.einsum("bk,kyx->byx", coef, fields)
    G = np.broadcast_to((10.0 / np.pi) * np.exp(-100.0 * r2), (B, n, n)).copy()
    return Plane(n, n, 2.0, 2.0, sig, sig.copy(), G, np.zeros((B, 4)),
                 np.zeros((n, n), np.int32), coef, coef.copy(), quad,
                 f"variable_scattering_{n}x{n}_B{B}", (), fields)


def variable_scattering_training() -> List[float]:
    """Sec. 4.3.4: 50 uniformly spaced mu_s over [49.9, 99.9]."""
    return [float(v) for v in np.linspace(49.9, 99.9, 50)]


def variable_scattering_test(n_test: int = 10, seed: int = 60300) -> List[float]:
    """Test draws mu_s ~ U[49.9, 99.9]."""
    return [float(v) for v in np.random.default_rng(seed).uniform(49.9, 99.9, n_test)]


def c1_checkerboard(n: int = 128, n_phi: int = 64) -> Plane:
    """4x4 checkerboard on [0,1]^2: light blocks (bx+by even) sigma_s=1, sigma_a=0.01;
    dark blocks sigma_s=0, sigma_a=10; G=1 on [0.375,0.625]^2; vacuum inflow."""
    block = _checker_blocks(n, n, 4, 4)
    light = np.array([((b % 4) + (b // 4)) % 2 == 0 for b in range(16)])
    ss = np.where(light, 1.0, 0.0)
    sa = np.where(light, 0.01, 10.0)
    bst = (ss + sa)[None, :]
    bss = ss[None, :]
    G = _central_source(n)[None]
    return Plane(n, n, 1.0, 1.0, _fill(block, bst), _fill(block, bss), G,
                 np.zeros((1, 4)), block, bst, bss, ("cheb", n_phi),
                 f"c1_checkerboard_{n}x{n}_cheb{n_phi}")


def c2_lattice(seeds: Sequence[int], n: int = 128, n_phi: int = 64,
               left_inflow: bool = False, name: str = "c2_lattice") -> Plane:
    """4x4 block lattice with per-block sigma_s ~ U[0.5,50], sigma_a ~ U[0.001,1]
    (16 draws of sigma_s then 16 of sigma_a, per instance seed); G=1 on the
    central square, vacuum inflow (or g ~ U[0,1] on x=0 if ``left_inflow``,
    drawn after the materials)."""
    block = _checker_blocks(n, n, 4, 4)
    B = len(seeds)
    bss = np.empty((B, 16))
    bsa = np.empty((B, 16))
    g = np.zeros((B, 4))
    for k, s in enumerate(seeds):
        rng = np.random.default_rng(s)
        bss[k] = rng.uniform(0.5, 50.0, 16)
        bsa[k] = rng.uniform(0.001, 1.0, 16)
        if left_inflow:
            g[k, 0] = rng.uniform(0.0, 1.0)
    bst = bss + bsa
    G = np.broadcast_to(_central_source(n), (B, n, n)).copy()
    return Plane(n, n, 1.0, 1.0, _fill(block, bst), _fill(block, bss), G, g, block,
                 bst, bss, ("cheb", n_phi), f"{name}_{n}x{n}_cheb{n_phi}_B{B}", tuple(seeds))


def c2_batch(B: int = 256, n: int = 128, n_phi: int = 64) -> Plane:
    """Test instances of the batched parametric lattice: seeds 20000+i."""
    return c2_lattice([20000 + i for i in range(B)], n, n_phi, name="c2_test")


def c2_training(N: int = 32, n: int = 128, n_phi: int = 64) -> Plane:
    """Training instances of the batched parametric lattice: seeds 30000+i."""
    return c2_lattice([30000 + i for i in range(N)], n, n_phi, name="c2_train")


@dataclass
class Request:
    """One parametric solve request of the serving stream."""
    rid: int
    arrival: float       # seconds after stream start
    n: int               # mesh is n x n
    n_phi: int           # directions on the unit circle
    seed: int            # material / inflow seed (c2_lattice with left inflow)


def c3_requests(n_req: int = 10000, rate: float = 1000.0, arrival_seed: int = 40000,
                draw_seed: int = 40001) -> List[Request]:
    """Serving stream: Poisson arrivals at ``rate`` requests/s; mesh uniform in
    {64,128,256}^2, directions uniform in {32,64,128}; each request's lattice
    and left inflow come from c2_lattice(seed, left_inflow=True)."""
    ra = np.random.default_rng(arrival_seed)
    rd = np.random.default_rng(draw_seed)
    t = np.cumsum(ra.exponential(1.0 / rate, n_req))
    ns = rd.choice([64, 128, 256], n_req)
    nphis = rd.choice([32, 64, 128], n_req)
    seeds = rd.integers(1, 2**31 - 1, n_req)
    return [Request(i, float(t[i]), int(ns[i]), int(nphis[i]), int(seeds[i])) for i in range(n_req)]


def c3_training(n: int, n_phi: int, N: int = 32) -> Plane:
    """Training set of one (mesh, directions) class of the serving stream."""
    key = {64: 0, 128: 1, 256: 2}[n] * 3 + {32: 0, 64: 1, 128: 2}[n_phi]
    return c2_lattice([41000 + key * 100 + i for i in range(N)], n, n_phi, left_inflow=True,
                      name="c3_train")


def c4_multiscale(n: int = 512, n_phi: int = 256, eps: float = 1e-3,
                  ss_thin: float = 1.0, sa_thin: float = 0.1, nb: int = 16) -> Plane:
    """16x16 checkerboard of (n/16)^2-cell blocks on [0,1]^2: thick blocks
    (bx+by even) sigma_s=1/eps, sigma_a=eps; thin blocks sigma_s=ss_thin,
    sigma_a=sa_thin and G=1; vacuum inflow.  The material map has two materials
    (0 thick, 1 thin), so the affine parameters are the two materials' values."""
    lattice = _checker_blocks(n, n, nb, nb)
    material = (((lattice % nb) + (lattice // nb)) % 2).astype(np.int32)
    ss = np.array([1.0 / eps, ss_thin])
    sa = np.array([eps, sa_thin])
    bst = (ss + sa)[None, :]
    bss = ss[None, :]
    Gb = np.array([[0.0, 1.0]])
    return Plane(n, n, 1.0, 1.0, _fill(material, bst), _fill(material, bss), _fill(material, Gb),
                 np.zeros((1, 4)), material, bst, bss, ("cheb", n_phi),
                 f"c4_multiscale_{n}x{n}_cheb{n_phi}")


def stack(planes: Sequence[Plane], name: str = None) -> Plane:
    """One batch from instances that share mesh, directions and material map."""
    p0 = planes[0]
    for p in planes:
        assert (p.nx, p.ny, p.Lx, p.Ly, p.quad) == (p0.nx, p0.ny, p0.Lx, p0.Ly, p0.quad)
        assert np.array_equal(p.block, p0.block)
    cat = lambda a: np.concatenate([getattr(p, a) for p in planes], axis=0)
    seeds = tuple(s for p in planes for s in p.seeds)
    return Plane(p0.nx, p0.ny, p0.Lx, p0.Ly, cat("sigma_t"), cat("sigma_s"), cat("G"), cat("g"),
                 p0.block, cat("block_sigma_t"), cat("block_sigma_s"), p0.quad,
                 name or p0.name, seeds, p0.block_fields)


def c4_training(N: int = 64, n: int = 512, n_phi: int = 256) -> Plane:
    """Training draws, one batch: eps ~ logU[5e-4, 2e-3], thin sigma_s ~ U[0.8,1.2],
    thin sigma_a ~ U[0.08,0.12]."""
    out = []
    for i in range(N):
        rng = np.random.default_rng(50000 + i)
        eps = float(np.exp(rng.uniform(np.log(5e-4), np.log(2e-3))))
        out.append(c4_multiscale(n, n_phi, eps, float(rng.uniform(0.8, 1.2)),
                                 float(rng.uniform(0.08, 0.12))))
    return stack(out, name=f"c4_train_{n}x{n}_cheb{n_phi}")


def random_plane(seed: int, nx: int = 13, ny: int = 9, n_phi: int = 8, B: int = 1,
                 nbx: int = 3, nby: int = 2, inflow: bool = True, Lx: float = 1.0,
                 Ly: float = 0.8) -> Plane:
    """Small random block-constant problem with ragged sizes for parity tests."""
    rng = np.random.default_rng(seed)
    block = _checker_blocks(nx, ny, nbx, nby)
    nb = nbx * nby
    bss = rng.uniform(0.0, 20.0, (B, nb))
    bsa = rng.uniform(0.05, 2.0, (B, nb))
    bst = bss + bsa
    G = rng.uniform(0.0, 1.0, (B, ny, nx))
    g = rng.uniform(0.0, 1.0, (B, 4)) if inflow else np.zeros((B, 4))
    return Plane(nx, ny, Lx, Ly, _fill(block, bst), _fill(block, bss), G, g, block, bst, bss,
                 ("cheb", n_phi), f"random_plane_{seed}", tuple([seed] * B))
