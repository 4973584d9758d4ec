"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs (permittivity maps, source placements, partition
lists, quad-tree core lists); it holds none of the method's arithmetic, so both the HIP path and the
CPU oracle can take their inputs from it.  Each generator uses
``numpy.random.default_rng(seed)`` with a fixed draw order.

The paper trains and tests on Gaussian-random-field and Voronoi permittivity
maps in [1, 8] with line sources (Methods, training data generation); those
datasets are not available, so these stand-ins keep the shapes, contrast and
structure of the benchmark problems instead: piecewise-constant blocks and
rectangles of permittivity in [1, 12], point sources, a PML on every side.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

H = 0.05          # cell size in wavelength units (20 cells per vacuum wavelength at lambda = 1)
NPML = 12
PML_M = 2
PML_LNR = -30.0


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    eps: np.ndarray                  # [ny][nx] float32
    wavelengths: list
    sources: list                    # list of (ix, iy)
    core_x: list
    core_y: list
    overlap: int = 8
    k_coarse: int = 0
    k_trial: int = 8
    h: float = H
    npml: int = NPML
    pml_m: int = PML_M
    pml_lnR: float = PML_LNR
    notes: dict = field(default_factory=dict)
    cores: list = None               # explicit cores (cx0, cx1, cy0, cy1); overrides core_x / core_y

    def J(self):
        """Current density [n_src][ny][nx] complex64, one unit cell per source."""
        J = np.zeros((len(self.sources), self.ny, self.nx), dtype=np.complex64)
        for s, (ix, iy) in enumerate(self.sources):
            J[s, iy, ix] = 1.0
        return J


def small_rectangles(seed=1):
    """128 x 128, eps = 1 plus 6 rectangles in [2, 12], 2 x 2 cores of 64, 1 wavelength."""
    rng = np.random.default_rng(seed)
    n = 128
    eps = np.ones((n, n), dtype=np.float64)
    for _ in range(6):
        w, hh = rng.integers(4, 25, 2)
        x0 = rng.integers(14, n - 14 - w + 1)
        y0 = rng.integers(14, n - 14 - hh + 1)
        val = rng.uniform(2, 12)
        eps[y0:y0 + hh, x0:x0 + w] = val
    return Workload("rect128_2x2_lu", n, n, eps.astype(np.float32), [1.0], [(n // 2, n // 2)],
                    [64, 64], [64, 64])


def block_eps(rng, nx, ny, block):
    vals = rng.uniform(1, 12, (ny // block, nx // block))
    return np.kron(vals, np.ones((block, block)))


def blocks_512(seed=2):
    """512 x 512, 16-cell blocks in [1, 12], 8 x 8 cores of 64, 4 wavelengths, one coarse basis each."""
    rng = np.random.default_rng(seed)
    n = 512
    eps = block_eps(rng, n, n, 16)
    return Workload("blocks512_8x8_4wl_2level", n, n, eps.astype(np.float32), [0.8, 1.0, 1.2, 1.5],
                    [(n // 2, n // 2)], [64] * 8, [64] * 8, k_coarse=1)


def blocks_1024(seed=3):
    """1024 x 1024, 64-cell blocks in [1, 12], 16 x 16 cores of 64, wavelength 1."""
    rng = np.random.default_rng(seed)
    n = 1024
    eps = block_eps(rng, n, n, 64)
    return Workload("blocks1024_16x16", n, n, eps.astype(np.float32), [1.0],
                    [(n // 2, n // 2)], [64] * 16, [64] * 16, k_coarse=1)


def uneven_2048x1536(seed=4, n_src=32):
    """2048 x 1536, 16-cell blocks, mixed 64/96 cores, 32 sources x 2 wavelengths."""
    rng = np.random.default_rng(seed)
    nx, ny = 2048, 1536
    eps = block_eps(rng, nx, ny, 16)
    src = []
    for _ in range(n_src):
        ix = int(rng.integers(20, 2028))
        iy = int(rng.integers(20, 1516))
        src.append((ix, iy))
    return Workload("uneven2048x1536_64rhs", nx, ny, eps.astype(np.float32), [1.0, 1.2], src,
                    [96] + [64] * 29 + [96], [96] + [64] * 21 + [96])


@dataclass
class DesignWorkload:
    """Inverse-design problem: FoM = sum of |E|^2 at focal cells over wavelengths."""
    name: str
    nx: int
    ny: int
    eps: np.ndarray                  # [ny][nx] float32 (design region drawn, background 1)
    wavelengths: list
    line: tuple                      # (row, x0, x1): unit line current J = 1 on [x0, x1) of that row
    focal: list                      # list of (ix, iy)
    design: tuple                    # (x0, x1, y0, y1)
    core_x: list
    core_y: list
    overlap: int = 8
    k_coarse: int = 1
    h: float = H
    npml: int = NPML

    def J(self):
        J = np.zeros((1, self.ny, self.nx), dtype=np.complex64)
        row, x0, x1 = self.line
        J[0, row, x0:x1] = 1.0
        return J


def inverse_design_1024(seed=5):
    """1024 x 1024, 256 x 256 design region at [384, 640)^2 with eps uniform in [1, 12],
    wavelengths {0.9, 1.1, 1.3}, unit line source on row 320 across the design
    columns, three focal cells in rows [704, 896) above it; 16 x 16 cores of 64."""
    rng = np.random.default_rng(seed)
    n = 1024
    eps = np.ones((n, n), dtype=np.float32)
    eps[384:640, 384:640] = rng.uniform(1, 12, (256, 256)).astype(np.float32)
    focal = [(int(rng.integers(384, 640)), int(rng.integers(704, 896))) for _ in range(3)]
    return DesignWorkload("design1024_16x16_3wl", n, n, eps, [0.9, 1.1, 1.3], (320, 384, 640), focal,
                          (384, 640, 384, 640), [64] * 16, [64] * 16)


def random_small(seed, nx, ny, core_x, core_y, wavelengths=(1.0,), n_src=1, k_coarse=0,
                 overlap=8, npml=NPML, block=8):
    """Small random test problem: blocks of eps in [1, 12], random source cells."""
    rng = np.random.default_rng(seed)
    eps = np.kron(rng.uniform(1, 12, (ny // block, nx // block)), np.ones((block, block)))
    src = [(int(rng.integers(npml + 2, nx - npml - 2)), int(rng.integers(npml + 2, ny - npml - 2)))
           for _ in range(n_src)]
    return Workload(f"random{nx}x{ny}_s{seed}", nx, ny, eps.astype(np.float32), list(wavelengths), src,
                    list(core_x), list(core_y), overlap=overlap, k_coarse=k_coarse, npml=npml)


def _even_half(n):
    return 2 * (n // 4)


def quadtree_cores(nx, ny, eps, h, wavelength, max_size=5.0, min_core=16, max_core=64):
    """Quad-tree partition of the grid (Methods, partitioner: a quadrant larger
    than a threshold of about five wavelengths is decomposed into four).

    The size of a quadrant is measured in local wavelengths, wavelength /
    sqrt(max eps over the quadrant) with h per cell, so high-index regions are
    refined further.  A quadrant is split while its longer side exceeds
    max_size local wavelengths or max_core cells; it is split into four, or
    into two along its longer side when the other side cannot be halved, as
    long as every half keeps at least min_core cells.  Split points are even,
    so even grids give even cores.  Returns the cores (cx0, cx1, cy0, cy1),
    half-open, depth-first (lower-left, lower-right, upper-left, upper-right).
    """
    eps = np.asarray(eps)
    out = []

    def rec(x0, x1, y0, y1):
        wx, wy = x1 - x0, y1 - y0
        lam = wavelength / np.sqrt(float(eps[y0:y1, x0:x1].max()))
        big = max(wx, wy) > max_core or max(wx, wy) * h > max_size * lam
        hx, hy = _even_half(wx), _even_half(wy)
        can_x = min(hx, wx - hx) >= min_core
        can_y = min(hy, wy - hy) >= min_core
        if not big or not (can_x or can_y):
            out.append((x0, x1, y0, y1))
            return
        xs = [(x0, x0 + hx), (x0 + hx, x1)] if can_x else [(x0, x1)]
        ys = [(y0, y0 + hy), (y0 + hy, y1)] if can_y else [(y0, y1)]
        for (a0, a1) in ys:
            for (b0, b1) in xs:
                rec(b0, b1, a0, a1)

    rec(0, nx, 0, ny)
    return out


def quadtree_512(seed=6):
    """512 x 512, vacuum with a central 256 x 256 region of 16-cell blocks of
    eps in [1, 8], 2 wavelengths {1.0, 1.2}, centre source, one coarse basis
    per subdomain; quad-tree cores for the shorter wavelength: 64-cell cores
    in vacuum, 32-cell cores over the high-index region."""
    rng = np.random.default_rng(seed)
    n = 512
    eps = np.ones((n, n))
    eps[128:384, 128:384] = np.kron(rng.uniform(1, 8, (16, 16)), np.ones((16, 16)))
    cores = quadtree_cores(n, n, eps, H, 1.0)
    return Workload("quadtree512_2wl_2level", n, n, eps.astype(np.float32), [1.0, 1.2], [(n // 2, n // 2)],
                    [], [], k_coarse=1, cores=cores)


def random_quadtree(seed, n=192, wavelengths=(1.0,), n_src=1, k_coarse=0, npml=NPML, hot=(48, 96, 48, 96)):
    """Small quad-tree test problem: vacuum (eps 1.5) with one block of eps in
    [6, 8] over hot = (x0, x1, y0, y1); the quad-tree refines the quadrant
    that holds it (48-cell cores, 24-cell cores inside), which leaves
    T-junctions between the refined quadrant and its neighbours."""
    rng = np.random.default_rng(seed)
    eps = np.full((n, n), 1.5)
    x0, x1, y0, y1 = hot
    eps[y0:y1, x0:x1] = np.kron(rng.uniform(6, 8, ((y1 - y0) // 8, (x1 - x0) // 8)), np.ones((8, 8)))
    cores = quadtree_cores(n, n, eps, H, min(wavelengths), min_core=max(16, npml + 4), max_core=48)
    src = [(int(rng.integers(npml + 2, n - npml - 2)), int(rng.integers(npml + 2, n - npml - 2)))
           for _ in range(n_src)]
    return Workload(f"quadtree{n}_s{seed}", n, n, eps.astype(np.float32), list(wavelengths), src, [], [],
                    k_coarse=k_coarse, npml=npml, cores=cores)


WORKLOADS = {
    "rect128": small_rectangles,
    "blocks512": blocks_512,
    "blocks1024": blocks_1024,
    "uneven2048": uneven_2048x1536,
    "quadtree512": quadtree_512,
}
