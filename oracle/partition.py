"""Overlapping rectangular partition, local Robin problems and one-level Schwarz.

Oracle, test infrastructure only.  Follows the "partitioner" abstraction of the
Methods section (two-level Schwarz subsection) and the subdomain boundary value
problem of Eq. 2.

Partition reading: the cores tile the grid, either as the tensor product of
the lists ``core_x`` and ``core_y`` or as any list of rectangles that covers
every cell exactly once (``Partition.from_cores``: the partitioner abstraction
allows arbitrary arrangements, e.g. a quad-tree, as long as the subdomains
cover the domain); each core is extended by ``ext = overlap // 2`` cells on
every side that is not on the global boundary ("interface sides"), so
neighbouring subdomains share ``overlap`` cells.  The restricted (RAS)
prolongation writes core cells only; the cores form a partition of unity.

Robin transmission (Eq. 2 with the exp(+i omega t) convention, outward normal
n, outgoing-absorbing sign):  g = du/dn + i kappa u,  kappa = k0 sqrt(eps).
Discretised at the midpoint between an interface boundary node p and its ghost
q just outside the subdomain:

    g_p(u) = (u_q - u_p)/h + i kappa_p (u_q + u_p)/2,
    =>  u_q = rho_p u_p + tau_p g_p,
        rho_p = (1 - i kappa_p h/2)/(1 + i kappa_p h/2),  tau_p = h/(1 + i kappa_p h/2).

Eliminating the ghost from row p of A (coupling a_pq) gives the local matrix
B_i (diagonal += a_pq rho_p) and the Robin data injection inj(g)_p = -a_pq tau_p g_p.
Identity used as a pin:  B_i R_i u = R_i A u + inj(g(u))  for every u.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

SIDES = ("bottom", "right", "top", "left")


@dataclass
class Tile:
    tx: int
    ty: int
    cx0: int
    cx1: int
    cy0: int
    cy1: int
    x0: int
    x1: int
    y0: int
    y1: int
    iface: dict = field(default_factory=dict)   # side -> bool (interface side?)

    @property
    def lx(self):
        return self.x1 - self.x0

    @property
    def ly(self):
        return self.y1 - self.y0

    def contains(self, ix, iy):
        return self.x0 <= ix < self.x1 and self.y0 <= iy < self.y1

    def local_index(self, ix, iy):
        return (iy - self.y0) * self.lx + (ix - self.x0)

    def global_indices(self, nx):
        ys, xs = np.meshgrid(np.arange(self.y0, self.y1), np.arange(self.x0, self.x1), indexing="ij")
        return (ys * nx + xs).ravel()

    def core_mask_local(self):
        ys, xs = np.meshgrid(np.arange(self.y0, self.y1), np.arange(self.x0, self.x1), indexing="ij")
        m = (xs >= self.cx0) & (xs < self.cx1) & (ys >= self.cy0) & (ys < self.cy1)
        return m.ravel()


class PartitionError(ValueError):
    pass


class Partition:
    """Overlapping extended subdomains over rectangular cores.

    Tensor form (``core_x``, ``core_y``): tile index = ty*ncx + tx.  General
    form (``from_cores``): tiles in the order of the core list, tx = ty = -1.
    """

    def __init__(self, nx, ny, core_x, core_y, overlap, npml=0):
        core_x = [int(c) for c in core_x]
        core_y = [int(c) for c in core_y]
        if sum(core_x) != nx or sum(core_y) != ny:
            raise PartitionError("core sizes must sum to the grid size")
        if min(core_x + core_y) <= 0:
            raise PartitionError("core sizes must be positive")
        xb = np.concatenate([[0], np.cumsum(core_x)])
        yb = np.concatenate([[0], np.cumsum(core_y)])
        cores = [(int(xb[tx]), int(xb[tx + 1]), int(yb[ty]), int(yb[ty + 1]))
                 for ty in range(len(core_y)) for tx in range(len(core_x))]
        self.ncx, self.ncy = len(core_x), len(core_y)
        self._build(nx, ny, cores, overlap, npml)
        for k, t in enumerate(self.tiles):
            t.ty, t.tx = divmod(k, self.ncx)

    @classmethod
    def from_cores(cls, nx, ny, cores, overlap, npml=0):
        """Partition from an explicit list of cores (cx0, cx1, cy0, cy1), half-open."""
        self = cls.__new__(cls)
        self.ncx = self.ncy = None
        self._build(nx, ny, [tuple(int(v) for v in c) for c in cores], overlap, npml)
        return self

    def _build(self, nx, ny, cores, overlap, npml):
        if overlap < 2 or overlap % 2:
            raise PartitionError("overlap must be even and >= 2")
        if not cores:
            raise PartitionError("empty partition")
        ext = overlap // 2
        owner = -np.ones((ny, nx), dtype=np.int64)
        for k, (cx0, cx1, cy0, cy1) in enumerate(cores):
            if not (0 <= cx0 < cx1 <= nx and 0 <= cy0 < cy1 <= ny):
                raise PartitionError("a core is empty or leaves the grid")
            if np.any(owner[cy0:cy1, cx0:cx1] >= 0):
                raise PartitionError("cores overlap")
            owner[cy0:cy1, cx0:cx1] = k
        if np.any(owner < 0):
            raise PartitionError("cores do not cover the grid")
        if len(cores) > 1 and ext + 1 > min(min(c[1] - c[0], c[3] - c[2]) for c in cores):
            raise PartitionError("ext + 1 must not exceed the smallest core")
        self.nx, self.ny, self.ext, self.npml = nx, ny, ext, npml
        self.owner = owner
        self.tiles = []
        for (cx0, cx1, cy0, cy1) in cores:
            iface = {"left": cx0 > 0, "right": cx1 < nx, "bottom": cy0 > 0, "top": cy1 < ny}
            x0 = cx0 - ext if iface["left"] else cx0
            x1 = cx1 + ext if iface["right"] else cx1
            y0 = cy0 - ext if iface["bottom"] else cy0
            y1 = cy1 + ext if iface["top"] else cy1
            t = Tile(-1, -1, cx0, cx1, cy0, cy1, x0, x1, y0, y1, iface)
            self._validate_tile(t)
            self.tiles.append(t)

    def _validate_tile(self, t):
        """No interface may sit inside the PML of its normal direction."""
        n, m = self.npml, self.npml
        for side, on in t.iface.items():
            if not on:
                continue
            if side in ("left", "right"):
                xb = t.x0 if side == "left" else t.x1 - 1
                if xb < n or xb > self.nx - m - 1:
                    raise PartitionError(f"interface x={xb} lies in the x-PML")
            else:
                yb = t.y0 if side == "bottom" else t.y1 - 1
                if yb < n or yb > self.ny - m - 1:
                    raise PartitionError(f"interface y={yb} lies in the y-PML")

    def tile_at(self, tx, ty):
        if self.ncx is None:
            raise PartitionError("tile_at needs a tensor partition")
        if 0 <= tx < self.ncx and 0 <= ty < self.ncy:
            return self.tiles[ty * self.ncx + tx]
        return None

    def neighbours(self, i):
        """Tiles j != i whose extended rectangle grown by one cell (its ring's
        ghost nodes) meets tile i's extended rectangle, in index order.  Every
        interface entry that touches tile i belongs to one of them."""
        t = self.tiles[i]
        return [j for j, u in enumerate(self.tiles)
                if j != i and u.x0 - 1 < t.x1 and t.x0 < u.x1 + 1 and u.y0 - 1 < t.y1 and t.y0 < u.y1 + 1]

    # ---------------------------------------------------------------- rings
    def ring_nodes(self, t):
        """Boundary nodes of the extended tile, counter-clockwise from lower-left."""
        nodes = [(x, t.y0) for x in range(t.x0, t.x1)]
        nodes += [(t.x1 - 1, y) for y in range(t.y0 + 1, t.y1)]
        nodes += [(x, t.y1 - 1) for x in range(t.x1 - 2, t.x0 - 1, -1)]
        nodes += [(t.x0, y) for y in range(t.y1 - 2, t.y0, -1)]
        return nodes

    def trace_entries(self, t):
        """Interface-ring entries of tile t as (p=(ix,iy), q=(ix,iy), side).

        Ordered by the counter-clockwise ring walk; a corner node on two
        interface sides contributes one entry per side (bottom, right, top,
        left order).  Nodes on the global boundary only contribute nothing.
        """
        out = []
        for (ix, iy) in self.ring_nodes(t):
            for side in SIDES:
                if not t.iface[side]:
                    continue
                if side == "bottom" and iy == t.y0:
                    out.append(((ix, iy), (ix, iy - 1), side))
                elif side == "right" and ix == t.x1 - 1:
                    out.append(((ix, iy), (ix + 1, iy), side))
                elif side == "top" and iy == t.y1 - 1:
                    out.append(((ix, iy), (ix, iy + 1), side))
                elif side == "left" and ix == t.x0:
                    out.append(((ix, iy), (ix - 1, iy), side))
        return out


def robin_coeffs(kappa, h):
    d = 1.0 + 0.5j * kappa * h
    rho = (1.0 - 0.5j * kappa * h) / d
    tau = h / d
    return rho, tau


class LocalProblem:
    """B_i, the Robin data injection and the trace map for one tile and one wavelength."""

    def __init__(self, part: Partition, t: Tile, A, eps, k0, h):
        self.part, self.t, self.h, self.k0 = part, t, h, k0
        nx = part.nx
        self.gidx = t.global_indices(nx)
        B = A[self.gidx][:, self.gidx].tolil()
        ent = part.trace_entries(t)
        self.entries = ent
        ne = len(ent)
        self.p_loc = np.empty(ne, dtype=np.int64)
        self.q_glob = np.empty(ne, dtype=np.int64)
        self.p_glob = np.empty(ne, dtype=np.int64)
        self.a_pq = np.empty(ne, dtype=np.complex128)
        self.kappa = np.empty(ne, dtype=np.complex128)
        for e, ((px, py), (qx, qy), side) in enumerate(ent):
            pg = py * nx + px
            qg = qy * nx + qx
            self.p_loc[e] = t.local_index(px, py)
            self.p_glob[e] = pg
            self.q_glob[e] = qg
            self.a_pq[e] = A[pg, qg]
            self.kappa[e] = k0 * np.sqrt(complex(eps[py, px]))
        self.rho, self.tau = robin_coeffs(self.kappa, h)
        for e in range(ne):
            pl = self.p_loc[e]
            B[pl, pl] = B[pl, pl] + self.a_pq[e] * self.rho[e]
        self.B = B.tocsc()
        self._lu = None
        self.core = t.core_mask_local()

    @property
    def lu(self):
        if self._lu is None:
            self._lu = spla.splu(self.B)
        return self._lu

    def solve(self, rhs):
        return self.lu.solve(np.asarray(rhs, dtype=np.complex128))

    def inj(self, g):
        """Local RHS contribution of Robin data g (one value per trace entry)."""
        out = np.zeros(self.B.shape[0], dtype=np.complex128)
        np.add.at(out, self.p_loc, -self.a_pq * self.tau * g)
        return out

    def trace_of_global(self, u):
        """g_p(u) for every trace entry, from a global field u."""
        up = u[self.p_glob]
        uq = u[self.q_glob]
        return (uq - up) / self.h + 0.5j * self.kappa * (uq + up)

    def restrict(self, v):
        return v[self.gidx]

    def prolong_core(self, u_loc, out):
        out[self.gidx[self.core]] = u_loc[self.core]


def build_local_problems(part, A, eps, wavelength, h):
    k0 = 2.0 * np.pi / wavelength
    return [LocalProblem(part, t, A, eps, k0, h) for t in part.tiles]


def oras_apply(locs, v):
    """One-level ORAS: M1^-1 v = sum_i Rt_i^T B_i^-1 R_i v (core-only prolongation)."""
    z = np.zeros_like(v, dtype=np.complex128)
    for L in locs:
        L.prolong_core(L.solve(L.restrict(v)), z)
    return z


def stationary_sweep(locs, b, x, g_prev=None, momentum=0.0):
    """One Robin-data sweep of the domain-decomposition loop (Algorithm 3 body).

    Boundary values g_i are the traces of the current global iterate on each
    subdomain's interface ring (get_bc); with momentum m they are blended with
    the previous ones, bc = m*bc + (1-m)*bc_new.  Each subdomain solves its
    local Robin problem and the results are assembled on the cores.
    Returns (x_new, g_used).
    """
    g_new = [L.trace_of_global(x) for L in locs]
    if g_prev is None or momentum == 0.0:
        g_used = g_new
    else:
        g_used = [momentum * gp + (1.0 - momentum) * gn for gp, gn in zip(g_prev, g_new)]
    x_new = np.zeros_like(b, dtype=np.complex128)
    for L, g in zip(locs, g_used):
        u = L.solve(L.restrict(b) + L.inj(g))
        L.prolong_core(u, x_new)
    return x_new, g_used
