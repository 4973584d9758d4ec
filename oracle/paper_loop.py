"""The paper's own outer loop: the stationary Robin-data iteration with
momentum and the coarse correction in Robin-data space (oracle, test
infrastructure only).  Follows Algorithm 3 and the two-level paragraphs of
the Methods (coarse equation and its normal equations) in this reading:

State: the Robin data g_i of every subdomain on its interface entries (the
"bc" of Algorithm 3), all subdomains stacked into one vector g.

One sweep (Algorithm 3 loop body): u_i = B_i^-1 (R_i b + inj(g_i)) for every
subdomain, x = sum_i Rt_i^T u_i (core-only assembly), g_new = the Robin
traces of x on every interface entry.  The sweep is affine in g:
g_new = T g + c, T the Robin-to-Robin map (the homogeneous part) and c the
traces of the assembled solves with g = 0; the exact data g* = traces(x*)
is its fixed point.

Momentum (Algorithm 3): g <- m g + (1 - m) g_new.

Coarse correction: the boundary mismatch of the sweep is e = g_new - g
(the data each subdomain satisfied against the traces its neighbours' solution
implies), which is the residual of the fixed-point equation (I - T) g = c.
With Q the basis boundary data (per subdomain, the k_coarse rotated
pseudo-plane-wave probes of the coarse space, zero on other subdomains) the
coarse equation (I - T) Q z = e is solved in the least-squares sense through
its normal equations ((I - T) Q)^H (I - T) Q z = ((I - T) Q)^H e, the matrix
assembled once.  The correction added after the momentum step is
(m Q + (1 - m) T Q) z: the coarse step applied to the data before the sweep,
carried through the sweep and the momentum blend, so that an error of g that
lies in span Q is removed in one iteration.  T Q is formed column by column
as the traces of the assembled homogeneous solves of the basis data, i.e. the
traces of the coarse basis fields.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .coarse import CoarseSpace


def entry_offsets(locs):
    off = np.zeros(len(locs) + 1, dtype=np.int64)
    for i, L in enumerate(locs):
        off[i + 1] = off[i] + len(L.entries)
    return off


def traces(locs, x):
    """Robin traces of a global field on every subdomain's interface entries, stacked."""
    return np.concatenate([L.trace_of_global(x) for L in locs]) if locs else np.zeros(0, complex)


def sweep(locs, b, g):
    """x = sum_i Rt_i^T B_i^-1 (R_i b + inj(g_i)) and its traces g_new."""
    off = entry_offsets(locs)
    x = np.zeros(b.shape[0], dtype=np.complex128)
    for i, L in enumerate(locs):
        u = L.solve(L.restrict(b) + L.inj(g[off[i]:off[i + 1]]))
        L.prolong_core(u, x)
    return x, traces(locs, x)


class RobinCoarse:
    """Q, T Q and the normal equations of (I - T) Q z = e."""

    def __init__(self, cs: CoarseSpace, locs):
        off = entry_offsets(locs)
        ne = int(off[-1])
        nc = cs.nc
        self.Q = np.zeros((ne, nc), dtype=np.complex128)
        self.TQ = np.zeros((ne, nc), dtype=np.complex128)
        Phi = cs.Phi.toarray() if nc else np.zeros((0, 0))
        for c in range(nc):
            i = cs.tile_of_col[c]
            self.Q[off[i]:off[i + 1], c] = cs.U_cols[c]
            self.TQ[:, c] = traces(locs, Phi[:, c])
        self.M = self.Q - self.TQ
        G = self.M.conj().T @ self.M
        zero = np.linalg.norm(self.M, axis=0) == 0
        G[zero, zero] = 1.0                 # a zero basis column keeps coefficient 0
        self.G = G
        self.chol = sla.cho_factor(G, lower=True) if nc else None
        self.nc = nc

    def coefficients(self, e):
        return sla.cho_solve(self.chol, self.M.conj().T @ e)

    def correction(self, e, m):
        z = self.coefficients(e)
        return m * (self.Q @ z) + (1.0 - m) * (self.TQ @ z)


def paper_loop(locs, A, b, momentum=0.0, coarse: RobinCoarse | None = None, tol=1e-6, max_iters=1000, g0=None):
    """Algorithm 3 from g = g0 (zero: the traces of x = 0).  Returns the
    assembled field of the last sweep, the number of sweeps, the relative
    residual history ||b - A x||/||b|| after each sweep, and the final data."""
    off = entry_offsets(locs)
    g = np.zeros(int(off[-1]), dtype=np.complex128) if g0 is None else np.array(g0, dtype=np.complex128)
    bn = np.linalg.norm(b)
    hist = []
    x = np.zeros_like(b, dtype=np.complex128)
    for k in range(max_iters):
        x, g_new = sweep(locs, b, g)
        hist.append(float(np.linalg.norm(b - A @ x) / bn))
        if hist[-1] <= tol:
            return x, k + 1, hist, g
        e = g_new - g
        g_next = momentum * g + (1.0 - momentum) * g_new
        if coarse is not None and coarse.nc:
            g_next = g_next + coarse.correction(e, momentum)
        g = g_next
    return x, max_iters, hist, g
