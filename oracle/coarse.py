"""Pseudo-plane-wave coarse space and the two-level preconditioner (oracle).

Test infrastructure only.  Follows the coarse-space paragraphs of Sec. 2.2 and
of the Methods two-level subsection, and the one-time pre-compute block of
Algorithm 3, in this reading:

1. Trial Robin data per subdomain: K pseudo-plane waves, directions
   theta_l = 2 pi l / K.  The phase is accumulated around the subdomain's
   boundary ring (counter-clockwise from the lower-left node) with the local
   wavenumber kappa = k0 sqrt(eps):  phi_{m+1} = phi_m + h (kappa_m +
   kappa_{m+1})/2 * d_l . (p_{m+1} - p_m),  x_l(p) = exp(-i phi(p)).
   Entries on the global boundary are dropped.
2. Gram-Schmidt (modified) orthonormalisation of the K trial vectors;
   dependent trial vectors are dropped (this happens on corner subdomains,
   whose interface ring is an L-shape).
3. Homogeneous local solves F_l = B_i^-1 inj(x_l) (no source term).
4. y_l = Robin traces of F_l on the interface rings of the neighbouring
   subdomains (every subdomain whose ring or ghost nodes reach into this one,
   diagonal neighbours included), where those rings lie inside the
   subdomain: the map x -> y is the Robin-to-Robin map.
5. Rayleigh-Ritz on (x, y) in its SVD form (the paper reports SVD works about
   as well as the eigen-decomposition): Y = U S V^H, the k_coarse right
   singular vectors with the largest singular values (slowest decaying
   modes) give the subdomain's basis, u_l = X V[:, l].  A subdomain with fewer
   independent probes than k_coarse gets zero basis columns, whose coefficient
   is fixed at 0 by a unit diagonal entry in G.
6. Basis fields phi_{i,l} = Rt_i^T B_i^-1 inj(u_l), spread over the global
   grid by the core-only (RAS) prolongation.

Coarse correction (volume reading of the normal equations
(conj(BQ))^T BQ z = (conj(BQ))^T e_bc): with W = A Phi and G = W^H W,
after the one-level result z1 = M1^-1 v the coefficients c = G^-1 W^H (v - A z1)
minimise ||v - A (z1 + Phi c)||, and z = z1 + Phi c.  G is factored once
(Cholesky, complex128).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .partition import oras_apply


def pseudo_plane_waves(part, t, loc, K, eps, k0, h):
    """Trial Robin data, one column per direction, over tile t's trace entries."""
    ring = part.ring_nodes(t)
    kap = np.array([k0 * np.sqrt(complex(eps[iy, ix])) for (ix, iy) in ring])
    pos = np.array(ring, dtype=np.float64)
    X_node = np.zeros((len(ring), K), dtype=np.complex128)
    for l in range(K):
        th = 2.0 * np.pi * l / K
        d = np.array([np.cos(th), np.sin(th)])
        phi = np.zeros(len(ring), dtype=np.complex128)
        for m in range(len(ring) - 1):
            step = pos[m + 1] - pos[m]
            phi[m + 1] = phi[m] + h * 0.5 * (kap[m] + kap[m + 1]) * (d @ step)
        X_node[:, l] = np.exp(-1j * phi)
    node_row = {p: r for r, p in enumerate(ring)}
    rows = [node_row[p] for (p, q, side) in loc.entries]
    return X_node[rows]


DROP_TOL = 1e-8      # a probe whose Gram-Schmidt residual is below this fraction of its norm is dependent


def mgs_columns(X, drop_tol=DROP_TOL):
    """Modified Gram-Schmidt; dependent columns are dropped (the result spans span X).

    On subdomains with only two interface sides the pseudo-plane waves can be
    linearly dependent; normalising a residual of rounding size would create
    a spurious direction, so such a probe is removed.
    """
    cols = []
    for l in range(X.shape[1]):
        v = np.array(X[:, l], dtype=np.complex128)
        n0 = np.linalg.norm(v)
        for q in cols:
            v = v - np.vdot(q, v) * q
        n = np.linalg.norm(v)
        if n > drop_tol * n0:
            cols.append(v / n)
    return np.stack(cols, axis=1)


def neighbour_traces(part, locs, i, F_loc):
    """Robin traces of local fields F (columns) on neighbours' interface rings inside tile i."""
    t = part.tiles[i]
    rows = []
    for j in part.neighbours(i):
        Lj = locs[j]
        for e, (p, q, side) in enumerate(Lj.entries):
            if t.contains(*p) and t.contains(*q):
                up = F_loc[t.local_index(*p)]
                uq = F_loc[t.local_index(*q)]
                rows.append((uq - up) / Lj.h + 0.5j * Lj.kappa[e] * (uq + up))
    if not rows:
        return np.zeros((0, F_loc.shape[1]), dtype=np.complex128)
    return np.array(rows)


class CoarseSpace:
    """Phi (global basis fields), W = A Phi, Cholesky of G = W^H W."""

    def __init__(self, part, locs, A, eps, wavelength, h, k_coarse, k_trial=8, rotation="svd"):
        k0 = 2.0 * np.pi / wavelength
        K = max(k_trial, k_coarse)
        n = part.nx * part.ny
        cols = []
        self.tile_of_col = []
        self.U_cols = []          # Robin data of each basis column on its tile's interface entries
        for i, (t, L) in enumerate(zip(part.tiles, locs)):
            if len(L.entries) == 0:
                continue
            X = mgs_columns(pseudo_plane_waves(part, t, L, K, eps, k0, h))
            Kt = X.shape[1]
            F = np.stack([L.solve(L.inj(X[:, l])) for l in range(Kt)], axis=1)
            if rotation == "svd":
                Y = neighbour_traces(part, locs, i, F)
                _, _, Vh = np.linalg.svd(Y, full_matrices=True)
                V = Vh.conj().T
            elif rotation == "eig":
                # Rayleigh-Ritz with H = X^H (Y projected back): use the eigenvectors
                # of Y^H Y (same right space as the SVD), ordered by decreasing eigenvalue.
                Y = neighbour_traces(part, locs, i, F)
                w, Vv = np.linalg.eigh(Y.conj().T @ Y)
                V = Vv[:, np.argsort(-w)]
            else:   # "none": keep the orthonormal trial directions as they are
                V = np.eye(Kt, dtype=np.complex128)
            for l in range(k_coarse):
                phi = np.zeros(n, dtype=np.complex128)
                u = np.zeros(len(L.entries), dtype=np.complex128)
                if l < Kt:          # fewer independent probes than k_coarse: zero column
                    L.prolong_core(F @ V[:, l], phi)
                    u = X @ V[:, l]
                cols.append(phi)
                self.tile_of_col.append(i)
                self.U_cols.append(u)
        # each basis field lives on one core: keep Phi and W = A Phi sparse
        self.Phi = (sp.csc_matrix(np.stack(cols, axis=1)) if cols
                    else sp.csc_matrix((n, 0), dtype=np.complex128))
        self.W = (A @ self.Phi).tocsc()
        self.G = (self.W.conj().T @ self.W).toarray()
        # a zero basis column gets a unit diagonal entry, so its coefficient is 0
        zero = np.asarray(abs(self.W).sum(axis=0)).ravel() == 0
        self.G[zero, zero] = 1.0
        self.nc = self.Phi.shape[1]
        self.chol = sla.cho_factor(self.G, lower=True) if self.nc else None

    def coefficients(self, t_vec):
        d = self.W.conj().T @ t_vec
        return sla.cho_solve(self.chol, d)


def two_level_apply(locs, A, cs: CoarseSpace, v):
    """z = z1 + Phi c with z1 = M1^-1 v and c = G^-1 W^H (v - A z1); returns (z, A z)."""
    z1 = oras_apply(locs, v)
    w1 = A @ z1
    if cs is None or cs.nc == 0:
        return z1, w1
    c = cs.coefficients(v - w1)
    return z1 + cs.Phi @ c, w1 + cs.W @ c
