"""Closed-form pins of the oracle's coarse-space construction (CPU only).

The coarse space of the two-level method (Sec. 2.2, coarse-space paragraphs;
Methods, two-level subsection; Algorithm 3 pre-compute block) starts from
pseudo-plane waves on each subdomain's boundary ring and keeps the rotated
probes whose neighbour traces decay slowest.  The least-squares and
span-invariance tests elsewhere hold for any basis; these tests pin the
construction itself:

* on a homogeneous medium a pseudo-plane wave is exactly the plane wave
  exp(-i kappa h d_l . (p - p0)) sampled on the ring (p0 the first ring node),
  for interior, edge and corner subdomains and for more than eight directions;
* that plane wave travels along +d_l in the exp(+i omega t) convention: its
  discrete Robin data vanish to O((kappa h)^2) on a side whose outward normal
  is d_l and are about 2 kappa |u| on the opposite side;
* the kept columns are the right singular vectors of the neighbour-trace
  matrix Y with the largest singular values, checked against eigenvalues of
  Y^H Y and against random directions of the probe span.
"""
import numpy as np
import scipy.linalg as sla

from oracle.coarse import CoarseSpace, mgs_columns, neighbour_traces, pseudo_plane_waves
from oracle.fdfd import assemble_A
from oracle.partition import Partition, build_local_problems
from paper_2509_03622_amd.workloads import random_small

H = 0.05


def _homogeneous(eps_val=2.25, lam=1.0, n=96, core=32, npml=8):
    eps = np.full((n, n), eps_val)
    A = assemble_A(eps, lam, H, npml)
    part = Partition(n, n, [core] * (n // core), [core] * (n // core), 8, npml=npml)
    locs = build_local_problems(part, A, eps, lam, H)
    return eps, part, locs


def test_pseudo_plane_waves_equal_sampled_plane_waves_on_homogeneous_medium():
    lam, eps_val = 1.0, 2.25
    eps, part, locs = _homogeneous(eps_val, lam)
    k0 = 2 * np.pi / lam
    kappa = k0 * np.sqrt(eps_val)
    # corner (0), edge (1), interior (4); K = 8 and K = 12 directions
    for ti in (0, 1, 4):
        t, L = part.tiles[ti], locs[ti]
        p0 = np.array(part.ring_nodes(t)[0], dtype=float)
        assert tuple(p0) == (t.x0, t.y0)
        P = np.array([p for (p, q, side) in L.entries], dtype=float)
        for K in (8, 12):
            X = pseudo_plane_waves(part, t, L, K, eps, k0, H)
            assert X.shape == (len(L.entries), K)
            for l in range(K):
                th = 2 * np.pi * l / K
                d = np.array([np.cos(th), np.sin(th)])
                expect = np.exp(-1j * kappa * H * ((P - p0) @ d))
                np.testing.assert_allclose(X[:, l], expect, rtol=0, atol=1e-12)


def test_pseudo_plane_wave_direction_is_outgoing_along_d():
    """Direction d_l = +x (l = 0) and -x (l = K/2) on the interior subdomain's
    right and left interface sides."""
    lam, eps_val = 1.0, 2.25
    eps, part, locs = _homogeneous(eps_val, lam)
    k0 = 2 * np.pi / lam
    kappa = k0 * np.sqrt(eps_val)
    ti = 4
    t, L = part.tiles[ti], locs[ti]
    K = 8
    X = pseudo_plane_waves(part, t, L, K, eps, k0, H)
    n = part.nx
    iy, ix = np.mgrid[0:n, 0:n]
    sides = np.array([side for (p, q, side) in L.entries])
    p0 = part.ring_nodes(t)[0]
    for l, out_side, in_side in ((0, "right", "left"), (K // 2, "left", "right")):
        th = 2 * np.pi * l / K
        # the plane wave whose ring samples are probe l, continued over the grid
        u = np.exp(-1j * kappa * H * ((ix - p0[0]) * np.cos(th) + (iy - p0[1]) * np.sin(th))).ravel()
        np.testing.assert_allclose(u[L.p_glob], X[:, l], rtol=0, atol=1e-12)
        g = L.trace_of_global(u)
        g_out = np.abs(g[sides == out_side])
        g_in = np.abs(g[sides == in_side])
        assert g_out.max() < 0.2 * (kappa * H) ** 2 * kappa
        np.testing.assert_allclose(g_in, 2 * kappa, rtol=0.05)


def _probe_data(part, locs, i, eps, k0, K):
    t, L = part.tiles[i], locs[i]
    X = mgs_columns(pseudo_plane_waves(part, t, L, K, eps, k0, H))
    F = np.stack([L.solve(L.inj(X[:, l])) for l in range(X.shape[1])], axis=1)
    Y = neighbour_traces(part, locs, i, F)
    return X, Y


def test_kept_columns_are_top_right_singular_vectors():
    lam = 1.0
    w = random_small(31, 96, 96, [32] * 3, [32] * 3, wavelengths=(lam,), npml=8, block=16)
    eps = w.eps.astype(float)
    A = assemble_A(eps, lam, w.h, 8)
    part = Partition(96, 96, [32] * 3, [32] * 3, 8, npml=8)
    locs = build_local_problems(part, A, eps, lam, w.h)
    k0 = 2 * np.pi / lam
    kc = 2
    cs = CoarseSpace(part, locs, A, eps, lam, w.h, k_coarse=kc, k_trial=8)
    rng = np.random.default_rng(4)
    for i in (0, 1, 4):
        X, Y = _probe_data(part, locs, i, eps, k0, 8)
        Kt = X.shape[1]
        cols = [c for c, ti in enumerate(cs.tile_of_col) if ti == i]
        assert len(cols) == kc
        # coefficients of the kept Robin data in the orthonormal probe basis
        a = [X.conj().T @ cs.U_cols[c] for c in cols]
        for c, ac in zip(cols, a):
            np.testing.assert_allclose(X @ ac, cs.U_cols[c], rtol=0, atol=1e-10)
            assert abs(np.linalg.norm(ac) - 1.0) < 1e-10
        assert abs(np.vdot(a[0], a[1])) < 1e-10
        # singular values from the eigenvalues of Y^H Y (a different routine)
        ev = np.sort(sla.eigvalsh(Y.conj().T @ Y))[::-1]
        sig = np.sqrt(np.maximum(ev, 0.0))
        assert sig[0] > 1.5 * sig[-1]                    # a real spread, so order matters
        for l in range(kc):
            assert abs(np.linalg.norm(Y @ a[l]) - sig[l]) <= 1e-8 * sig[0]
        # no unit direction of the probe span decays slower than the first kept one
        best = np.linalg.norm(Y @ a[0])
        for _ in range(200):
            v = rng.standard_normal(Kt) + 1j * rng.standard_normal(Kt)
            v /= np.linalg.norm(v)
            assert np.linalg.norm(Y @ v) <= best * (1 + 1e-12)
