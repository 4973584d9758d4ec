"""Pins of the oracle's partition, Robin transmission, FGMRES and coarse space (CPU only)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.coarse import CoarseSpace, two_level_apply
from oracle.fdfd import assemble_A, point_source, solve_direct, source_rhs
from oracle.fgmres import fgmres, fgmres_fixed, givens
from oracle.partition import Partition, PartitionError, build_local_problems, oras_apply, stationary_sweep
from oracle.schwarz import SchwarzProblem
from paper_2509_03622_amd.workloads import random_small


def _problem(seed=0, n=96, cores=(32, 32, 32), lam=1.0, npml=8, k_coarse=0):
    w = random_small(seed, n, n, cores, cores, wavelengths=(lam,), npml=npml)
    P = SchwarzProblem(w.eps, lam, w.h, npml, w.core_x, w.core_y, w.overlap, k_coarse=k_coarse)
    return w, P


def test_partition_geometry():
    part = Partition(128, 128, [64, 64], [64, 64], 8, npml=12)
    t0, t3 = part.tiles[0], part.tiles[3]
    assert (t0.x0, t0.x1, t0.y0, t0.y1) == (0, 68, 0, 68)
    assert (t3.x0, t3.x1, t3.y0, t3.y1) == (60, 128, 60, 128)
    # the cores partition the grid exactly once
    cover = np.zeros((128, 128), int)
    for t in part.tiles:
        cover[t.cy0:t.cy1, t.cx0:t.cx1] += 1
    assert np.all(cover == 1)
    # trace entries: interface sides only; the inner corner is counted on both sides
    ent = part.trace_entries(t0)
    assert len(ent) == 68 + 68
    assert sum(1 for p, q, s in ent if p == (67, 67)) == 2


def test_partition_validation():
    with pytest.raises(PartitionError):
        Partition(128, 128, [64, 63], [64, 64], 8)
    with pytest.raises(PartitionError):
        Partition(128, 128, [64, 64], [64, 64], 7)
    with pytest.raises(PartitionError):
        Partition(128, 128, [8, 120], [64, 64], 8, npml=12)     # interface inside the x-PML


def test_robin_identity_every_tile():
    """B_i R_i u = R_i A u + inj(g(u)) for an arbitrary u (exact algebra)."""
    w, P = _problem(1)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(w.nx * w.ny) + 1j * rng.standard_normal(w.nx * w.ny)
    Au = P.A @ u
    for L in P.locs:
        lhs = L.B @ L.restrict(u)
        rhs = L.restrict(Au) + L.inj(L.trace_of_global(u))
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)


def test_local_problem_reproduces_global_solution():
    w, P = _problem(2)
    b = source_rhs(w.J()[0], 1.0)
    xs = solve_direct(P.A, b)
    for L in P.locs:
        u = L.solve(L.restrict(b) + L.inj(L.trace_of_global(xs)))
        assert np.linalg.norm(u - L.restrict(xs)) <= 1e-10 * np.linalg.norm(L.restrict(xs))


def test_outgoing_trace_small_incoming_large():
    """A +x plane wave has a small Robin trace on the +x side (outgoing) and ~2ik on the -x side."""
    errs = []
    for n in (40, 80):
        lam = 1.0
        h = 2.0 / n
        k = 2 * np.pi / lam
        eps = np.ones((n, n))
        A = assemble_A(eps, lam, h, 0)
        part = Partition(n, n, [n // 2, n // 2], [n], 4)
        locs = build_local_problems(part, A, eps, lam, h)
        kd = 2 / h * np.arcsin(k * h / 2)             # discrete wavenumber
        y, x = np.mgrid[0:n, 0:n]
        u = np.exp(-1j * kd * h * x).ravel()
        g_right = locs[0].trace_of_global(u)          # tile 0: interface on its +x side
        g_left = locs[1].trace_of_global(u)           # tile 1: interface on its -x side
        ratio = np.max(np.abs(g_right)) / np.min(np.abs(g_left))
        assert np.min(np.abs(g_left)) == pytest.approx(2 * k, rel=0.05)
        errs.append(ratio)
    assert errs[0] < 0.02
    assert 3.0 <= errs[0] / errs[1] <= 5.0          # O((kh)^2)


def test_stationary_sweep_equals_volume_step():
    w, P = _problem(3)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(w.nx * w.ny) + 1j * rng.standard_normal(w.nx * w.ny)
    b = source_rhs(w.J()[0], 1.0)
    x_new, _ = stationary_sweep(P.locs, b, x)
    ref = x + oras_apply(P.locs, b - P.A @ x)
    assert np.linalg.norm(x_new - ref) <= 1e-12 * np.linalg.norm(ref)


def test_stationary_sweep_converges_with_momentum():
    w, P = _problem(4, n=64, cores=(32, 32), npml=6)
    b = source_rhs(w.J()[0], 1.0)
    xs = solve_direct(P.A, b)
    x = np.zeros_like(b)
    g = None
    for _ in range(400):
        x, g = stationary_sweep(P.locs, b, x, g, momentum=0.2)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-4


def test_givens_zeroes_subdiagonal():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s = givens(a, b)
        assert abs(-np.conj(s) * a + c * b) < 1e-14
        assert abs(c * a + s * b) == pytest.approx(np.hypot(abs(a), abs(b)))
    c, s = givens(0.0, 2 + 1j)
    assert c == 0 and abs(s * (2 + 1j) - (2 + 1j)) < 1e-15


def test_fgmres_identity_matches_scipy_gmres():
    """With M = I the iteration count equals SciPy's restarted GMRES within one."""
    rng = np.random.default_rng(2)
    n = 300
    M = np.diag(rng.uniform(1, 3, n)) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    M = M + 1j * 0.2 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist, res = fgmres(lambda v: M @ v, b, tol=1e-8, restart=30, max_iters=500)
    count = [0]

    def cb(_):
        count[0] += 1
    xs, info = spla.gmres(M, b, rtol=1e-8, restart=30, maxiter=50, callback=cb, callback_type="pr_norm")
    assert info == 0
    assert abs(it - count[0]) <= 1
    assert np.linalg.norm(b - M @ x) / np.linalg.norm(b) <= 1e-8
    np.testing.assert_allclose(x, np.linalg.solve(M, b), rtol=1e-6)


def test_fgmres_history_monotone_and_lstsq():
    rng = np.random.default_rng(4)
    n = 120
    M = np.eye(n) + 0.5 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 0j
    x, it, hist, res = fgmres(lambda v: M @ v, b, tol=1e-10, restart=10, max_iters=200)
    for c0 in range(0, len(hist), 10):
        seg = hist[c0:c0 + 10]
        assert all(seg[i + 1] <= seg[i] * (1 + 1e-12) for i in range(len(seg) - 1))
    # the Givens recurrence gives the same minimum as a dense least-squares solve
    xk, k, h5 = fgmres_fixed(lambda v: M @ v, b, lambda v: v, 0.0, 5)
    K = np.stack([np.linalg.matrix_power(M, j) @ b for j in range(5)], axis=1)
    y, *_ = np.linalg.lstsq(M @ K, b, rcond=None)
    assert np.linalg.norm(b - M @ (K @ y)) / np.linalg.norm(b) == pytest.approx(h5[-1], rel=1e-8)


def test_single_tile_is_exact_preconditioner():
    w = random_small(5, 64, 64, [64], [64], npml=8)
    P = SchwarzProblem(w.eps, 1.0, w.h, 8, [64], [64], 8)
    x, it, hist, res = P.solve(w.J()[0], tol=1e-10)
    assert it == 1 and res < 1e-10


def test_schwarz_fgmres_matches_direct():
    w, P = _problem(6)
    b = source_rhs(w.J()[0], 1.0)
    xs = solve_direct(P.A, b)
    x, it, hist, res = P.solve(w.J()[0], tol=1e-10, max_iters=400)
    assert res <= 1e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-7
    assert 2 < it < 400


def test_coarse_correction_is_least_squares():
    w, P = _problem(7, k_coarse=2)
    cs = P.cs
    assert cs.nc == 2 * 9
    rng = np.random.default_rng(1)
    v = rng.standard_normal(w.nx * w.ny) + 1j * rng.standard_normal(w.nx * w.ny)
    z1 = oras_apply(P.locs, v)
    z, Az = two_level_apply(P.locs, P.A, cs, v)
    np.testing.assert_allclose(Az, P.A @ z, rtol=0, atol=1e-10 * np.linalg.norm(Az))
    t = v - Az
    assert np.linalg.norm(cs.W.conj().T @ t) <= 1e-10 * np.linalg.norm(v) * np.linalg.norm(cs.W.toarray())
    assert np.linalg.norm(t) <= np.linalg.norm(v - P.A @ z1)
    # basis fields live on their own core only
    Phi = cs.Phi.toarray()
    for col, i in enumerate(cs.tile_of_col):
        tt = P.part.tiles[i]
        f = np.abs(Phi[:, col]).reshape(w.ny, w.nx)
        mask = np.zeros_like(f, bool)
        mask[tt.cy0:tt.cy1, tt.cx0:tt.cx1] = True
        assert np.all(f[~mask] == 0) and np.any(f[mask] != 0)


def test_coarse_span_invariance():
    """Keeping all K trial directions, the correction does not depend on the rotation."""
    w = random_small(8, 96, 96, [32] * 3, [32] * 3, npml=8)
    A = assemble_A(w.eps, 1.0, w.h, 8)
    part = Partition(96, 96, [32] * 3, [32] * 3, 8, npml=8)
    locs = build_local_problems(part, A, w.eps, 1.0, w.h)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(96 * 96) + 1j * rng.standard_normal(96 * 96)
    outs = []
    for rot in ("svd", "eig", "none"):
        cs = CoarseSpace(part, locs, A, w.eps, 1.0, w.h, k_coarse=4, k_trial=4, rotation=rot)
        outs.append(two_level_apply(locs, A, cs, v)[0])
    for o in outs[1:]:
        assert np.linalg.norm(o - outs[0]) <= 1e-9 * np.linalg.norm(outs[0])


def test_two_level_converges_to_direct_solution():
    """The two-level preconditioned FGMRES reaches the direct solution (the coarse
    correction changes the path, not the fixed point)."""
    w = random_small(9, 128, 128, [32] * 4, [32] * 4, npml=8, block=16)
    P = SchwarzProblem(w.eps, 1.2, w.h, 8, w.core_x, w.core_y, 8, k_coarse=2)
    b = source_rhs(w.J()[0], 1.2)
    xs = solve_direct(P.A, b)
    x, it, hist, res = P.solve(w.J()[0], tol=1e-9, max_iters=800)
    assert res <= 1e-9
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-6


def test_dependent_probes_are_dropped_and_span_is_kept():
    """On a corner subdomain (L-shaped interface ring) the 8 pseudo-plane waves are
    linearly dependent; Gram-Schmidt keeps an orthonormal basis of their span."""
    from oracle.coarse import mgs_columns, pseudo_plane_waves
    w = random_small(22, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.1,), npml=12, block=16)
    A = assemble_A(w.eps, 1.1, w.h, 12)
    part = Partition(192, 192, [64] * 3, [64] * 3, 8, 12)
    locs = build_local_problems(part, A, w.eps.astype(float), 1.1, w.h)
    raw = pseudo_plane_waves(part, part.tiles[0], locs[0], 8, w.eps, 2 * np.pi / 1.1, w.h)
    sv = np.linalg.svd(raw, compute_uv=False)
    assert sv[-1] < 1e-10 * sv[0]                      # rank 7 in exact arithmetic
    Q = mgs_columns(raw)
    assert Q.shape[1] == 7
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(7), atol=1e-12)
    resid = raw - Q @ (Q.conj().T @ raw)
    assert np.linalg.norm(resid) < 1e-10 * np.linalg.norm(raw)
    # an interior subdomain keeps all 8
    Q4 = mgs_columns(pseudo_plane_waves(part, part.tiles[4], locs[4], 8, w.eps, 2 * np.pi / 1.1, w.h))
    assert Q4.shape[1] == 8
