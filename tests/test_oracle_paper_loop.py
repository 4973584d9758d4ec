"""Pins of the oracle's Algorithm 3 loop (stationary Robin-data iteration with
momentum and the Robin-space coarse correction) against what the mathematics
fixes independently of the code:

* the exact data g* = traces(x*) is a fixed point: one sweep returns x* and
  reproduces g*;
* without momentum or coarse correction one sweep from the traces of any x is
  the volume step x + M1^-1 (b - A x) (the Robin identity, exact);
* T Q computed from the coarse basis fields (rotated probe solves) equals the
  homogeneous sweep of the basis Robin data (a different route through the
  local solves);
* the coarse coefficients satisfy the normal equations' orthogonality
  ((I - T) Q)^H (e - (I - T) Q z) = 0;
* an error of the Robin data inside span Q is removed by one iteration, for
  any momentum (exact to rounding);
* the loop converges to the direct solution.
"""
import numpy as np
import pytest

from oracle.coarse import CoarseSpace
from oracle.fdfd import assemble_A, solve_direct, source_rhs
from oracle.paper_loop import RobinCoarse, paper_loop, sweep, traces
from oracle.partition import Partition, build_local_problems, oras_apply
from paper_2509_03622_amd.workloads import random_small


@pytest.fixture(scope="module")
def prob():
    w = random_small(61, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.0,), npml=12, block=16)
    lam = 1.0
    A = assemble_A(w.eps, lam, w.h, w.npml)
    part = Partition(w.nx, w.ny, w.core_x, w.core_y, w.overlap, w.npml)
    locs = build_local_problems(part, A, w.eps.astype(np.float64), lam, w.h)
    b = source_rhs(w.J()[0], lam)
    xs = solve_direct(A, b)
    cs = CoarseSpace(part, locs, A, w.eps.astype(np.float64), lam, w.h, 2, 8)
    return w, A, locs, b, xs, RobinCoarse(cs, locs)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_exact_data_is_a_fixed_point(prob):
    w, A, locs, b, xs, rc = prob
    gs = traces(locs, xs)
    x, gn = sweep(locs, b, gs)
    assert rel(x, xs) < 1e-10
    assert rel(gn, gs) < 1e-10


def test_sweep_without_momentum_is_the_volume_step(prob):
    w, A, locs, b, xs, rc = prob
    rng = np.random.default_rng(3)
    xp = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
    x, _ = sweep(locs, b, traces(locs, xp))
    ref = xp + oras_apply(locs, b - A @ xp)
    assert rel(x, ref) < 1e-10


def test_TQ_equals_homogeneous_sweep_of_basis_data(prob):
    w, A, locs, b, xs, rc = prob
    zero = np.zeros_like(b)
    for c in range(rc.nc):
        _, tq = sweep(locs, zero, rc.Q[:, c])
        assert np.linalg.norm(tq - rc.TQ[:, c]) <= 1e-10 * max(np.linalg.norm(rc.TQ[:, c]), 1e-300)


def test_coarse_coefficients_solve_the_normal_equations(prob):
    w, A, locs, b, xs, rc = prob
    rng = np.random.default_rng(5)
    e = rng.standard_normal(rc.Q.shape[0]) + 1j * rng.standard_normal(rc.Q.shape[0])
    z = rc.coefficients(e)
    ortho = rc.M.conj().T @ (e - rc.M @ z)
    assert np.linalg.norm(ortho) < 1e-9 * np.linalg.norm(rc.M.conj().T @ e)


@pytest.mark.parametrize("m", [0.0, 0.3, 0.7])
def test_coarse_span_error_removed_in_one_iteration(prob, m):
    w, A, locs, b, xs, rc = prob
    gs = traces(locs, xs)
    rng = np.random.default_rng(7)
    z0 = rng.standard_normal(rc.nc) + 1j * rng.standard_normal(rc.nc)
    g = gs + rc.Q @ z0
    x, gn = sweep(locs, b, g)
    g_next = m * g + (1 - m) * gn + rc.correction(gn - g, m)
    assert rel(g_next, gs) < 1e-10
    # without the correction the error would persist
    assert rel(m * g + (1 - m) * gn, gs) > 1e-3


@pytest.mark.parametrize("m,coarse", [(0.0, False), (0.3, False), (0.0, True)])
def test_loop_converges_to_direct_solution(prob, m, coarse):
    w, A, locs, b, xs, rc = prob
    x, it, hist, g = paper_loop(locs, A, b, momentum=m, coarse=rc if coarse else None, tol=1e-6, max_iters=300)
    assert it < 300 and hist[-1] <= 1e-6
    assert rel(x, xs) < 1e-5
    assert len(hist) == it
