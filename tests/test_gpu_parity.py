"""GPU parity: every step of the Schwarz sweep, called through the C ABI,
against the FP64 oracle on the same seeded inputs.

Tolerances (complex64 arithmetic against complex128):
* operator and traces: 1e-6 relative L2 (a handful of FP32 roundings per entry);
* exact local solves and the one-level sweep: 2e-5 (block-Thomas in FP32 on
  factors formed in FP64; measured ~4e-7 on the hardest tiles);
* whole solves: field within 1e-5 of the direct solution when the oracle's
  own FP64 Schwarz-FGMRES at the same tolerance is within 5e-6 of it, and
  iteration counts within one of the oracle's, also for restart lengths 7
  and 31 (the largest Krylov dimension, with a full cycle before the
  restart).
"""
import numpy as np
import pytest

from oracle.coarse import CoarseSpace, two_level_apply
from oracle.fdfd import assemble_A, solve_direct, source_rhs
from oracle.partition import Partition, build_local_problems, oras_apply
from oracle.schwarz import SchwarzProblem
from paper_2509_03622_amd.workloads import random_small, small_rectangles

from gpu_common import dev, host, make_gpu_problem, rel

pytestmark = pytest.mark.gpu


def ragged():
    # 200 x 128 grid, cores [60, 64, 76] x [60, 68]: extended tiles 64..80 wide,
    # both block orientations, two wavelengths and two sources per wavelength.
    return random_small(21, 200, 128, [60, 64, 76], [60, 68], wavelengths=(0.9, 1.3), n_src=2, npml=10)


def oracle_parts(w, lam):
    A = assemble_A(w.eps, lam, w.h, w.npml, w.pml_m, w.pml_lnR)
    part = Partition(w.nx, w.ny, w.core_x, w.core_y, w.overlap, w.npml)
    locs = build_local_problems(part, A, w.eps.astype(np.float64), lam, w.h)
    return A, part, locs


def test_operator_matches_oracle():
    w = ragged()
    ctx, P = make_gpu_problem(w, k_coarse=0)
    rng = np.random.default_rng(0)
    ns = 2
    x = (rng.standard_normal((len(w.wavelengths), ns, w.ny, w.nx)) +
         1j * rng.standard_normal((len(w.wavelengths), ns, w.ny, w.nx))).astype(np.complex64)
    b = (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)).astype(np.complex64)
    xd, bd = dev(x), dev(b)
    y = dev(np.zeros_like(x))
    r = dev(np.zeros_like(x))
    P.apply_operator(xd, y, None, ns)
    P.apply_operator(xd, r, bd, ns)
    y, r = host(y), host(r)
    for wi, lam in enumerate(w.wavelengths):
        A = assemble_A(w.eps, lam, w.h, w.npml)
        for s in range(ns):
            ref = A @ x[wi, s].ravel().astype(np.complex128)
            assert rel(y[wi, s].ravel(), ref) < 1e-6
            assert rel(r[wi, s].ravel(), b[wi, s].ravel() - ref) < 1e-6


def test_local_solves_match_sparse_lu():
    w = ragged()
    ctx, P = make_gpu_problem(w, k_coarse=0)
    nt, lc, ne, nc = P.sizes()
    rng = np.random.default_rng(1)
    rhs = (rng.standard_normal((len(w.wavelengths), lc)) + 1j * rng.standard_normal((len(w.wavelengths), lc)))
    u = dev(np.zeros_like(rhs))
    P.local_solve(dev(rhs), u)
    u = host(u)
    worst = 0.0
    for wi, lam in enumerate(w.wavelengths):
        A, part, locs = oracle_parts(w, lam)
        for t, L in enumerate(locs):
            info = P.tile_info(t)
            assert info[:4] == [L.t.x0, L.t.x1, L.t.y0, L.t.y1]
            off = info[8]
            n = L.B.shape[0]
            ref = L.solve(rhs[wi, off:off + n])
            worst = max(worst, rel(u[wi, off:off + n], ref))
    assert worst < 2e-5, worst


def test_schwarz_sweep_matches_oracle():
    w = ragged()
    ctx, P = make_gpu_problem(w, k_coarse=0)
    rng = np.random.default_rng(2)
    shape = (len(w.wavelengths), 2, w.ny, w.nx)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    z = dev(np.zeros(shape))
    P.schwarz_sweep(dev(v), z, 2)
    z = host(z)
    for wi, lam in enumerate(w.wavelengths):
        A, part, locs = oracle_parts(w, lam)
        for s in range(2):
            ref = oras_apply(locs, v[wi, s].ravel())
            assert rel(z[wi, s].ravel(), ref) < 2e-5


def test_robin_traces_match_oracle():
    w = ragged()
    ctx, P = make_gpu_problem(w, k_coarse=0)
    nt, lc, ne, nc = P.sizes()
    rng = np.random.default_rng(3)
    shape = (len(w.wavelengths), w.ny, w.nx)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    g = dev(np.zeros((len(w.wavelengths), ne)))
    P.robin_trace(dev(x), g)
    g = host(g)
    for wi, lam in enumerate(w.wavelengths):
        A, part, locs = oracle_parts(w, lam)
        ref = np.concatenate([L.trace_of_global(x[wi].ravel()) for L in locs])
        assert ref.shape[0] == ne
        assert rel(g[wi], ref) < 1e-6


@pytest.mark.parametrize("k_coarse,k_trial", [(4, 4), (1, 8)])
def test_two_level_preconditioner_matches_oracle(k_coarse, k_trial):
    """With k_coarse = k_trial the coarse span is the whole probe span, so the
    correction does not depend on the Rayleigh-Ritz rotation; with k_coarse = 1
    the selected direction must agree too.  The selected singular vector moves
    by at most (trace error) x sigma_1 / (sigma_1 - sigma_2), and the smallest
    relative gap on this problem is 0.039 (a factor 25 on the FP32 trace error
    of about 1e-7 -- 1e-6); both cases measure 5e-7 (z) and 1e-6 (A z) and are
    held to 1e-5."""
    tol = 1e-5
    w = random_small(22, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.1,), npml=12, block=16)
    w.k_coarse, w.k_trial = k_coarse, k_trial
    ctx, P = make_gpu_problem(w)
    nt, lc, ne, nc = P.sizes()
    assert nc == 9 * k_coarse
    rng = np.random.default_rng(4)
    v = rng.standard_normal((1, 1, w.ny, w.nx)) + 1j * rng.standard_normal((1, 1, w.ny, w.nx))
    z, Az = dev(np.zeros(v.shape)), dev(np.zeros(v.shape))
    P.precond_apply(dev(v), z, Az, 1)
    z, Az = host(z), host(Az)
    A, part, locs = oracle_parts(w, 1.1)
    cs = CoarseSpace(part, locs, A, w.eps.astype(np.float64), 1.1, w.h, k_coarse, k_trial)
    zr, Azr = two_level_apply(locs, A, cs, v.ravel())
    print(f"k_coarse {k_coarse}: z {rel(z.ravel(), zr):.2e}, Az {rel(Az.ravel(), Azr):.2e}")
    assert rel(z.ravel(), zr) < tol
    assert rel(Az.ravel(), Azr) < tol


def test_rect128_solve_matches_direct_and_oracle_iterations():
    w = small_rectangles()
    ctx, P = make_gpu_problem(w)
    E, hist, iters, fin, st = P.solve(w.J(), tol=1e-6, restart=30, max_iters=1000)
    assert st == 0
    lam = w.wavelengths[0]
    A = assemble_A(w.eps, lam, w.h, w.npml)
    b = source_rhs(w.J()[0], lam)
    xs = solve_direct(A, b)
    op = SchwarzProblem(w.eps, lam, w.h, w.npml, w.core_x, w.core_y, w.overlap)
    xo, it_o, hist_o, res_o = op.solve(w.J()[0], tol=1e-6)
    assert rel(xo, xs) < 5e-6                   # the oracle's own accuracy at this tolerance
    assert rel(E[0, 0].ravel(), xs) < 1e-5
    assert abs(int(iters[0, 0]) - it_o) <= 1
    assert fin[0, 0] <= 1e-6
    assert np.linalg.norm(b - A @ E[0, 0].ravel().astype(np.complex128)) / np.linalg.norm(b) < 2e-6
    h = hist[0, 0, :iters[0, 0]]
    np.testing.assert_allclose(h[:10], np.array(hist_o[:10]), rtol=2e-3)
    assert np.all(hist[0, 0, iters[0, 0]:] == -1)


@pytest.mark.parametrize("restart", [7, 31])
def test_restart_lengths_match_oracle(restart):
    # 31 is the largest Krylov dimension the library takes: this one-level
    # problem needs 48 iterations, so a whole cycle runs the Gram-Schmidt
    # passes over 31 basis vectors before the restart
    w = random_small(61, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.0,), npml=12, block=16)
    ctx, P = make_gpu_problem(w, k_coarse=0)
    E, hist, iters, fin, st = P.solve(w.J(), tol=1e-6, restart=restart, max_iters=1000)
    assert st == 0
    lam = w.wavelengths[0]
    A = assemble_A(w.eps, lam, w.h, w.npml)
    xs = solve_direct(A, source_rhs(w.J()[0], lam))
    op = SchwarzProblem(w.eps, lam, w.h, w.npml, w.core_x, w.core_y, w.overlap)
    xo, it_o, hist_o, res_o = op.solve(w.J()[0], tol=1e-6, restart=restart)
    print(f"restart {restart}: GPU {int(iters[0, 0])} iterations, oracle {it_o}")
    assert it_o > restart
    assert rel(E[0, 0].ravel(), xs) < 1e-5
    assert abs(int(iters[0, 0]) - it_o) <= 1
    assert fin[0, 0] <= 1e-6
    np.testing.assert_allclose(hist[0, 0, :10], np.array(hist_o[:10]), rtol=2e-3)
    P.close()
    ctx.close()


def test_batched_wavelengths_and_sources_two_level():
    w = random_small(23, 192, 192, [64] * 3, [64] * 3, wavelengths=(0.9, 1.2), n_src=2, npml=12,
                     k_coarse=1, block=16)
    ctx, P = make_gpu_problem(w)
    E, hist, iters, fin, st = P.solve(w.J(), tol=1e-6, restart=30, max_iters=600)
    assert st == 0
    for wi, lam in enumerate(w.wavelengths):
        op = SchwarzProblem(w.eps, lam, w.h, w.npml, w.core_x, w.core_y, w.overlap, k_coarse=1)
        for s in range(2):
            b = source_rhs(w.J()[s], lam)
            xs = solve_direct(op.A, b)
            xo, it_o, hist_o, res_o = op.solve(w.J()[s], tol=1e-6, max_iters=600)
            err_o = rel(xo, xs)
            if err_o <= 5e-6:
                assert rel(E[wi, s].ravel(), xs) < 1e-5
            else:
                # the oracle's own iterate misses x* at this tolerance: compare with
                # its iterate after the GPU's iteration count
                xk, _, _, _ = op.solve(w.J()[s], tol=1e-300, max_iters=int(iters[wi, s]))
                assert rel(E[wi, s].ravel(), xk) < 1e-5, (rel(E[wi, s].ravel(), xk), err_o)
            assert abs(int(iters[wi, s]) - it_o) <= 1, (lam, s, iters[wi, s], it_o)
            assert fin[wi, s] <= 1e-6


@pytest.mark.parametrize("k_coarse,k_trial", [(1, 8), (2, 4)])
def test_coarse_basis_fields_match_oracle(k_coarse, k_trial):
    """Each basis field agrees with the oracle's up to a unit complex factor
    (singular vectors are unique up to phase when the singular values are distinct)."""
    w = random_small(22, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.1,), npml=12, block=16)
    w.k_coarse, w.k_trial = k_coarse, k_trial
    ctx, P = make_gpu_problem(w)
    phis, box = P.coarse_basis(0)
    A, part, locs = oracle_parts(w, 1.1)
    cs = CoarseSpace(part, locs, A, w.eps.astype(np.float64), 1.1, w.h, k_coarse, k_trial)
    Phi = cs.Phi.toarray()
    worst = []
    for col, ti in enumerate(cs.tile_of_col):
        l = col % k_coarse
        bx0, by0, bw, bh = box[ti]
        ref = Phi[:, col].reshape(w.ny, w.nx)[by0:by0 + bh, bx0:bx0 + bw]
        g = phis[ti][l].astype(np.complex128)
        ph = np.vdot(g, ref) / abs(np.vdot(g, ref))
        worst.append((rel(g * ph, ref), ti, l))
    print(sorted(worst)[-5:])
    assert max(worst)[0] < 1e-4, sorted(worst)[-5:]


def uneven():
    """Mixed 96/64 cores: 100 x 100 corner subdomains (short side above the LDS
    factorisation limit), 100 x 72 edge subdomains, 72 x 72 interior ones."""
    return random_small(51, 320, 256, [96, 64, 64, 96], [96, 64, 96], wavelengths=(1.0, 1.2), n_src=3,
                        npml=12, k_coarse=1, block=16)


def test_uneven_subdomains_local_solves_match_sparse_lu():
    w = uneven()
    ctx, P = make_gpu_problem(w, k_coarse=0)
    nt, lc, ne, nc = P.sizes()
    rng = np.random.default_rng(4)
    rhs = (rng.standard_normal((len(w.wavelengths), lc)) + 1j * rng.standard_normal((len(w.wavelengths), lc)))
    u = dev(np.zeros_like(rhs))
    P.local_solve(dev(rhs), u)
    u = host(u)
    worst, shapes = 0.0, set()
    for wi, lam in enumerate(w.wavelengths):
        A, part, locs = oracle_parts(w, lam)
        for t, L in enumerate(locs):
            off = P.tile_info(t)[8]
            n = L.B.shape[0]
            shapes.add((L.t.x1 - L.t.x0, L.t.y1 - L.t.y0))
            worst = max(worst, rel(u[wi, off:off + n], L.solve(rhs[wi, off:off + n])))
    assert (100, 100) in shapes and (100, 72) in shapes and (72, 100) in shapes, shapes
    assert worst < 2e-5, worst


def test_uneven_subdomains_many_sources_solve():
    w = uneven()
    ctx, P = make_gpu_problem(w)
    E, hist, iters, fin, st = P.solve(w.J(), tol=1e-6, restart=30, max_iters=800)
    assert st == 0, (iters, fin)
    for wi, lam in enumerate(w.wavelengths):
        A = assemble_A(w.eps, lam, w.h, w.npml)
        for s in range(len(w.sources)):
            xs = solve_direct(A, source_rhs(w.J()[s], lam))
            assert rel(E[wi, s].ravel(), xs) < 1e-5, (wi, s)
    lam = w.wavelengths[0]
    op = SchwarzProblem(w.eps, lam, w.h, w.npml, w.core_x, w.core_y, w.overlap, k_coarse=1)
    xo, it_o, hist_o, res_o = op.solve(w.J()[0], tol=1e-6)
    assert abs(int(iters[0, 0]) - it_o) <= 1, (int(iters[0, 0]), it_o)
