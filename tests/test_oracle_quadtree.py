"""Pins of the oracle on general (non-tensor) partitions: quad-tree cores with
T-junctions, where one side of a subdomain borders two smaller neighbours
(Methods, partitioner: arbitrary arrangements of subdomains that cover the
domain, e.g. a quad-tree that splits quadrants larger than about five
wavelengths).

* the quad-tree generator follows its rule on a case worked by hand (48-cell
  cores in eps 1.5, 24-cell cores over the eps 6..8 block) and on the 512 x 512
  workload (64-cell cores in vacuum, 32 over the high-index square);
* an explicit core list equal to a tensor partition gives the same tiles;
  gaps, overlaps and too-small cores are rejected;
* the neighbour set of a refined subdomain at a T-junction, worked by hand;
* the Robin identity B_i R_i u = R_i A u + inj(g(u)) on every subdomain, and
  the local problems reproduce the global solution (exact algebra);
* the stationary sweep equals the volume step x + M1^-1 (b - A x);
* the coarse correction is a least-squares minimiser (W^H t = 0) and the
  two-level FGMRES reaches the direct solution;
* the Algorithm 3 loop with the Robin-space coarse correction converges to
  the direct solution, and an error inside span Q is removed in one step.
"""
import numpy as np
import pytest

from oracle.coarse import two_level_apply
from oracle.fdfd import assemble_A, solve_direct, source_rhs
from oracle.paper_loop import RobinCoarse, paper_loop, sweep, traces
from oracle.partition import Partition, PartitionError, build_local_problems, oras_apply
from oracle.schwarz import SchwarzProblem
from paper_2509_03622_amd.workloads import quadtree_512, random_quadtree


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def qt():
    w = random_quadtree(1)
    P = SchwarzProblem(w.eps, 1.0, w.h, w.npml, None, None, w.overlap, k_coarse=2, cores=w.cores)
    b = source_rhs(w.J()[0], 1.0)
    return w, P, b, solve_direct(P.A, b)


def test_quadtree_rule_worked_by_hand():
    w = random_quadtree(1)
    # eps 1.5: 5 local wavelengths = 5 / sqrt(1.5) / 0.05 = 81.6 cells, so the
    # 96-cell quadrants split once more only because of the 48-cell cap; the
    # quadrant [48, 96)^2 holds eps >= 6 (5 local wavelengths <= 40.8 cells
    # < 48) and splits into four 24-cell cores; 24 < 2 * 16 stops there
    sizes = sorted((c[1] - c[0], c[3] - c[2]) for c in w.cores)
    assert sizes == [(24, 24)] * 4 + [(48, 48)] * 15
    assert sorted(c for c in w.cores if c[1] - c[0] == 24) == [
        (48, 72, 48, 72), (48, 72, 72, 96), (72, 96, 48, 72), (72, 96, 72, 96)]
    part = Partition.from_cores(w.nx, w.ny, w.cores, w.overlap, w.npml)
    assert np.all(part.owner >= 0)


def test_quadtree_512_rule():
    w = quadtree_512()
    small = [c for c in w.cores if c[1] - c[0] == 32]
    big = [c for c in w.cores if c[1] - c[0] == 64]
    assert len(small) == 64 and len(big) == 48 and len(w.cores) == 112
    assert all(128 <= c[0] and c[1] <= 384 and 128 <= c[2] and c[3] <= 384 for c in small)
    assert all(not (128 <= c[0] and c[1] <= 384 and 128 <= c[2] and c[3] <= 384) for c in big)
    Partition.from_cores(w.nx, w.ny, w.cores, w.overlap, w.npml)


def test_core_list_equals_tensor_partition():
    a = Partition(192, 160, [64, 60, 68], [96, 64], 8, npml=12)
    cores = [(t.cx0, t.cx1, t.cy0, t.cy1) for t in a.tiles]
    b = Partition.from_cores(192, 160, cores, 8, npml=12)
    for ta, tb in zip(a.tiles, b.tiles):
        assert (ta.x0, ta.x1, ta.y0, ta.y1, ta.iface) == (tb.x0, tb.x1, tb.y0, tb.y1, tb.iface)
        assert a.trace_entries(ta) == b.trace_entries(tb)
    for i in range(len(a.tiles)):
        # in a tensor partition with wide cores the neighbours are the 3 x 3 stencil
        t = a.tiles[i]
        exp = sorted(j for j, u in enumerate(a.tiles) if j != i and abs(u.tx - t.tx) <= 1 and abs(u.ty - t.ty) <= 1)
        assert a.neighbours(i) == exp == b.neighbours(i)


def test_core_list_validation():
    good = [(0, 64, 0, 128), (64, 128, 0, 64), (64, 128, 64, 128)]
    Partition.from_cores(128, 128, good, 8, npml=12)
    with pytest.raises(PartitionError):       # a gap
        Partition.from_cores(128, 128, good[:2], 8, npml=12)
    with pytest.raises(PartitionError):       # an overlap
        Partition.from_cores(128, 128, good + [(60, 70, 60, 70)], 8, npml=12)
    with pytest.raises(PartitionError):       # a core thinner than overlap/2 + 1
        Partition.from_cores(128, 128, [(0, 64, 0, 128), (64, 68, 0, 128), (68, 128, 0, 128)], 8, npml=0)
    with pytest.raises(PartitionError):       # an interface inside the PML
        Partition.from_cores(128, 128, [(0, 8, 0, 128), (8, 128, 0, 128)], 8, npml=12)
    with pytest.raises(PartitionError):       # outside the grid
        Partition.from_cores(128, 128, [(0, 130, 0, 128)], 8)


def test_t_junction_neighbours(qt):
    w, P, b, xs = qt
    part = P.part
    i = w.cores.index((48, 72, 48, 72))
    # its extended tile [44, 76)^2 meets the three 48-cell cores below and to
    # the left of the refined quadrant (extended tiles reach 52 or 44..100)
    # and the other three 24-cell cores; nothing beyond x or y = 96
    exp = {w.cores.index(c) for c in [(0, 48, 0, 48), (48, 96, 0, 48), (0, 48, 48, 96),
                                       (72, 96, 48, 72), (48, 72, 72, 96), (72, 96, 72, 96)]}
    assert set(part.neighbours(i)) == exp
    # the right side of core (0, 48, 48, 96) borders two refined cores
    t = part.tiles[w.cores.index((0, 48, 48, 96))]
    right = {part.owner[y, t.cx1] for y in range(t.cy0, t.cy1)}
    assert right == {w.cores.index((48, 72, 48, 72)), w.cores.index((48, 72, 72, 96))}


def test_quadtree_robin_identity_every_tile(qt):
    w, P, b, xs = qt
    rng = np.random.default_rng(5)
    u = rng.standard_normal(w.nx * w.ny) + 1j * rng.standard_normal(w.nx * w.ny)
    Au = P.A @ u
    for L in P.locs:
        lhs = L.B @ L.restrict(u)
        rhs = L.restrict(Au) + L.inj(L.trace_of_global(u))
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)


def test_quadtree_local_problems_reproduce_global_solution(qt):
    w, P, b, xs = qt
    for L in P.locs:
        u = L.solve(L.restrict(b) + L.inj(L.trace_of_global(xs)))
        assert rel(u, L.restrict(xs)) < 1e-10


def test_quadtree_sweep_is_volume_step(qt):
    w, P, b, xs = qt
    rng = np.random.default_rng(3)
    xp = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
    x, _ = sweep(P.locs, b, traces(P.locs, xp))
    assert rel(x, xp + oras_apply(P.locs, b - P.A @ xp)) < 1e-10


def test_quadtree_coarse_least_squares_and_fgmres(qt):
    w, P, b, xs = qt
    cs = P.cs
    assert cs.nc == 2 * len(w.cores)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
    z, Az = two_level_apply(P.locs, P.A, cs, v)
    t = v - Az
    assert np.linalg.norm(cs.W.conj().T @ t) <= 1e-10 * np.linalg.norm(v) * np.linalg.norm(cs.W.toarray())
    x, it, hist, res = P.solve(w.J()[0], tol=1e-9, max_iters=400)
    assert res <= 1e-9 and rel(x, xs) < 1e-6


def test_quadtree_paper_loop(qt):
    w, P, b, xs = qt
    rc = RobinCoarse(P.cs, P.locs)
    # an error of the Robin data inside span Q is removed by one iteration
    gs = traces(P.locs, xs)
    z0 = np.random.default_rng(7).standard_normal(rc.nc) + 0j
    g = gs + rc.Q @ z0
    x, gn = sweep(P.locs, b, g)
    assert rel(0.3 * g + 0.7 * gn + rc.correction(gn - g, 0.3), gs) < 1e-10
    x, n, hist, g = paper_loop(P.locs, P.A, b, momentum=0.3, coarse=rc, tol=1e-6, max_iters=300)
    assert n < 300 and hist[-1] <= 1e-6 and rel(x, xs) < 1e-5


def test_quadtree_two_way_split_worked_by_hand():
    """160 x 32 vacuum, cores of at most 48 cells and halves of at least 16:
    the root splits four ways into 80 x 16 quadrants; those are still longer
    than 48 but their 16-cell height cannot be halved, so each splits in two
    along x into 40 x 16 leaves."""
    from paper_2509_03622_amd.workloads import quadtree_cores
    cores = quadtree_cores(160, 32, np.ones((32, 160)), 0.05, 1.0, min_core=16, max_core=48)
    assert cores == [(0, 40, 0, 16), (40, 80, 0, 16), (80, 120, 0, 16), (120, 160, 0, 16),
                     (0, 40, 16, 32), (40, 80, 16, 32), (80, 120, 16, 32), (120, 160, 16, 32)]
    Partition.from_cores(160, 32, cores, 8, npml=0)
