"""Failure handling through the C ABI (GPU context needed; no kernel is made to fail)."""
import numpy as np
import pytest

from paper_2509_03622_amd.workloads import random_small

pytestmark = pytest.mark.gpu


def _ctx():
    from paper_2509_03622_amd import nosdd
    return nosdd, nosdd.Context(0, nosdd.torch_stream_handle())


def test_invalid_partitions_are_rejected():
    nosdd, ctx = _ctx()
    eps = np.ones((128, 128), np.float32)
    with pytest.raises(nosdd.NosddError) as e:
        nosdd.Problem(ctx, eps, 0.05, 12, [64, 63], [64, 64], 8, [1.0])
    assert e.value.status == -4
    with pytest.raises(nosdd.NosddError) as e:
        nosdd.Problem(ctx, eps, 0.05, 12, [8, 120], [64, 64], 8, [1.0])     # interface inside the PML
    assert e.value.status == -4
    with pytest.raises(nosdd.NosddError) as e:
        nosdd.Problem(ctx, eps, 0.05, 12, [64, 64], [64, 64], 7, [1.0])     # odd overlap
    assert e.value.status == -4
    for v in (np.nan, 0.0, -2.0):               # kappa = k0 sqrt(eps) must be real
        bad = eps.copy()
        bad[3, 3] = v
        with pytest.raises(nosdd.NosddError) as e:
            nosdd.Problem(ctx, bad, 0.05, 12, [64, 64], [64, 64], 8, [1.0])
        assert e.value.status == -1


def test_grid_beyond_the_cell_limit_is_rejected():
    # 2^15 x 2^14 = 2^29 cells, the smallest grid past the limit; rejected before eps is read
    import ctypes as C
    nosdd, ctx = _ctx()
    L = ctx.L
    eps = np.ones(16, np.float32)
    g = nosdd.Grid(1 << 15, 1 << 14, 0.05, 12, 2, -30.0)
    cx, cy = (C.c_int * 1)(1 << 15), (C.c_int * 1)(1 << 14)
    part = nosdd.PartitionSpec(cx, 1, cy, 1, 8)
    wl = np.ones(1, np.float64)
    hp = C.c_void_p()
    st = L.nosdd_problem_create(ctx.h, C.byref(g), eps.ctypes.data, C.byref(part), wl.ctypes.data, 1, C.byref(hp))
    assert st == -1 and not hp.value
    assert b"too large" in L.nosdd_last_error(ctx.h)


def test_solve_before_setup_and_missing_weights():
    nosdd, ctx = _ctx()
    w = random_small(40, 128, 128, [64, 64], [64, 64])
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths)
    with pytest.raises(nosdd.NosddError) as e:
        P.solve(w.J())
    assert e.value.status == -8
    with pytest.raises(nosdd.NosddError) as e:
        P.setup(sub_solver=1, nn_weights=None)
    assert e.value.status == -7
    with pytest.raises(nosdd.NosddError) as e:
        P.setup(sub_solver=1, nn_weights="/nonexistent/weights.bin")
    assert e.value.status == -7


def test_unreachable_tolerance_reports_not_converged():
    nosdd, ctx = _ctx()
    w = random_small(41, 128, 128, [64, 64], [64, 64])
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths)
    P.setup()
    E, hist, iters, fin, st = P.solve(w.J(), tol=1e-6, max_iters=3)
    assert st == 1 and int(iters[0, 0]) == 3 and fin[0, 0] > 1e-6
    assert np.all(hist[0, 0, :3] > 0)


def test_zero_source_gives_zero_field_without_iterations():
    nosdd, ctx = _ctx()
    w = random_small(42, 128, 128, [64, 64], [64, 64])
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths)
    P.setup()
    E, hist, iters, fin, st = P.solve(np.zeros((1, 128, 128), np.complex64))
    assert st == 0 and int(iters[0, 0]) == 0 and np.all(E == 0)


def test_repeated_solves_are_bit_identical():
    nosdd, ctx = _ctx()
    w = random_small(43, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.0, 1.3), k_coarse=1, block=16)
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths)
    P.setup(k_coarse=1)
    E1, h1, i1, f1, _ = P.solve(w.J())
    E2, h2, i2, f2, _ = P.solve(w.J())
    assert np.array_equal(E1, E2) and np.array_equal(h1, h2) and np.array_equal(i1, i2)


def test_graph_replay_is_bit_identical_to_eager_launch():
    """The captured per-step graphs replay the eager kernel sequence exactly:
    fields, residual histories and iteration counts agree bit for bit, over
    several solves in a row with eager work and synchronisations in between."""
    import torch
    from paper_2509_03622_amd import nosdd
    w = random_small(41, 192, 160, [64, 64, 64], [80, 80], wavelengths=(0.9, 1.3), n_src=2, k_coarse=1)
    ctx = nosdd.Context(0, nosdd.torch_stream_handle())
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths, w.pml_m, w.pml_lnR)
    P.setup(k_coarse=1, k_trial=8)
    P.graphs(False)
    E0, h0, it0, f0, s0 = P.solve(w.J(), tol=1e-6, restart=30, max_iters=600)
    assert s0 == 0
    P.graphs(True)
    for rep in range(3):
        E1, h1, it1, f1, s1 = P.solve(w.J(), tol=1e-6, restart=30, max_iters=600)
        assert s1 == 0
        assert np.array_equal(it0, it1), (rep, it0, it1)
        assert np.array_equal(h0, h1), rep
        assert np.array_equal(E0, E1), rep
        x = torch.ones(4, device="cuda")           # unrelated eager work between replays
        torch.cuda.synchronize()
        del x
    P.close()
    ctx.close()


def test_autotuned_launch_parameters_keep_the_result():
    """The autotuner only picks among launch parameters with the same
    arithmetic: the tuned solve reaches the same field as the defaults."""
    from paper_2509_03622_amd import nosdd
    w = random_small(42, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.1,), n_src=2, k_coarse=1)
    ctx = nosdd.Context(0, nosdd.torch_stream_handle())
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths, w.pml_m, w.pml_lnR)
    P.setup(k_coarse=1, k_trial=8)
    P.autotune(False)
    E0, h0, it0, f0, s0 = P.solve(w.J(), tol=1e-6, restart=30, max_iters=600)
    t0 = P.tuning()
    assert not t0["tuned_gram_schmidt"] and not t0["tuned_subdomain_solve"]
    P.autotune(True)
    E1, h1, it1, f1, s1 = P.solve(w.J(), tol=1e-6, restart=30, max_iters=600)
    t1 = P.tuning()
    assert t1["tuned_gram_schmidt"] and t1["tuned_subdomain_solve"], t1
    assert t1["solve_prefetch_depth"] in (3, 4, 5)
    assert all(v > 0 for v in t1["gs_workgroups_per_rhs"])
    assert s0 == 0 and s1 == 0
    assert np.all(np.abs(it0 - it1) <= 1), (it0, it1)
    assert np.linalg.norm(E1 - E0) <= 2e-6 * np.linalg.norm(E0)
    P.close()
    ctx.close()


def test_single_subdomain_is_an_exact_solve():
    """One subdomain covering the grid (no interfaces, no Robin data, no coarse
    space): the preconditioner is the exact inverse, so FGMRES converges in one
    iteration, Algorithm 3 in one sweep, both to the direct solution."""
    import torch
    from gpu_common import make_gpu_problem, rel
    from oracle.fdfd import assemble_A, solve_direct, source_rhs
    w = random_small(44, 64, 64, [64], [64], wavelengths=(1.0, 1.3), npml=8, k_coarse=1)
    ctx, P = make_gpu_problem(w)
    assert P.sizes()[2] == 0 and P.sizes()[3] == 0          # no interface entries, no coarse columns
    E, hist, it, fin, st = P.solve(w.J(), tol=1e-6, max_iters=50)
    assert st == 0 and np.all(it == 1), it
    J = torch.from_numpy(w.J()).cuda()
    E2 = torch.zeros((2, 1, 64, 64), dtype=torch.complex64, device="cuda")
    hist2, it2, fin2, st2 = P.solve_paper(J, E2, tol=1e-5, max_iters=5)
    assert st2 == 0 and np.all(it2 == 1), it2
    E2 = E2.cpu().numpy()
    for wi, lam in enumerate(w.wavelengths):
        xs = solve_direct(assemble_A(w.eps, lam, w.h, w.npml), source_rhs(w.J()[0], lam))
        assert rel(E[wi, 0].ravel(), xs) < 1e-5
        assert rel(E2[wi, 0].ravel(), xs) < 1e-5
    P.close()
    ctx.close()
