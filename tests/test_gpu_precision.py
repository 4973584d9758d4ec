"""Residuals below single precision: the outer FGMRES keeps its iterate and
every restart residual in FP64 (iterative refinement around FP32 Krylov
cycles), so tolerances far below the FP32 rounding level are reached with
FP32 subdomain solves and with the BF16 network preconditioner alike.

* Exact LU subdomain solves: tol 1e-10; the complex64 field's FP64 residual
  stays within the complex64 rounding bound above it, and the FP64 iterate
  returned by nosdd_solve_device_c64 has residual <= 1e-10 itself and matches
  the FP64 direct solution to 1e-8.
* NN-FGMRES subdomain solves (trained network): tol 1e-9, same checks.
"""
import os

import numpy as np
import pytest

from oracle.fdfd import assemble_A, solve_direct, source_rhs
from paper_2509_03622_amd.workloads import random_small, small_rectangles

from gpu_common import make_gpu_problem, rel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAINED = os.path.join(ROOT, "paper_2509_03622_amd", "weights", "fno_c64_m16_l4.bin")


def _check_field(w, lam, E, fin, tol):
    A = assemble_A(w.eps, lam, w.h, w.npml)
    b = source_rhs(w.J()[0], lam)
    xs = solve_direct(A, b)
    x = E.ravel().astype(np.complex128)
    u = np.sqrt(2.0) * 2.0 ** -24 * (1 + 2.0 ** -24)
    res = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    bound = float(fin) * (1 + 1e-6) + u * np.linalg.norm(abs(A) @ abs(x)) / np.linalg.norm(b)
    print(f"explicit residual of the FP64 iterate {fin:.2e}; of the complex64 field {res:.2e} (bound {bound:.2e}); "
          f"field error {rel(x, xs):.2e}")
    assert fin <= tol
    assert res <= bound
    return rel(x, xs)


def _check_fp64(w, lam, P, tol):
    import torch
    J = torch.from_numpy(w.J()).cuda()
    E64 = torch.zeros((1, 1, w.ny, w.nx), dtype=torch.complex128, device="cuda")
    hist, it, fin, st = P.solve_device_c64(J, E64, tol=tol, max_iters=3000)
    assert st == 0, (it, fin)
    x = E64.cpu().numpy()[0, 0].ravel()
    A = assemble_A(w.eps, lam, w.h, w.npml)
    b = source_rhs(w.J()[0], lam)
    res = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    err = rel(x, solve_direct(A, b))
    print(f"FP64 iterate: residual {res:.2e}, field error {err:.2e}")
    assert res <= tol * 1.001
    assert err < 1e-8


def test_exact_lu_reaches_1e10():
    w = small_rectangles()
    ctx, P = make_gpu_problem(w)
    E, hist, it, fin, st = P.solve(w.J(), tol=1e-10, restart=30, max_iters=3000)
    assert st == 0, (it, fin)
    err = _check_field(w, w.wavelengths[0], E[0, 0], fin[0, 0], 1e-10)
    # the complex64 rounding of the returned field limits its error to ~1e-7
    assert err < 1e-6
    _check_fp64(w, w.wavelengths[0], P, 1e-10)


def test_nn_fgmres_reaches_1e9():
    if not os.path.exists(TRAINED):
        pytest.skip("trained weights not present")
    from paper_2509_03622_amd import nosdd
    w = random_small(32, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.0,), npml=12, k_coarse=1, block=16)
    ctx = nosdd.Context(0, nosdd.torch_stream_handle())
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths, w.pml_m, w.pml_lnR)
    P.setup(k_coarse=1, k_trial=8, sub_solver=1, nn_weights=TRAINED, inner_max=8, inner_tol=1e-2)
    E, hist, it, fin, st = P.solve(w.J(), tol=1e-9, restart=30, max_iters=3000)
    assert st == 0, (it, fin)
    print("NN-FGMRES outer iterations to 1e-9:", int(it[0, 0]))
    err = _check_field(w, 1.0, E[0, 0], fin[0, 0], 1e-9)
    assert err < 1e-6
    _check_fp64(w, 1.0, P, 1e-9)


def test_stagnation_stops_the_solve_early():
    """A tolerance below what the FP64 iterate can reach (rounding of the
    operator itself) makes the explicit residual stop decreasing; the solve
    then ends after one cycle without progress instead of running to
    max_iters, and says so."""
    import torch
    w = small_rectangles()
    ctx, P = make_gpu_problem(w)
    J = torch.from_numpy(w.J()).cuda()
    E64 = torch.zeros((1, 1, w.ny, w.nx), dtype=torch.complex128, device="cuda")
    max_iters = 20000
    hist, it, fin, st = P.solve_device_c64(J, E64, tol=1e-18, max_iters=max_iters)
    msg = ctx.L.nosdd_last_error(ctx.h).decode()
    print(f"stopped after {int(it[0, 0])} iterations at {float(fin[0, 0]):.2e}: {msg}")
    assert st == 1
    assert int(it[0, 0]) < max_iters // 4
    assert "did not decrease" in msg
    assert float(fin[0, 0]) < 1e-9
