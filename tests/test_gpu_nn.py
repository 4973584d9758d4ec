"""GPU parity of the neural subdomain path, through the C ABI.

* One network application (BF16 MFMA channel mixes with FP32 accumulation,
  FP32 truncated DFTs) against the oracle's NumPy forward pass in FP64 on the
  same BF16 weights: relative L2 error per subdomain below 3e-2 (BF16 rounding
  of activations at every layer).
* The flexible outer GMRES with the NN-FGMRES subdomain solver converges to
  the tolerance and the field matches the direct solution to 1e-5 whatever
  the quality of the network (the network only changes the iteration count).
"""
import os

import numpy as np
import pytest

from oracle.fdfd import assemble_A, pml_stretch, solve_direct, source_rhs
from oracle.fno import fno_forward, load_weights
from oracle.partition import Partition
from paper_2509_03622_amd.workloads import random_small

from gpu_common import dev, host, rel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAINED = os.path.join(ROOT, "paper_2509_03622_amd", "weights", "fno_c64_m16_l4.bin")


@pytest.fixture(scope="module")
def random_weights(tmp_path_factory):
    torch = pytest.importorskip("torch")
    from paper_2509_03622_amd import fno_train as ft
    torch.manual_seed(3)
    model = ft.build_model(64, 16, 4)
    ft.round_model_to_bf16(model)
    path = str(tmp_path_factory.mktemp("w") / "random.bin")
    ft.write_weights(model, path)
    return path


def _problem(w, weights, steps=2, tol=0.1):
    from paper_2509_03622_amd import nosdd
    ctx = nosdd.Context(0, nosdd.torch_stream_handle())
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths, w.pml_m, w.pml_lnR)
    P.setup(k_coarse=w.k_coarse, k_trial=w.k_trial, sub_solver=1, nn_weights=weights, inner_max=steps, inner_tol=tol)
    return ctx, P


def test_network_application_matches_oracle(random_weights):
    w = random_small(31, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.1,), npml=12, block=16)
    ctx, P = _problem(w, random_weights)
    nt, lc, ne, nc = P.sizes()
    rng = np.random.default_rng(5)
    v = rng.standard_normal((1, lc)) + 1j * rng.standard_normal((1, lc))
    e = dev(np.zeros_like(v))
    P.nn_apply(dev(v), e)
    e = host(e)[0]
    wt = load_weights(random_weights)
    lam = w.wavelengths[0]
    k0 = 2 * np.pi / lam
    sc, _ = pml_stretch(w.nx, w.npml, w.pml_m, w.pml_lnR, k0, w.h)
    part = Partition(w.nx, w.ny, w.core_x, w.core_y, w.overlap, w.npml)
    worst = 0.0
    for t, tile in enumerate(part.tiles):
        off = P.tile_info(t)[8]
        n = tile.lx * tile.ly
        vt = v[0, off:off + n].reshape(tile.ly, tile.lx)
        mask = np.zeros((tile.ly, tile.lx))
        if tile.iface["left"]:
            mask[:, 0] = 1
        if tile.iface["right"]:
            mask[:, -1] = 1
        if tile.iface["bottom"]:
            mask[0, :] = 1
        if tile.iface["top"]:
            mask[-1, :] = 1
        ref = fno_forward(wt, vt, w.eps[tile.y0:tile.y1, tile.x0:tile.x1].astype(np.float64), k0 * w.h,
                          1 / sc[tile.x0:tile.x1], 1 / sc[tile.y0:tile.y1], mask)
        worst = max(worst, rel(e[off:off + n].reshape(tile.ly, tile.lx), ref))
    assert worst < 3e-2, worst


@pytest.mark.parametrize("weights", ["random", "trained"])
def test_nn_fgmres_solve_reaches_direct_solution(weights, random_weights):
    path = random_weights if weights == "random" else TRAINED
    if not os.path.exists(path):
        pytest.skip("trained weights not present")
    w = random_small(32, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.0,), npml=12, k_coarse=1, block=16)
    ctx, P = _problem(w, path, steps=2, tol=0.1)
    E, hist, iters, fin, st = P.solve(w.J(), tol=1e-6, restart=30, max_iters=1500)
    assert st == 0, (iters, fin)
    A = assemble_A(w.eps, 1.0, w.h, w.npml)
    xs = solve_direct(A, source_rhs(w.J()[0], 1.0))
    assert rel(E[0, 0].ravel(), xs) < 1e-5
    print("NN-FGMRES outer iterations", int(iters[0, 0]))
