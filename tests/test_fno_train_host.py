"""Host checks of the offline FNO trainer against the oracle (CPU only):
the trainer's network equals the oracle's NumPy forward pass through a
weights file written by one and read by the other, and the trainer's local
Robin operator equals the oracle's B_i on exactly solved samples."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.fdfd import assemble_A
from oracle.fno import fno_forward, load_weights
from oracle.partition import LocalProblem, Partition
from paper_2509_03622_amd import fno_train as ft


def test_weights_roundtrip_and_forward_matches_oracle(tmp_path):
    torch.manual_seed(0)
    model = ft.build_model(C=8, modes=4, layers=2).double()
    with torch.no_grad():
        for p in model.parameters():
            p.add_(0.05 * torch.randn_like(p))
    ft.round_model_to_bf16(model)
    path = os.path.join(tmp_path, "w.bin")
    ft.write_weights(model, path)
    w = load_weights(path)
    rng = np.random.default_rng(1)
    t, lam = 4, 1.1
    x0, x1, y0, y1, side = ft.tile_box(t)
    eps = rng.uniform(1, 12, (y1 - y0, x1 - x0)).astype(np.float32)
    aux = ft.aux_inputs(t, lam, eps)
    v = (rng.standard_normal(eps.shape) + 1j * rng.standard_normal(eps.shape))
    with torch.no_grad():
        e_t = model(torch.from_numpy(v)[None], torch.from_numpy(aux.astype(np.float64))[None])[0].numpy()
    isx = aux[2, 0, :] + 1j * aux[3, 0, :]
    isy = aux[4, :, 0] + 1j * aux[5, :, 0]
    e_o = fno_forward(w, v, eps.astype(np.float64), 2 * np.pi / lam * ft.H, isx.astype(np.complex128),
                      isy.astype(np.complex128), aux[6])
    assert np.linalg.norm(e_t - e_o) <= 1e-5 * np.linalg.norm(e_o)


@pytest.mark.parametrize("tile", [0, 1, 4, 8])
def test_trainer_operator_equals_oracle_local_matrix(tile):
    rng = np.random.default_rng(tile)
    eps = np.kron(rng.uniform(1, 12, (24, 24)), np.ones((8, 8)))
    lam = 1.3
    A = assemble_A(eps, lam, ft.H, ft.NPML)
    part = Partition(ft.GRID, ft.GRID, [ft.CORE] * 3, [ft.CORE] * 3, 2 * ft.EXT, ft.NPML)
    t = part.tiles[tile]
    L = LocalProblem(part, t, A, eps, 2 * np.pi / lam, ft.H)
    u = rng.standard_normal((t.ly, t.lx)) + 1j * rng.standard_normal((t.ly, t.lx))
    ref = (L.B @ u.ravel()).reshape(t.ly, t.lx)
    coef = ft.local_operator(tile, lam, eps[t.y0:t.y1, t.x0:t.x1])
    out = ft.apply_op(torch.from_numpy(coef)[None], torch.from_numpy(u)[None])[0].numpy()
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)
