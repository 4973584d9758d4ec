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


def test_weights_file_reads_back_exactly(tmp_path):
    torch.manual_seed(1)
    model = ft.build_model(C=8, modes=4, layers=2)
    with torch.no_grad():
        for p in model.parameters():
            p.add_(0.05 * torch.randn_like(p))
    ft.round_model_to_bf16(model)
    path = os.path.join(tmp_path, "w.bin")
    ft.write_weights(model, path)
    other = ft.build_model(C=8, modes=4, layers=2)
    ft.read_weights(other, path)
    for p, q in zip(model.parameters(), other.parameters()):
        assert torch.equal(p, q)
    with pytest.raises(ValueError):
        ft.read_weights(ft.build_model(C=8, modes=4, layers=3), path)


def test_residual_clip_keeps_phase_and_bounds_magnitude():
    b = torch.full((1, 2, 2), 2.0 + 0j, dtype=torch.complex128)           # rms(b) = 2
    r = torch.tensor([[[3 + 4j, 0.5j], [-10.0 + 0j, 1 - 1j]]], dtype=torch.complex128)
    out = ft.clip_residual(r, b, 1.5)                                      # limit 3
    exp = torch.tensor([[[0.6 * (3 + 4j), 0.5j], [-3.0 + 0j, 1 - 1j]]], dtype=torch.complex128)
    assert torch.allclose(out, exp, rtol=0, atol=1e-15)


class _Scaled(torch.nn.Module):
    """M(r) = a r: the fixed-point recurrence becomes a Richardson iteration."""

    def __init__(self, a):
        super().__init__()
        self.a = torch.nn.Parameter(torch.tensor(a, dtype=torch.complex128))

    def forward(self, r, aux):
        return self.a * r


def _diag_problem(d, c, n=4):
    coef = torch.zeros((1, 5, n, n), dtype=torch.complex128)
    coef[:, 4] = d                                                          # B = d I
    b = torch.full((1, n, n), c, dtype=torch.complex128)
    return coef, b, b / d


def test_fixed_point_step_is_richardson_without_clipping():
    """B = d I, M(r) = a r, frozen weights: r_j = (1 - a d)^j b, so the relative
    residual after step j is |1 - a d|^j."""
    d, a, c = 2.0 - 0.5j, 0.3 + 0.1j, 1.0 + 2.0j
    coef, b, y = _diag_problem(d, c)
    model = _Scaled(a)
    opt = torch.optim.SGD(model.parameters(), lr=0.0)
    hist = ft.fixed_point_train_step(model, opt, coef, None, b, y, 5, th_clip=1e9)
    q = abs(1 - a * d)
    np.testing.assert_allclose(hist, [q ** j for j in range(1, 6)], rtol=1e-12)


def test_fixed_point_step_clips_the_residual_it_feeds_back():
    """A diverging Richardson step (|1 - a d| = 2.5 > th = 1.5): the residual fed
    to step 2 is clipped to th rms(b) with its phase, so r_2 = (1 - a d) b -
    a d th (1 - a d)/|1 - a d| b and the reported residual is not clipped."""
    d, a, c, th = 1.0 + 0j, 3.5 + 0j, 0.5 - 1.5j, 1.5
    coef, b, y = _diag_problem(d, c)
    model = _Scaled(a)
    opt = torch.optim.SGD(model.parameters(), lr=0.0)
    hist = ft.fixed_point_train_step(model, opt, coef, None, b, y, 2, th_clip=th)
    q = 1 - a * d
    r2 = q - a * d * th * q / abs(q)
    np.testing.assert_allclose(hist, [abs(q), abs(r2)], rtol=1e-12)


def test_fixed_point_training_reduces_the_loss():
    """With the weights free, a few batches of the fixed-point recurrence move
    a towards 1/d (each step's graph ends at its own optimizer step)."""
    d, c = 2.0 + 0j, 1.0 + 0j
    coef, b, y = _diag_problem(d, c)
    model = _Scaled(0.1 + 0j)
    opt = torch.optim.SGD(model.parameters(), lr=0.05)
    first = ft.fixed_point_train_step(model, opt, coef, None, b, y, 3, th_clip=4.0)
    for _ in range(20):
        last = ft.fixed_point_train_step(model, opt, coef, None, b, y, 3, th_clip=4.0)
    assert last[0] < 0.5 * first[0]
    assert abs(model.a.item() - 0.5) < abs(0.1 - 0.5)


def test_modulated_lowrank_weights_roundtrip_and_forward_matches_oracle(tmp_path):
    """The modulated low-rank network (Fig. 2: R from a rank-r factor pair,
    mode-wise modulation from the auxiliary channels) written by the trainer
    (weights file version 2) and read by the oracle gives the same output."""
    torch.manual_seed(2)
    model = ft.build_model(C=8, modes=4, layers=2, rank=3).double()
    with torch.no_grad():
        for p in model.parameters():
            p.add_(0.05 * torch.randn_like(p))
        model.mf2w.add_(0.3 * torch.randn_like(model.mf2w))     # a modulation far from 1
    ft.round_model_to_bf16(model)
    path = os.path.join(tmp_path, "w2.bin")
    ft.write_weights(model, path)
    other = ft.build_model(C=8, modes=4, layers=2, rank=3)
    ft.read_weights(other, path)
    for p, q in zip(model.parameters(), other.parameters()):
        assert torch.equal(p.float(), q)
    w = load_weights(path)
    rng = np.random.default_rng(3)
    for t, lam in ((4, 1.1), (0, 0.9), (5, 1.4)):
        x0, x1, y0, y1, side = ft.tile_box(t)
        eps = rng.uniform(1, 12, (y1 - y0, x1 - x0)).astype(np.float32)
        aux = ft.aux_inputs(t, lam, eps)
        v = (rng.standard_normal(eps.shape) + 1j * rng.standard_normal(eps.shape))
        with torch.no_grad():
            e_t = model(torch.from_numpy(v)[None], torch.from_numpy(aux.astype(np.float64))[None])[0].numpy()
            mod_t = model.modulation(torch.from_numpy(aux.astype(np.float64))[None])[0].numpy()
        from oracle.fno import modulation
        np.testing.assert_allclose(modulation(w, aux.astype(np.float64)), mod_t, rtol=1e-12, atol=1e-12)
        isx = aux[2, 0, :] + 1j * aux[3, 0, :]
        isy = aux[4, :, 0] + 1j * aux[5, :, 0]
        e_o = fno_forward(w, v, eps.astype(np.float64), 2 * np.pi / lam * ft.H, isx.astype(np.complex128),
                          isy.astype(np.complex128), aux[6])
        assert np.linalg.norm(e_t - e_o) <= 1e-5 * np.linalg.norm(e_o)
