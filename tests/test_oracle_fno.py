"""Pins of the oracle's FNO forward pass (CPU only): closed-form single-mode
responses of the spectral layer, NumPy FFT agreement of the truncated DFT,
and zero-in/zero-out."""
import numpy as np

from oracle.fno import dft_truncated, fourier_block, fno_forward, idft_truncated, kept_kx


def _mode_field(Lx, Ly, kx, ky):
    y, x = np.mgrid[0:Ly, 0:Lx]
    return 2 * np.pi * (kx * x / Lx + ky * y / Ly)


def test_truncated_dft_matches_fft():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((3, 68, 72))           # [C][Ly][Lx]
    X = dft_truncated(u, 16)
    F = np.fft.fft2(u, axes=(2, 1))                # F[c, ky, kx] layout -> transpose
    F = np.transpose(F, (0, 2, 1))                 # [c][kx][ky]
    ref = F[:, kept_kx(72, 16)][:, :, :16]
    np.testing.assert_allclose(X, ref, rtol=1e-10, atol=1e-9)


def test_inverse_matches_irfft_of_truncated_spectrum():
    rng = np.random.default_rng(1)
    Lx, Ly, m = 72, 68, 16
    X = rng.standard_normal((2, 2 * m, m)) + 1j * rng.standard_normal((2, 2 * m, m))
    full = np.zeros((2, Lx, Ly // 2 + 1), complex)
    full[:, kept_kx(Lx, m), :m] = X
    ref = np.fft.irfft2(full, s=(Lx, Ly), axes=(1, 2))       # [c][x][y]
    out = idft_truncated(X, Lx, Ly, m)
    np.testing.assert_allclose(out, np.transpose(ref, (0, 2, 1)), rtol=1e-10, atol=1e-12)


def test_single_mode_closed_form():
    Lx, Ly, m = 72, 72, 16
    r = 0.7 - 0.4j
    for (kx, ky) in ((3, 5), (-4, 2), (6, 0)):
        th = _mode_field(Lx, Ly, kx, ky)
        u = np.cos(th)[None]
        R = np.full((2 * m, m, 1, 1), r, dtype=complex)
        out = fourier_block(u, R, np.zeros((1, 1)), np.zeros(1), m, act=False)[0]
        if ky > 0:
            ref = np.abs(r) * np.cos(th + np.angle(r))
        else:
            ref = r.real * np.cos(th)
        np.testing.assert_allclose(out, ref, atol=1e-12)
    # a mode outside the kept band is removed entirely
    u = np.cos(_mode_field(Lx, Ly, 20, 3))[None]
    R = np.ones((2 * m, m, 1, 1), complex)
    out = fourier_block(u, R, np.zeros((1, 1)), np.zeros(1), m, act=False)
    assert np.max(np.abs(out)) < 1e-12


def _random_weights(rng, C=8, m=4, L=2):
    w = {"modes": m, "layers": L,
         "lift_w": rng.standard_normal((C, 9)) * 0.3, "lift_b": np.zeros(C),
         "proj1_w": rng.standard_normal((16, C)) * 0.3, "proj1_b": np.zeros(16),
         "proj2_w": rng.standard_normal((2, 16)) * 0.3, "proj2_b": np.zeros(2)}
    for l in range(L):
        w[f"R{l}"] = (rng.standard_normal((2 * m, m, C, C)) + 1j * rng.standard_normal((2 * m, m, C, C))) * 0.01
        w[f"W{l}"] = rng.standard_normal((C, C)) * 0.3
        w[f"b{l}"] = np.zeros(C)
    return w


def test_zero_input_zero_output_and_scale_equivariance():
    rng = np.random.default_rng(2)
    w = _random_weights(rng)
    Ly, Lx = 20, 24
    eps = rng.uniform(1, 12, (Ly, Lx))
    isx = np.ones(Lx, complex)
    isy = np.ones(Ly, complex)
    mask = np.zeros((Ly, Lx))
    z = fno_forward(w, np.zeros((Ly, Lx), complex), eps, 0.3, isx, isy, mask)
    assert np.all(z == 0)
    v = rng.standard_normal((Ly, Lx)) + 1j * rng.standard_normal((Ly, Lx))
    e1 = fno_forward(w, v, eps, 0.3, isx, isy, mask)
    e2 = fno_forward(w, 5.0 * v, eps, 0.3, isx, isy, mask)
    np.testing.assert_allclose(e2, 5.0 * e1, rtol=1e-12)      # the rms normalisation


def test_bf16_rounding_matches_torch_bfloat16():
    """The emulation's rounding equals torch's float32 -> bfloat16 conversion
    (round to nearest, ties to even), ties and signs included."""
    import torch
    from oracle.fno import round_bf16
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-8, 8, 20000)).astype(np.float32)
    # exact ties: a bfloat16 value plus half an ulp, with even and odd last bits
    base = rng.integers(0x3000, 0x5000, 2000).astype(np.uint32) << 16       # finite bfloat16 values
    ties = (base | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties, np.float32([0.0, -0.0, 1.0, 3.0e38])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_bf16(x), ref)
    z = x[:100] + 1j * x[100:200]
    np.testing.assert_array_equal(round_bf16(z), ref[:100] + 1j * ref[100:200])
