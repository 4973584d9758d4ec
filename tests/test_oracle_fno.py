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


# ------------------------------------------------------------ modulated low-rank network
def test_lowrank_expansion_index_order():
    """R[k][i][o] = sum_r A[k][r] B[r][i][o]: rank one is the outer product, and
    the mix through the expanded R equals the factored evaluation
    sum_r A[k][r] (X[k] B[r]) that never forms R."""
    from oracle.fno import expand_lowrank
    rng = np.random.default_rng(11)
    m, C, r = 3, 5, 4
    cplx = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    A1, B1 = cplx(2 * m, m, 1), cplx(1, C, C)
    np.testing.assert_allclose(expand_lowrank(A1, B1), np.multiply.outer(A1[..., 0], B1[0]), rtol=1e-13)
    A, B = cplx(2 * m, m, r), cplx(r, C, C)
    R = expand_lowrank(A, B)
    X = cplx(C, 2 * m, m)                            # [i][kx][ky] as in fourier_block
    Y_dense = np.einsum("ikq,kqio->okq", X, R)
    Y_fact = np.zeros((C, 2 * m, m), complex)
    for kx in range(2 * m):
        for ky in range(m):
            for rr in range(r):
                Y_fact[:, kx, ky] += A[kx, ky, rr] * (X[:, kx, ky] @ B[rr])
    np.testing.assert_allclose(Y_dense, Y_fact, rtol=1e-12, atol=1e-12)


def test_adaptive_pool_bins_by_hand():
    from oracle.fno import adaptive_avg_pool
    for Ly, Lx in ((72, 72), (68, 52)):
        y, x = np.mgrid[0:Ly, 0:Lx].astype(float)
        out = adaptive_avg_pool(np.stack([y, x, np.full((Ly, Lx), 2.5)]), 4)
        rows = [np.arange((p * Ly) // 4, ((p + 1) * Ly) // 4).mean() for p in range(4)]
        cols = [np.arange((q * Lx) // 4, ((q + 1) * Lx) // 4).mean() for q in range(4)]
        np.testing.assert_allclose(out[0], np.repeat(np.array(rows)[:, None], 4, 1), rtol=1e-14)
        np.testing.assert_allclose(out[1], np.repeat(np.array(cols)[None, :], 4, 0), rtol=1e-14)
        np.testing.assert_allclose(out[2], 2.5, rtol=1e-14)
    # 72 / 4: bins of 18 rows, centres 8.5, 26.5, 44.5, 62.5
    np.testing.assert_allclose(adaptive_avg_pool(np.mgrid[0:72, 0:4][0][None].astype(float), 4)[0][:, 0],
                               [8.5, 26.5, 44.5, 62.5])


def test_conv3x3_matches_library_correlation():
    """Zero-padded 3 x 3 cross-correlation: each (out, in) pair equals
    scipy.signal.correlate2d(mode='same'); a centre tap is the identity."""
    from scipy.signal import correlate2d
    from oracle.fno import conv3x3
    rng = np.random.default_rng(12)
    a = rng.standard_normal((3, 11, 9))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    out = conv3x3(a, w, b)
    for o in range(2):
        ref = b[o] + sum(correlate2d(a[i], w[o, i], mode="same") for i in range(3))
        np.testing.assert_allclose(out[o], ref, rtol=1e-12, atol=1e-12)
    eye = np.zeros((3, 3, 3, 3))
    for i in range(3):
        eye[i, i, 1, 1] = 1.0
    np.testing.assert_allclose(conv3x3(a, eye, np.zeros(3)), a, rtol=0, atol=0)


def _mod_weights(m=2, L=2, mc=3, P=2, mh=4):
    return {"modes": m, "layers": L, "mod_pool": P,
            "mod_conv_w": np.zeros((mc, 7, 3, 3)), "mod_conv_b": np.zeros(mc),
            "mod_fc1_w": np.zeros((mh, mc * P * P)), "mod_fc1_b": np.zeros(mh),
            "mod_fc2_w": np.zeros((L * 2 * m * m * 2, mh)), "mod_fc2_b": np.zeros(L * 2 * m * m * 2)}


def test_modulation_single_channel_closed_form():
    """Only aux channel 0 (constant c) feeds one centre tap (weight w0, bias
    b0) and one hidden unit (weight f); every output is g times that unit:
    mod = 1 + g_re leaky(f leaky(w0 c + b0)) + i g_im leaky(...)."""
    from oracle.fno import leaky, modulation
    m, L = 2, 2
    wt = _mod_weights(m, L)
    c, w0, b0, f = 0.37, -1.7, 0.2, 2.3
    wt["mod_conv_w"][0, 0, 1, 1] = w0
    wt["mod_conv_b"][0] = b0
    wt["mod_fc1_w"][0, 0] = f                        # feature (channel 0, bin 0)
    g = np.random.default_rng(13).standard_normal(L * 2 * m * m * 2)
    wt["mod_fc2_w"][:, 0] = g
    aux = np.zeros((7, 12, 10))
    aux[0] = c
    h = f * leaky(np.array(w0 * c + b0))
    hval = float(leaky(np.array(h)))
    o = (g * hval).reshape(L, 2 * m, m, 2)
    mod = modulation(wt, aux)
    np.testing.assert_allclose(mod, 1.0 + o[..., 0] + 1j * o[..., 1], rtol=1e-14)
    # a path that outputs zero is the identity modulation
    assert np.all(modulation(_mod_weights(m, L), aux) == 1.0)


def test_modulated_single_mode_closed_form():
    """A single kept Fourier mode through a modulated block is multiplied by
    mod[k] r (the unmodulated closed form with r -> mod[k] r)."""
    Lx, Ly, m = 72, 68, 16
    r = 0.7 - 0.4j
    rng = np.random.default_rng(14)
    mod = rng.standard_normal((2 * m, m)) + 1j * rng.standard_normal((2 * m, m))
    for (kx, ky) in ((3, 5), (-4, 2), (6, 0)):
        th = _mode_field(Lx, Ly, kx, ky)
        u = np.cos(th)[None]
        R = np.full((2 * m, m, 1, 1), r, dtype=complex)
        out = fourier_block(u, R, np.zeros((1, 1)), np.zeros(1), m, act=False, mod=mod)[0]
        col = lambda k: k if k >= 0 else 2 * m + k             # storage position of kx
        rr = mod[col(kx), ky] * r
        if ky > 0:       # one kept mode; its conjugate partner comes from the Hermitian completion
            ref = np.abs(rr) * np.cos(th + np.angle(rr))
        else:            # (kx, 0) and (-kx, 0) are both kept, each with its own modulation
            rm = mod[col(-kx), 0] * r
            ref = 0.5 * (np.real(rr * np.exp(1j * th)) + np.real(rm * np.exp(-1j * th)))
        np.testing.assert_allclose(out, ref, atol=1e-12)
