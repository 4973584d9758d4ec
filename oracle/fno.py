"""NumPy forward pass of the subdomain Fourier neural operator (oracle).

Test infrastructure only.  Architecture (Fig. 2 of the paper): lift (1x1) ->
L Fourier blocks -> project (1x1, 1x1).  Two variants share every convention
below: the plain network (a dense complex R per block) and the modulated
low-rank network of Fig. 2 (``modulation``/``lowrank`` below: R built from a
low-dimensional tensor by a linear expansion over the kept modes, and the
spectral product of every block multiplied mode by mode by a tensor that a
small convolution / pooling / fully connected path computes from the
auxiliary inputs alone).

Each Fourier block computes  u <- act(W u + b + F^-1(R . F(u)))  where F is the
2D DFT of each channel truncated to the low modes, R a complex channel mix per
kept mode, W a 1x1 channel mix and act the leaky ReLU (identity after the
last block).  Conventions, shared with the weights file:

* arrays are [channel][y][x]; the tile is Lx x Ly cells;
* forward DFT  X[kx,ky] = sum_{x,y} u[y,x] exp(-2 pi i (kx x/Lx + ky y/Ly)),
  kept modes kx in {0..m-1} U {Lx-m..Lx-1} (stored in that order), ky in {0..m-1};
* inverse  u[y,x] = 1/(Lx Ly) sum_{kept} c_ky Re(X[kx,ky] exp(+2 pi i (...)))
  with c_0 = 1 and c_ky = 2 for ky >= 1 (real-signal Hermitian completion);
* spectral mix  Y[o,kx,ky] = sum_i X[i,kx,ky] R[kx,ky,i,o];
* input channels: Re v/s, Im v/s (s = rms of v over the tile), (eps-1)/11,
  k0 h sqrt(eps), Re/Im(1/s_x), Re/Im(1/s_y), interface-ring mask;
* output e = (o_0 + i o_1) * s.

Arithmetic is float64 on float32 weights.  Parity of the trained behaviour is
unpinned (no values printed in the paper); the forward map itself is pinned
in the tests.
"""
from __future__ import annotations

import numpy as np

LEAKY = 0.01


def leaky(x):
    return np.where(x >= 0, x, LEAKY * x)


def kept_kx(Lx, m):
    return np.concatenate([np.arange(m), np.arange(Lx - m, Lx)])


def dft_truncated(u, m):
    """u [C][Ly][Lx] real -> X [C][2m][m] complex (kx major, ky minor)."""
    C, Ly, Lx = u.shape
    kx = kept_kx(Lx, m)
    ky = np.arange(m)
    Ex = np.exp(-2j * np.pi * np.outer(np.arange(Lx), kx) / Lx)     # [x][kx]
    Ey = np.exp(-2j * np.pi * np.outer(np.arange(Ly), ky) / Ly)     # [y][ky]
    X = np.zeros((C, 2 * m, m), dtype=np.complex128)
    for c in range(C):
        X[c] = Ex.T @ u[c].T @ Ey          # sum_x sum_y Ex[x,kx] u[y,x] Ey[y,ky]
    return X


def idft_truncated(X, Lx, Ly, m):
    """X [C][2m][m] -> u [C][Ly][Lx] real, Hermitian completion along ky."""
    C = X.shape[0]
    kx = kept_kx(Lx, m)
    ky = np.arange(m)
    cky = np.where(ky == 0, 1.0, 2.0)
    Ex = np.exp(2j * np.pi * np.outer(kx, np.arange(Lx)) / Lx)      # [kx][x]
    Ey = np.exp(2j * np.pi * np.outer(ky, np.arange(Ly)) / Ly)      # [ky][y]
    out = np.zeros((C, Ly, Lx))
    for c in range(C):
        full = Ey.T @ (X[c] * cky[None, :]).T @ Ex                 # [y][x]
        out[c] = full.real / (Lx * Ly)
    return out


def round_bf16(a):
    """Round to the nearest bfloat16 (ties to even) through float32, returned as float64.

    Used only by the BF16 emulation of the forward pass: a matrix-core
    product with BF16 operands and FP32 accumulation sees exactly these
    operand values."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return round_bf16(a.real) + 1j * round_bf16(a.imag)
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def fourier_block(u, R, W, bias, m, act=True, bf16=False, mod=None):
    """One block: act(W u + b + F^-1(mod . (R . F(u)))).  R [2m][m][Cin][Cout]
    complex; mod [2m][m] complex (None: no modulation).

    bf16: the block's input u is rounded to bfloat16 (activations stored in
    bfloat16 between blocks), and so are the truncated spectrum X and R
    before their product, as a matrix-core implementation with BF16 operands
    sees them, and the inverse-transform term before it joins the 1 x 1 mix
    (it is stored in bfloat16 between the two stages); the transforms, sums
    and bias stay exact."""
    C, Ly, Lx = u.shape
    if bf16:
        u = round_bf16(u)              # activations are stored in bfloat16 between blocks
    X = dft_truncated(u, m)
    if bf16:
        X = round_bf16(X)
        R = round_bf16(R)              # a no-op for weights stored in bfloat16
    Y = np.einsum("ikq,kqio->okq", X, R)
    if mod is not None:
        Y = Y * mod[None]
    spec = idft_truncated(Y, Lx, Ly, m)
    if bf16:
        spec = round_bf16(spec)        # stored in bfloat16 for the pointwise stage
    pw = np.einsum("oi,iyx->oyx", W, round_bf16(u) if bf16 else u) + bias[:, None, None]
    out = pw + spec
    return leaky(out) if act else out


def expand_lowrank(A, B):
    """R[k][i][o] = sum_r A[k][r] B[r][i][o]: the linear layer A (rank r -> the
    kept modes k, complex) applied to the low-dimensional tensor B (Fig. 2
    caption; Sec. 2.1, low-rank parameterisation of R).  A [2m][m][r],
    B [r][Cin][Cout] -> R [2m][m][Cin][Cout]."""
    return np.einsum("xyr,rio->xyio", A, B)


def adaptive_avg_pool(a, P):
    """Average of a [C][Ly][Lx] over a P x P grid of bins; bin (p, q) covers
    rows floor(p Ly / P) .. floor((p+1) Ly / P) - 1 and the same for columns."""
    C, Ly, Lx = a.shape
    out = np.zeros((C, P, P))
    for p in range(P):
        y0, y1 = (p * Ly) // P, ((p + 1) * Ly) // P
        for q in range(P):
            x0, x1 = (q * Lx) // P, ((q + 1) * Lx) // P
            out[:, p, q] = a[:, y0:y1, x0:x1].mean(axis=(1, 2))
    return out


def conv3x3(a, w, b):
    """Zero-padded 3 x 3 convolution (cross-correlation): a [Cin][Ly][Lx],
    w [Cout][Cin][3][3], b [Cout] -> [Cout][Ly][Lx]."""
    Cin, Ly, Lx = a.shape
    ap = np.pad(a, ((0, 0), (1, 1), (1, 1)))
    out = np.zeros((w.shape[0], Ly, Lx)) + b[:, None, None]
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oi,iyx->oyx", w[:, :, dy, dx], ap[:, dy:dy + Ly, dx:dx + Lx])
    return out


def modulation(weights, aux):
    """Modulation tensor of every block from the seven auxiliary channels
    aux [7][Ly][Lx] (Fig. 2: convolution, pooling and fully connected layers):
    leaky(conv3x3) -> P x P average pool -> leaky(FC) -> FC, read as
    mod[l][kx][ky] = 1 + (o_re + i o_im) (identity when the path outputs 0)."""
    w = weights
    L, m = int(w["layers"]), int(w["modes"])
    h = leaky(conv3x3(aux, w["mod_conv_w"], w["mod_conv_b"]))
    p = adaptive_avg_pool(h, int(w["mod_pool"])).ravel()
    f = leaky(w["mod_fc1_w"] @ p + w["mod_fc1_b"])
    o = (w["mod_fc2_w"] @ f + w["mod_fc2_b"]).reshape(L, 2 * m, m, 2)
    return 1.0 + o[..., 0] + 1j * o[..., 1]


def build_inputs(v, eps, k0h, inv_sx, inv_sy, ring_mask):
    """The 9 input channels for a local residual v [Ly][Lx] (complex)."""
    s = np.sqrt(np.mean(np.abs(v) ** 2))
    vn = v / s if s > 0 else v * 0
    Ly, Lx = v.shape
    ch = [vn.real, vn.imag, (eps - 1.0) / 11.0, k0h * np.sqrt(eps),
          np.broadcast_to(inv_sx.real[None, :], (Ly, Lx)),
          np.broadcast_to(inv_sx.imag[None, :], (Ly, Lx)),
          np.broadcast_to(inv_sy.real[:, None], (Ly, Lx)),
          np.broadcast_to(inv_sy.imag[:, None], (Ly, Lx)),
          ring_mask.astype(np.float64)]
    return np.stack(ch).astype(np.float64), s


def fno_forward(weights, v, eps, k0h, inv_sx, inv_sy, ring_mask, bf16=False):
    """Apply the network to one local residual v [Ly][Lx]; returns e [Ly][Lx] complex.

    bf16=True is the emulation of a BF16 matrix-core forward pass: every
    activation tensor between blocks is rounded to bfloat16 (it is stored so),
    and so are the operands of every learned channel mix (spectral mix, 1x1
    mix, first projection); everything else is exact (the lift and the last
    projection are not matrix-core products; the transforms are, but on
    operands split into two BF16 parts, within about 2^-16 of exact)."""
    wt = {k: np.asarray(a, dtype=np.float64) if not np.iscomplexobj(a) else np.asarray(a, np.complex128)
          for k, a in weights.items()}
    m = int(weights["modes"])
    nl = int(weights["layers"])
    x, s = build_inputs(v, eps, k0h, inv_sx, inv_sy, ring_mask)
    if s == 0:
        return np.zeros_like(v, dtype=np.complex128)
    mod = modulation(wt, x[2:]) if "mod_conv_w" in wt else None
    u = np.einsum("oi,iyx->oyx", wt["lift_w"], x) + wt["lift_b"][:, None, None]
    for l in range(nl):
        u = fourier_block(u, wt[f"R{l}"], wt[f"W{l}"], wt[f"b{l}"], m, act=(l < nl - 1), bf16=bf16,
                          mod=None if mod is None else mod[l])
    p = leaky(np.einsum("oi,iyx->oyx", wt["proj1_w"], round_bf16(u) if bf16 else u)
              + wt["proj1_b"][:, None, None])
    o = np.einsum("oi,iyx->oyx", wt["proj2_w"], p) + wt["proj2_b"][:, None, None]
    return (o[0] + 1j * o[1]) * s


def load_weights(path):
    """Read a weights file ("NOSDDFNO" header, bfloat16 tensors) into the dict
    fno_forward takes (float32 values, complex R)."""
    import struct
    with open(path, "rb") as f:
        raw = f.read()
    if raw[:8] != b"NOSDDFNO":
        raise ValueError("not a weights file")
    version, C, m, L, in_ch, hidden, dtype = struct.unpack("<7i", raw[8:36])
    if version not in (1, 2) or dtype != 1:
        raise ValueError("unsupported weights file version/dtype")
    hdr = 36
    if version == 2:
        rank, mod_ch, mod_pool, mod_hidden = struct.unpack("<4i", raw[36:52])
        hdr = 52
    bits = np.frombuffer(raw[hdr:], dtype=np.uint16)
    vals = (bits.astype(np.uint32) << 16).view(np.float32)
    pos = [0]

    def take(*shape):
        n = int(np.prod(shape))
        out = vals[pos[0]:pos[0] + n].reshape(shape)
        pos[0] += n
        return out
    w = {"modes": m, "layers": L, "lift_w": take(C, in_ch), "lift_b": take(C)}
    for l in range(L):
        if version == 1:
            rr = take(2 * m, m, C, C)
            ri = take(2 * m, m, C, C)
            w[f"R{l}"] = rr.astype(np.float64) + 1j * ri.astype(np.float64)
        else:
            # low-rank R: the network's spectral weights are the expansion of the
            # stored (bfloat16) factors; the BF16 emulation rounds it like any
            # other matrix-core operand
            Ar, Ai = take(2 * m, m, rank), take(2 * m, m, rank)
            Br, Bi = take(rank, C, C), take(rank, C, C)
            w[f"A{l}"] = Ar.astype(np.float64) + 1j * Ai.astype(np.float64)
            w[f"B{l}"] = Br.astype(np.float64) + 1j * Bi.astype(np.float64)
            w[f"R{l}"] = expand_lowrank(w[f"A{l}"], w[f"B{l}"])
        w[f"W{l}"] = take(C, C)
        w[f"b{l}"] = take(C)
    w["proj1_w"] = take(hidden, C)
    w["proj1_b"] = take(hidden)
    w["proj2_w"] = take(2, hidden)
    w["proj2_b"] = take(2)
    if version == 2:
        w["mod_pool"] = mod_pool
        w["mod_conv_w"] = take(mod_ch, 7, 3, 3)
        w["mod_conv_b"] = take(mod_ch)
        w["mod_fc1_w"] = take(mod_hidden, mod_ch * mod_pool * mod_pool)
        w["mod_fc1_b"] = take(mod_hidden)
        w["mod_fc2_w"] = take(L * 2 * m * m * 2, mod_hidden)
        w["mod_fc2_b"] = take(L * 2 * m * m * 2)
    if pos[0] != vals.size:
        raise ValueError("weights file size does not match its header")
    return w
