"""Offline trainer of the subdomain Fourier neural operator (PyTorch-ROCm).

Training follows the paper's recurrent flexible-GMRES scheme (Algorithm 1,
training branch): for each batch of subdomain problems B_i x = b the network
is the preconditioner of an FGMRES run of N steps; after every step the loss
c_r ||b - B x_j||^2 + c_d ||x_j - y||^2 (relative, per sample) is
back-propagated and the optimizer steps, then the Krylov quantities (basis,
preconditioned directions, Hessenberg entries) are detached.

``--scheme fixed-point`` trains with the fixed-point recurrence instead
(Algorithm 2): from x = 0, N times e = M(r), x <- x + e, r = b - B x, the
same loss, an optimizer step, and the residual fed to the next step is
detached and clipped.  Clipping reading: every complex entry of r whose
magnitude exceeds th_clip * rms(b) (per sample) is scaled down to that
magnitude with its phase kept; the fixed-point recurrence diverges on these
indefinite problems while the network is still poor, and the clip bounds
what it is fed.

The data are exactly solved subdomain problems written by the oracle's
training-set script (an .npz of eps, wavelength, right-hand side and solution
per subdomain position of a 3 x 3 partition of a 192 x 192 grid, cores of 64,
overlap 8, 12-cell PML, h = 0.05).  The local Robin operator used for the
physics loss is built here from the same definitions (5-point UPML stencil,
midpoint Robin closure on interface sides).

Network (shared conventions with the HIP inference kernels and the oracle):
input channels [Re v/s, Im v/s, (eps-1)/11, k0 h sqrt(eps), Re/Im 1/s_x,
Re/Im 1/s_y, interface-ring mask] with s = rms(v); lift 9 -> C; L Fourier
blocks act(W u + b + F^-1(R . F u)) with kept modes kx in {0..m-1} U
{Lx-m..Lx-1}, ky in {0..m-1}, leaky ReLU 0.01 (identity after the last
block); projection C -> 128 (leaky) -> 2; output (o0 + i o1) * s.

Weights file: "NOSDDFNO" magic, int32 header [version=1, C, modes, layers,
in_ch=9, hidden=128, dtype=1 (bf16)], then bfloat16 tensors in order
lift_w[C][9], lift_b[C], per layer R_re[2m][m][C][C], R_im[2m][m][C][C],
W[C][C], b[C], then proj1_w[128][C], proj1_b[128], proj2_w[2][128], proj2_b[2].

Usage: python -m paper_2509_03622_amd.fno_train --data tiles.npz --out weights.bin [--minutes 15]
       [--scheme fixed-point --clip 4] [--init weights.bin (continue from a weights file)]
"""
from __future__ import annotations

import argparse
import math
import os
import struct
import time

import numpy as np

GRID, CORE, EXT, NPML, H = 192, 64, 4, 12, 0.05
PML_M, PML_LNR = 2, -30.0
IN_CH, HIDDEN = 9, 128
MAGIC = b"NOSDDFNO"


# ----------------------------------------------------------------- geometry and operator
def tile_box(t):
    """Extended box and interface sides of position t (ty*3+tx) in the 3 x 3 partition."""
    tx, ty = t % 3, t // 3
    cx0, cy0 = CORE * tx, CORE * ty
    left, right, bottom, top = tx > 0, tx < 2, ty > 0, ty < 2
    x0 = cx0 - EXT if left else cx0
    x1 = cx0 + CORE + EXT if right else cx0 + CORE
    y0 = cy0 - EXT if bottom else cy0
    y1 = cy0 + CORE + EXT if top else cy0 + CORE
    return x0, x1, y0, y1, dict(left=left, right=right, bottom=bottom, top=top)


def stretch_profiles(n, k0):
    """Cell-centre and face stretches of a UPML of NPML cells on each side (exp(+i w t))."""
    sh = (PML_M + 1) * (-PML_LNR) / (2.0 * k0 * NPML * H)

    def s(q):
        d = np.clip(np.maximum(NPML - 0.5 - q, q - (n - NPML - 0.5)) / NPML, 0.0, 1.0)
        return 1.0 - 1j * sh * d ** PML_M
    c = np.arange(n, dtype=np.float64)
    return s(c), s(c - 0.5), s(c + 0.5)


def local_operator(t, lam, eps_tile):
    """Stencil coefficients (cm_x, cp_x, cm_y, cp_y, diag) of B_i, each [ly][lx] complex."""
    x0, x1, y0, y1, side = tile_box(t)
    k0 = 2 * np.pi / lam
    sc, sm, sp = stretch_profiles(GRID, k0)
    cxm = -1.0 / (sm * sc * H * H)
    cxp = -1.0 / (sp * sc * H * H)
    xs, ys = np.arange(x0, x1), np.arange(y0, y1)
    ly, lx = y1 - y0, x1 - x0
    cmx = np.broadcast_to(cxm[xs][None, :], (ly, lx)).astype(np.complex128)
    cpx = np.broadcast_to(cxp[xs][None, :], (ly, lx)).astype(np.complex128)
    cmy = np.broadcast_to(cxm[ys][:, None], (ly, lx)).astype(np.complex128)
    cpy = np.broadcast_to(cxp[ys][:, None], (ly, lx)).astype(np.complex128)
    eps = eps_tile.astype(np.float64)
    diag = -(cmx + cpx + cmy + cpy) - k0 * k0 * eps
    kap = k0 * np.sqrt(eps)
    rho = (1 - 0.5j * kap * H) / (1 + 0.5j * kap * H)
    diag = diag.copy()
    if side["left"]:
        diag[:, 0] += cmx[:, 0] * rho[:, 0]
    if side["right"]:
        diag[:, -1] += cpx[:, -1] * rho[:, -1]
    if side["bottom"]:
        diag[0, :] += cmy[0, :] * rho[0, :]
    if side["top"]:
        diag[-1, :] += cpy[-1, :] * rho[-1, :]
    return np.stack([cmx, cpx, cmy, cpy, diag])


def aux_inputs(t, lam, eps_tile):
    """Seven constant input channels [(eps-1)/11, k0h sqrt(eps), Re/Im 1/s_x, Re/Im 1/s_y, ring mask]."""
    x0, x1, y0, y1, side = tile_box(t)
    k0 = 2 * np.pi / lam
    sc, _, _ = stretch_profiles(GRID, k0)
    ly, lx = y1 - y0, x1 - x0
    isx = 1.0 / sc[x0:x1]
    isy = 1.0 / sc[y0:y1]
    mask = np.zeros((ly, lx))
    if side["left"]:
        mask[:, 0] = 1
    if side["right"]:
        mask[:, -1] = 1
    if side["bottom"]:
        mask[0, :] = 1
    if side["top"]:
        mask[-1, :] = 1
    eps = eps_tile.astype(np.float64)
    return np.stack([(eps - 1) / 11.0, k0 * H * np.sqrt(eps),
                     np.broadcast_to(isx.real[None, :], (ly, lx)), np.broadcast_to(isx.imag[None, :], (ly, lx)),
                     np.broadcast_to(isy.real[:, None], (ly, lx)), np.broadcast_to(isy.imag[:, None], (ly, lx)),
                     mask]).astype(np.float32)


# ----------------------------------------------------------------- model
MOD_CH, MOD_POOL, MOD_HIDDEN = 8, 4, 64


def pool_bins(a, P):
    """Average of a [B][C][Ly][Lx] over a P x P grid of bins, bin (p, q) covering
    rows floor(p Ly / P) .. floor((p+1) Ly / P) - 1 (and the same for columns)."""
    import torch
    Ly, Lx = a.shape[-2:]
    rows = []
    for p in range(P):
        y0, y1 = (p * Ly) // P, ((p + 1) * Ly) // P
        rows.append(torch.stack([a[..., y0:y1, (q * Lx) // P:((q + 1) * Lx) // P].mean(dim=(-1, -2))
                                 for q in range(P)], dim=-1))
    return torch.stack(rows, dim=-2)


def build_model(C=64, modes=16, layers=4, hidden=HIDDEN, rank=0):
    """rank = 0: the plain network (dense complex R per block).  rank > 0: the
    modulated low-rank network of Fig. 2: R_l = sum_r A_l[k][r] B_l[r] (a
    linear expansion over the kept modes of a rank-r tensor) and the spectral
    product multiplied mode by mode by mod_l = 1 + (o_re + i o_im), where o
    comes from the auxiliary channels through leaky(conv 3x3, MOD_CH
    channels) -> MOD_POOL x MOD_POOL average pool -> leaky(FC, MOD_HIDDEN) -> FC."""
    import torch
    import torch.nn as nn

    class FNO(nn.Module):
        def __init__(self):
            super().__init__()
            self.C, self.m, self.L, self.rank = C, modes, layers, rank
            g = 1.0 / math.sqrt(C)
            self.lift_w = nn.Parameter(torch.randn(C, IN_CH) / math.sqrt(IN_CH))
            self.lift_b = nn.Parameter(torch.zeros(C))
            if rank == 0:
                self.Rr = nn.ParameterList([nn.Parameter(torch.randn(2 * modes, modes, C, C) * g / C)
                                            for _ in range(layers)])
                self.Ri = nn.ParameterList([nn.Parameter(torch.randn(2 * modes, modes, C, C) * g / C)
                                            for _ in range(layers)])
            else:
                a = 1.0 / math.sqrt(rank)
                self.Ar = nn.ParameterList([nn.Parameter(torch.randn(2 * modes, modes, rank) * a) for _ in range(layers)])
                self.Ai = nn.ParameterList([nn.Parameter(torch.randn(2 * modes, modes, rank) * a) for _ in range(layers)])
                self.Br = nn.ParameterList([nn.Parameter(torch.randn(rank, C, C) * g / C) for _ in range(layers)])
                self.Bi = nn.ParameterList([nn.Parameter(torch.randn(rank, C, C) * g / C) for _ in range(layers)])
                nf = MOD_CH * MOD_POOL * MOD_POOL
                self.mcw = nn.Parameter(torch.randn(MOD_CH, 7, 3, 3) / math.sqrt(63))
                self.mcb = nn.Parameter(torch.zeros(MOD_CH))
                self.mf1w = nn.Parameter(torch.randn(MOD_HIDDEN, nf) / math.sqrt(nf))
                self.mf1b = nn.Parameter(torch.zeros(MOD_HIDDEN))
                self.mf2w = nn.Parameter(torch.zeros(layers * 2 * modes * modes * 2, MOD_HIDDEN))
                self.mf2b = nn.Parameter(torch.zeros(layers * 2 * modes * modes * 2))
            self.W = nn.ParameterList([nn.Parameter(torch.randn(C, C) * g) for _ in range(layers)])
            self.b = nn.ParameterList([nn.Parameter(torch.zeros(C)) for _ in range(layers)])
            self.p1w = nn.Parameter(torch.randn(hidden, C) * g)
            self.p1b = nn.Parameter(torch.zeros(hidden))
            self.p2w = nn.Parameter(torch.randn(2, hidden) / math.sqrt(hidden) * 0.1)
            self.p2b = nn.Parameter(torch.zeros(2))

        def spectral_weights(self, l):
            if self.rank == 0:
                return torch.complex(self.Rr[l], self.Ri[l])      # [kx][ky][Cin][Cout]
            A = torch.complex(self.Ar[l], self.Ai[l])
            B = torch.complex(self.Br[l], self.Bi[l])
            return torch.einsum("xyr,rio->xyio", A, B)

        def modulation(self, aux):
            """[B][L][2m][m] complex from the auxiliary channels aux [B][7][Ly][Lx]."""
            import torch.nn.functional as Fn
            h = Fn.leaky_relu(Fn.conv2d(aux, self.mcw, self.mcb, padding=1), 0.01)
            p = pool_bins(h, MOD_POOL).flatten(1)
            f = Fn.leaky_relu(p @ self.mf1w.t() + self.mf1b, 0.01)
            o = (f @ self.mf2w.t() + self.mf2b).reshape(-1, self.L, 2 * self.m, self.m, 2)
            return torch.complex(1.0 + o[..., 0], o[..., 1])

        def spectral(self, u, l, mod=None):
            Bn, C, Ly, Lx = u.shape
            m = self.m
            F = torch.fft.rfftn(u, dim=(-1, -2))                 # [B][C][Ly/2+1][Lx], halved along y
            kx = torch.cat([torch.arange(m), torch.arange(Lx - m, Lx)]).to(u.device)
            X = F[:, :, :m, :][:, :, :, kx]                      # [B][C][ky][kx]
            X = X.permute(0, 3, 2, 1)                            # [B][kx][ky][C]
            R = self.spectral_weights(l)                          # [kx][ky][Cin][Cout]
            Y = torch.einsum("bxyi,xyio->bxyo", X, R)
            if mod is not None:
                Y = Y * mod[:, l, :, :, None]
            full = torch.zeros(Bn, C, Ly // 2 + 1, Lx, dtype=F.dtype, device=u.device)
            full[:, :, :m, kx] = Y.permute(0, 3, 2, 1)
            return torch.fft.irfftn(full, s=(Lx, Ly), dim=(-1, -2))

        def forward(self, v, aux):
            """v [B][Ly][Lx] complex, aux [B][7][Ly][Lx] -> e [B][Ly][Lx] complex."""
            import torch.nn.functional as Fn
            s = torch.sqrt(torch.mean(torch.abs(v) ** 2, dim=(-1, -2), keepdim=True)).clamp_min(1e-30)
            vn = v / s
            x = torch.cat([vn.real[:, None], vn.imag[:, None], aux], dim=1)
            mod = self.modulation(aux) if self.rank > 0 else None
            u = torch.einsum("oi,biyx->boyx", self.lift_w, x) + self.lift_b[None, :, None, None]
            for l in range(self.L):
                pw = torch.einsum("oi,biyx->boyx", self.W[l], u) + self.b[l][None, :, None, None]
                u = pw + self.spectral(u, l, mod)
                if l < self.L - 1:
                    u = Fn.leaky_relu(u, 0.01)
            p = Fn.leaky_relu(torch.einsum("oi,biyx->boyx", self.p1w, u) + self.p1b[None, :, None, None], 0.01)
            o = torch.einsum("oi,biyx->boyx", self.p2w, p) + self.p2b[None, :, None, None]
            return torch.complex(o[:, 0], o[:, 1]) * s

    return FNO()


def apply_op(coef, u):
    """B u for stencil coefficients coef [B][5][Ly][Lx] (zero field outside the tile)."""
    import torch
    out = coef[:, 4] * u
    out = out + coef[:, 0] * torch.nn.functional.pad(u[..., :-1], (1, 0))
    out = out + coef[:, 1] * torch.nn.functional.pad(u[..., 1:], (0, 1))
    out = out + coef[:, 2] * torch.nn.functional.pad(u[..., :-1, :], (0, 0, 1, 0))
    out = out + coef[:, 3] * torch.nn.functional.pad(u[..., 1:, :], (0, 0, 0, 1))
    return out


# ----------------------------------------------------------------- weights I/O
def bf16_bits(a):
    """Round float32 -> bfloat16 (nearest even) and return the uint16 bit patterns."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def _ordered_params(model):
    """Parameters in weights-file order (version 1: plain; version 2: modulated low rank)."""
    params = [model.lift_w, model.lift_b]
    for l in range(model.L):
        if model.rank == 0:
            params += [model.Rr[l], model.Ri[l]]
        else:
            params += [model.Ar[l], model.Ai[l], model.Br[l], model.Bi[l]]
        params += [model.W[l], model.b[l]]
    params += [model.p1w, model.p1b, model.p2w, model.p2b]
    if model.rank > 0:
        params += [model.mcw, model.mcb, model.mf1w, model.mf1b, model.mf2w, model.mf2b]
    return params


def _header(model):
    ver = 1 if model.rank == 0 else 2
    h = struct.pack("<7i", ver, model.C, model.m, model.L, IN_CH, HIDDEN, 1)
    if ver == 2:
        h += struct.pack("<4i", model.rank, MOD_CH, MOD_POOL, MOD_HIDDEN)
    return h


def write_weights(model, path):
    t = lambda p: p.detach().float().cpu().numpy()
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(_header(model))
        for p in _ordered_params(model):
            f.write(bf16_bits(t(p)).tobytes())


def read_weights(model, path):
    """Load a weights file written by write_weights into a model of the same shape."""
    import torch
    hdr = _header(model)
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError(f"{path}: not a weights file")
        got = f.read(len(hdr))
        if got != hdr:
            raise ValueError(f"{path}: header does not match the model")
        raw = np.frombuffer(f.read(), dtype=np.uint16)
    params = _ordered_params(model)
    off = 0
    with torch.no_grad():
        for p in params:
            n = p.numel()
            vals = (raw[off:off + n].astype(np.uint32) << 16).view(np.float32).reshape(tuple(p.shape))
            p.copy_(torch.from_numpy(vals.copy()))
            off += n
    if off != raw.size:
        raise ValueError(f"{path}: {raw.size - off} trailing values")


def round_model_to_bf16(model):
    import torch
    with torch.no_grad():
        for p in model.parameters():
            p.copy_(torch.from_numpy(bf16_bits(p.detach().float().cpu().numpy()).astype(np.uint32) << 16)
                    .view(torch.float32).reshape(p.shape))


# ----------------------------------------------------------------- training
class Data:
    def __init__(self, path, device):
        import torch
        d = np.load(path)
        self.groups = []
        for t in range(9):
            if f"eps_{t}" not in d:
                continue
            eps, lam, b, y = d[f"eps_{t}"], d[f"lam_{t}"], d[f"b_{t}"], d[f"y_{t}"]
            self.groups.append(dict(t=t, eps=eps, lam=lam, b=b, y=y, n=len(lam)))
        self.device = device
        self.total = sum(g["n"] for g in self.groups)
        self.torch = torch

    def batch(self, rng, bs, held_out=False):
        """A batch from one subdomain position; the last 1/40 of every position is held out."""
        torch = self.torch
        w = np.array([g["n"] for g in self.groups], dtype=float)
        g = self.groups[rng.choice(len(self.groups), p=w / w.sum())]
        n_tr = max(1, g["n"] - max(1, g["n"] // 40))
        lo, hi = (n_tr, g["n"]) if held_out and n_tr < g["n"] else (0, n_tr)
        idx = rng.integers(lo, hi, size=bs)
        coef = np.stack([local_operator(g["t"], g["lam"][i], g["eps"][i]) for i in idx])
        aux = np.stack([aux_inputs(g["t"], g["lam"][i], g["eps"][i]) for i in idx])
        dev = self.device
        return (torch.from_numpy(coef.astype(np.complex64)).to(dev), torch.from_numpy(aux).to(dev),
                torch.from_numpy(g["b"][idx]).to(dev), torch.from_numpy(g["y"][idx]).to(dev))


def fgmres_train_step(model, opt, coef, aux, b, y, N, c_r=1.0, c_d=0.1):
    """One batch of the recurrent FGMRES training; returns per-step relative residuals."""
    import torch
    Bn = b.shape[0]
    nrm = lambda a: torch.sqrt(torch.sum(torch.abs(a) ** 2, dim=(-1, -2)))
    bn = nrm(b)
    yn = nrm(y)
    V = [b / bn[:, None, None]]
    Z = []
    Hc = torch.zeros(Bn, N + 1, N, dtype=b.dtype, device=b.device)
    hist = []
    for j in range(N):
        opt.zero_grad(set_to_none=True)
        z = model(V[j], aux)
        w = apply_op(coef, z)
        hcol = []
        for i in range(j + 1):
            h = torch.sum(torch.conj(V[i]) * w, dim=(-1, -2))
            w = w - h[:, None, None] * V[i]
            hcol.append(h)
        hn = nrm(w)
        Hj = Hc.detach().clone()
        Hj[:, :j + 1, j] = torch.stack(hcol, dim=1)
        Hj[:, j + 1, j] = hn.to(b.dtype)
        Hbar = Hj[:, :j + 2, :j + 1]
        rhs = torch.zeros(Bn, j + 2, dtype=b.dtype, device=b.device)
        rhs[:, 0] = bn.to(b.dtype)
        G = torch.conj(Hbar.transpose(1, 2)) @ Hbar
        G = G + 1e-12 * torch.eye(j + 1, device=b.device, dtype=b.dtype) * torch.abs(G).amax(dim=(1, 2), keepdim=True)
        coefs = torch.linalg.solve(G, (torch.conj(Hbar.transpose(1, 2)) @ rhs[..., None]))[..., 0]
        x = z * coefs[:, j, None, None]
        for i in range(j):
            x = x + Z[i] * coefs[:, i, None, None]
        r = b - apply_op(coef, x)
        rel_r = nrm(r) / bn
        loss = c_r * torch.mean(rel_r ** 2) + c_d * torch.mean((nrm(x - y) / yn) ** 2)
        loss.backward()
        torch.nn.utils.clip_grad_norm_(model.parameters(), 1.0)
        opt.step()
        hist.append(rel_r.detach().mean().item())
        Z.append(z.detach())
        Hc = Hj.detach()
        V.append((w / hn[:, None, None]).detach())
    return hist


def clip_residual(r, b, th_clip):
    """Entries of r with |r| > th_clip * rms(b) (per sample) scaled to that magnitude, phase kept."""
    import torch
    rms = torch.sqrt(torch.mean(torch.abs(b) ** 2, dim=(-1, -2)))
    lim = (th_clip * rms)[:, None, None]
    mag = torch.abs(r)
    scale = torch.where(mag > lim, lim / torch.clamp(mag, min=torch.finfo(mag.dtype).tiny), torch.ones_like(mag))
    return r * scale


def fixed_point_train_step(model, opt, coef, aux, b, y, N, th_clip, c_r=1.0, c_d=0.1):
    """One batch of the fixed-point training (Algorithm 2); returns per-step relative residuals."""
    import torch
    nrm = lambda a: torch.sqrt(torch.sum(torch.abs(a) ** 2, dim=(-1, -2)))
    bn = nrm(b)
    yn = nrm(y)
    x = torch.zeros_like(b)
    r = b
    hist = []
    for j in range(N):
        opt.zero_grad(set_to_none=True)
        x = x + model(r, aux)                 # earlier updates carry no graph (detached below)
        res = b - apply_op(coef, x)
        rel_r = nrm(res) / bn
        loss = c_r * torch.mean(rel_r ** 2) + c_d * torch.mean((nrm(x - y) / yn) ** 2)
        loss.backward()
        torch.nn.utils.clip_grad_norm_(model.parameters(), 1.0)
        opt.step()
        hist.append(rel_r.detach().mean().item())
        x = x.detach()
        r = clip_residual(res.detach(), b, th_clip)
    return hist


def evaluate(model, data, rng, steps=30, n=32):
    """NN-FGMRES on held-out samples: residual after step 1, and steps to 1e-6 (float32)."""
    import torch
    coef, aux, b, y = data.batch(rng, n, held_out=True)
    with torch.no_grad():
        Bn = b.shape[0]
        nrm = lambda a: torch.sqrt(torch.sum(torch.abs(a) ** 2, dim=(-1, -2)))
        bn = nrm(b)
        V = [b / bn[:, None, None]]
        Z = []
        H = torch.zeros(Bn, steps + 1, steps, dtype=b.dtype, device=b.device)
        res = []
        for j in range(steps):
            z = model(V[j], aux)
            w = apply_op(coef, z)
            for _ in range(2):
                for i in range(j + 1):
                    h = torch.sum(torch.conj(V[i]) * w, dim=(-1, -2))
                    w = w - h[:, None, None] * V[i]
                    H[:, i, j] += h
            hn = nrm(w)
            H[:, j + 1, j] = hn.to(b.dtype)
            Z.append(z)
            V.append(w / hn[:, None, None])
            Hbar = H[:, :j + 2, :j + 1]
            rhs = torch.zeros(Bn, j + 2, dtype=b.dtype, device=b.device)
            rhs[:, 0] = bn.to(b.dtype)
            sol = torch.linalg.lstsq(Hbar.cpu(), rhs[..., None].cpu()).solution[..., 0].to(b.device)
            x = sum(Z[i] * sol[:, i, None, None] for i in range(j + 1))
            res.append((nrm(b - apply_op(coef, x)) / bn).cpu().numpy())
        res = np.array(res)            # [steps][Bn]
    below = (res <= 1e-6)
    first = np.where(below.any(0), below.argmax(0) + 1, steps + 1)
    return float(np.median(res[0])), float(np.median(first)), res


def evaluate_many(model, data, seed, batches=16, n=32, steps=30):
    """evaluate() over several held-out batches drawn from a fixed seed, pooled
    (16 x 32 = 512 subdomains by default): median residual after 1, 2, 4, 8
    and 16 NN-FGMRES steps, and the median number of steps to 1e-3, 1e-5 and
    1e-6 (steps + 1 when not reached)."""
    rng = np.random.default_rng(seed)
    res = np.concatenate([evaluate(model, data, rng, steps, n)[2] for _ in range(batches)], axis=1)
    out = {"samples": res.shape[1]}
    for k in (1, 2, 4, 8, 16):
        out[f"res_after_{k}"] = float(np.median(res[k - 1]))
    for t in (1e-3, 1e-5, 1e-6):
        below = res <= t
        out[f"steps_to_{t:g}"] = float(np.median(np.where(below.any(0), below.argmax(0) + 1, steps + 1)))
    return out


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--data", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--minutes", type=float, default=15.0)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--recurrence", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--width", type=int, default=64)
    ap.add_argument("--modes", type=int, default=16)
    ap.add_argument("--layers", type=int, default=4)
    ap.add_argument("--rank", type=int, default=0,
                    help="0: plain network; r > 0: modulated network with rank-r spectral weights (Fig. 2)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--scheme", choices=("fgmres", "fixed-point"), default="fgmres",
                    help="recurrent FGMRES training (Algorithm 1) or fixed-point training with clipping (Algorithm 2)")
    ap.add_argument("--clip", type=float, default=4.0,
                    help="fixed-point scheme: clip threshold th_clip, in units of rms(b) per sample")
    ap.add_argument("--init", default=None, metavar="WEIGHTS",
                    help="start from these weights (a file of the same network shape) instead of random ones")
    ap.add_argument("--eval", nargs="+", metavar="WEIGHTS",
                    help="only evaluate these weights files on the same held-out batches (no training)")
    a = ap.parse_args()
    dev = torch.device("cuda" if torch.cuda.is_available() else "cpu")
    torch.manual_seed(a.seed)
    rng = np.random.default_rng(a.seed)
    data = Data(a.data, dev)
    if a.eval:
        for path in a.eval:
            model = build_model(a.width, a.modes, a.layers, rank=a.rank).to(dev)
            read_weights(model, path)
            ev = evaluate_many(model, data, seed=12345)
            print(f"[fno_train] eval {path}: " + ", ".join(f"{k} {v:.3g}" for k, v in ev.items()), flush=True)
        return
    model = build_model(a.width, a.modes, a.layers, rank=a.rank).to(dev)
    if a.init:
        read_weights(model, a.init)
    n_par = sum(p.numel() for p in model.parameters())
    print(f"[fno_train] {'modulated rank-%d' % a.rank if a.rank else 'plain'} network, {n_par} weights",
          flush=True)
    opt = torch.optim.Adam(model.parameters(), lr=a.lr)
    t0 = time.time()
    it = 0
    budget = a.minutes * 60
    last = t0
    while time.time() - t0 < budget:
        frac = (time.time() - t0) / budget
        for g in opt.param_groups:
            g["lr"] = a.lr * (0.02 + 0.98 * 0.5 * (1 + math.cos(math.pi * frac)))
        coef, aux, b, y = data.batch(rng, a.batch)
        if a.scheme == "fgmres":
            hist = fgmres_train_step(model, opt, coef, aux, b, y, a.recurrence)
        else:
            hist = fixed_point_train_step(model, opt, coef, aux, b, y, a.recurrence, a.clip)
        it += 1
        if time.time() - last > 30:
            last = time.time()
            print(f"[fno_train] {time.time() - t0:6.0f}s batches {it} rel.res per step "
                  + " ".join(f"{h:.2e}" for h in hist), flush=True)
    round_model_to_bf16(model)
    write_weights(model, a.out)
    r1, steps, _ = evaluate(model, data, rng)
    print(f"[fno_train] done ({a.scheme}): {it} batches; held-out median residual after 1 step {r1:.3e}, "
          f"median steps to 1e-6 {steps:.0f}; weights -> {a.out}", flush=True)


if __name__ == "__main__":
    main()
