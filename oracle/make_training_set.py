"""Write a training set of exactly solved subdomain Robin problems (test and
training infrastructure; it only calls the oracle).

Each sample is one extended subdomain of a 3 x 3 partition (cores of 64, 8-cell
overlap, 12-cell PML) of a 192 x 192 grid with piecewise-constant permittivity
in [1, 12] on blocks of random size, a random wavelength with k0 h in
[0.21, 0.39] (h = 0.05, wavelength in [0.8, 1.5]), random smooth Robin data on
its interface ring and, for half of the samples, a random interior source.
About a quarter of the samples are edge or corner subdomains, which contain
PML.  The local right-hand side is b = R_i f + inj(g) and the stored solution
is y = B_i^-1 b (sparse LU, complex128, stored as complex64).

Output (numpy .npz, no pickled objects), per subdomain position t = 0..8:
  eps_t [n][ly][lx] float32, lam_t [n] float64, b_t, y_t [n][ly][lx] complex64.

Usage: python oracle/make_training_set.py --n 20000 --out /tmp/tiles.npz [--procs 16]
"""
from __future__ import annotations

import argparse
import os
import sys

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"      # one BLAS thread per worker process

import numpy as np            # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.fdfd import assemble_A                     # noqa: E402
from oracle.partition import LocalProblem, Partition   # noqa: E402

N_GLOBAL, CORE, NPML, H, OVERLAP = 192, 64, 12, 0.05, 8


def _smooth_1d(rng, n, width):
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    k = np.exp(-0.5 * (np.arange(-3 * width, 3 * width + 1) / max(width, 1e-3)) ** 2)
    k /= np.sqrt(np.sum(k ** 2))
    return np.convolve(np.concatenate([x, x, x]), k, mode="same")[n:2 * n]


def one_sample(seed):
    rng = np.random.default_rng(seed)
    block = int(rng.choice([4, 8, 16, 32]))
    nb = N_GLOBAL // block
    eps = np.kron(rng.uniform(1, 12, (nb, nb)), np.ones((block, block)))
    lam = float(rng.uniform(0.8, 1.5))
    tile = 4 if rng.uniform() < 0.75 else int(rng.choice([0, 1, 2, 3, 5, 6, 7, 8]))
    A = assemble_A(eps, lam, H, NPML)
    part = Partition(N_GLOBAL, N_GLOBAL, [CORE] * 3, [CORE] * 3, OVERLAP, NPML)
    t = part.tiles[tile]
    L = LocalProblem(part, t, A, eps, 2 * np.pi / lam, H)
    ne = len(L.entries)
    g = _smooth_1d(rng, ne, float(rng.uniform(1, 20))) * float(rng.uniform(0.2, 5.0))
    b = L.inj(g)
    if rng.uniform() < 0.5:
        f = np.zeros((t.ly, t.lx), dtype=np.complex128)
        for _ in range(int(rng.integers(1, 6))):
            cx, cy = rng.integers(0, t.lx), rng.integers(0, t.ly)
            f[cy, cx] += (rng.standard_normal() + 1j * rng.standard_normal()) * 2 * np.pi / lam * 10
        b = b + f.ravel()
    y = L.solve(b)
    e = eps[t.y0:t.y1, t.x0:t.x1]
    return tile, lam, e.astype(np.float32), b.reshape(t.ly, t.lx).astype(np.complex64), \
        y.reshape(t.ly, t.lx).astype(np.complex64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--out", required=True)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1))
    a = ap.parse_args()
    seeds = [a.seed + i for i in range(a.n)]
    if a.procs > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(a.procs) as pool:
            res = []
            for i, r in enumerate(pool.imap(one_sample, seeds, chunksize=16)):
                res.append(r)
                if (i + 1) % 2000 == 0:
                    print(f"[make_training_set] {i + 1}/{a.n}", flush=True)
    else:
        res = [one_sample(s) for s in seeds]
    out = {}
    for t in range(9):
        sel = [r for r in res if r[0] == t]
        if not sel:
            continue
        out[f"eps_{t}"] = np.stack([r[2] for r in sel])
        out[f"lam_{t}"] = np.array([r[1] for r in sel])
        out[f"b_{t}"] = np.stack([r[3] for r in sel])
        out[f"y_{t}"] = np.stack([r[4] for r in sel])
    np.savez(a.out, **out)
    print(f"[make_training_set] wrote {a.out}: " + ", ".join(f"{k}{v.shape}" for k, v in out.items() if k.startswith('eps')),
          flush=True)


if __name__ == "__main__":
    main()
