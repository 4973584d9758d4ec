"""Writes uneven2048_reference.npz: the direct solution x* = A^-1 b of the
2048 x 1536 workload (wavelength 1.0; sources 0 and 17) at 4096 seeded grid
points, for the GPU field check of the full-size 64-RHS solve.

Calls only the oracle (Eq. 1 operator with UPML, SuperLU direct solve) on the
seeded synthetic inputs; a full field is 50 MB, so only samples are stored,
with the norms the check needs.  About 5 minutes and 13 GB on one host core:

    python tests/golden/make_uneven2048_reference.py
"""
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as spla

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
from oracle.fdfd import assemble_A, rel_residual, source_rhs  # noqa: E402
from paper_2509_03622_amd.workloads import uneven_2048x1536  # noqa: E402

WAVELENGTH_INDEX = 0
SOURCES = (0, 17)
N_SAMPLES = 4096
SEED = 2048


def main():
    w = uneven_2048x1536()
    lam = w.wavelengths[WAVELENGTH_INDEX]
    J = w.J()
    A = assemble_A(w.eps, lam, w.h, w.npml, w.pml_m, w.pml_lnR)
    t0 = time.perf_counter()
    lu = spla.splu(A.tocsc())
    print(f"factorised in {time.perf_counter() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(SEED)
    idx = np.sort(rng.choice(w.nx * w.ny, size=N_SAMPLES, replace=False))
    out = {"wavelength_index": np.int64(WAVELENGTH_INDEX), "sources": np.array(SOURCES, dtype=np.int64),
           "index": idx.astype(np.int64)}
    for s in SOURCES:
        b = source_rhs(J[s], lam)
        x = lu.solve(b)
        res = rel_residual(A, x, b)
        print(f"source {s}: relative residual of x* {res:.2e}", flush=True)
        out[f"x_{s}"] = x[idx]
        out[f"norm_{s}"] = np.float64(np.linalg.norm(x))
        out[f"sample_norm_{s}"] = np.float64(np.linalg.norm(x[idx]))
        out[f"residual_{s}"] = np.float64(res)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "uneven2048_reference.npz")
    np.savez_compressed(path, **out)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
