"""GPU parity of the many-source subdomain solve (one workgroup per subdomain,
wavelength and group of sources; factor blocks expanded once in LDS; the
block products of the whole group as FP32 MFMA contractions), through the C
ABI.

* One Schwarz sweep z = M1^-1 v with 5 vectors per wavelength (a partial
  source group), on mixed 100 x 100 / 100 x 72 / 72 x 72 subdomains (groups of
  16) and on ragged 64..80-cell subdomains of both block orientations (groups
  of 32): every vector against the oracle's ORAS to 2e-5, and against the
  one-source-per-workgroup kernel to 1e-5 (same products, other summation
  order).
* A whole two-level solve with 6 sources and 2 wavelengths: every field within
  1e-5 of the direct solution, and the outer iteration counts within one of
  the one-source-per-workgroup path's.
"""
import numpy as np
import pytest

from oracle.fdfd import assemble_A, solve_direct, source_rhs
from oracle.partition import Partition, build_local_problems, oras_apply
from paper_2509_03622_amd.workloads import random_small

from gpu_common import dev, host, make_gpu_problem, rel

pytestmark = pytest.mark.gpu


def _oracle_locs(w, lam):
    A = assemble_A(w.eps, lam, w.h, w.npml, w.pml_m, w.pml_lnR)
    part = Partition(w.nx, w.ny, w.core_x, w.core_y, w.overlap, w.npml)
    return A, build_local_problems(part, A, w.eps.astype(np.float64), lam, w.h)


@pytest.mark.parametrize("name,w", [
    ("mixed 100/72, groups of 16",
     random_small(71, 320, 256, [96, 64, 64, 96], [96, 64, 96], wavelengths=(1.0, 1.2), npml=12, block=16)),
    ("ragged 64..80, groups of 32",
     random_small(72, 200, 128, [60, 64, 76], [60, 68], wavelengths=(0.9, 1.3), npml=10)),
])
def test_sweep_with_many_sources_matches_oracle_and_single_path(name, w):
    ctx, P = make_gpu_problem(w, k_coarse=0)
    n_src = 5
    rng = np.random.default_rng(8)
    shape = (len(w.wavelengths), n_src, w.ny, w.nx)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    z_multi = dev(np.zeros(shape))
    P.schwarz_sweep(dev(v), z_multi, n_src)
    z_multi = host(z_multi)
    P.multi_source(False)
    z_single = dev(np.zeros(shape))
    P.schwarz_sweep(dev(v), z_single, n_src)
    z_single = host(z_single)
    P.multi_source(True)
    worst_o, worst_s = 0.0, 0.0
    for wi, lam in enumerate(w.wavelengths):
        A, locs = _oracle_locs(w, lam)
        for s in range(n_src):
            ref = oras_apply(locs, v[wi, s].ravel())
            worst_o = max(worst_o, rel(z_multi[wi, s].ravel(), ref))
            worst_s = max(worst_s, rel(z_multi[wi, s], z_single[wi, s]))
    print(name, "vs oracle", worst_o, "vs single-source kernel", worst_s)
    assert worst_o < 2e-5, worst_o
    assert worst_s < 1e-5, worst_s
    P.close()
    ctx.close()


def test_many_source_solve_matches_direct_and_single_path():
    w = random_small(73, 320, 256, [96, 64, 64, 96], [96, 64, 96], wavelengths=(1.0, 1.2), n_src=6, npml=12,
                     k_coarse=1, block=16)
    ctx, P = make_gpu_problem(w)
    E, hist, it_m, fin, st = P.solve(w.J(), tol=1e-6, restart=30, max_iters=800)
    assert st == 0, (it_m, fin)
    P.multi_source(False)
    E1, hist1, it_s, fin1, st1 = P.solve(w.J(), tol=1e-6, restart=30, max_iters=800)
    P.multi_source(True)
    assert st1 == 0
    assert np.all(np.abs(it_m - it_s) <= 1), (it_m, it_s)
    for wi, lam in enumerate(w.wavelengths):
        A = assemble_A(w.eps, lam, w.h, w.npml)
        for s in range(len(w.sources)):
            xs = solve_direct(A, source_rhs(w.J()[s], lam))
            assert rel(E[wi, s].ravel(), xs) < 1e-5, (wi, s, rel(E[wi, s].ravel(), xs))
    P.close()
    ctx.close()
