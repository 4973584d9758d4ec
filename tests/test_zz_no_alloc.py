"""The allocation-free two-level preconditioner (nosdd_precond_apply_noalloc)
against nosdd_precond_apply, through the C ABI: two calls in a row, the second
with a smaller batch, each equal to the allocating entry point's result; an
oversized batch is rejected before any work is issued."""
import ctypes as C

import numpy as np
import pytest

from paper_2509_03622_amd.workloads import random_small

from gpu_common import dev, host, make_gpu_problem, rel

pytestmark = pytest.mark.gpu


def _rand(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def test_noalloc_precond_matches_allocating_entry_point():
    import torch
    w = random_small(71, 192, 192, [64] * 3, [64] * 3, wavelengths=(0.9, 1.2), npml=12, k_coarse=2, block=16)
    ctx, P = make_gpu_problem(w)
    rng = np.random.default_rng(9)
    nwl = len(w.wavelengths)
    for n_src in (3, 1):                            # the second call takes a smaller batch
        v = dev(_rand(rng, (nwl, n_src, w.ny, w.nx)))
        z_ref = torch.zeros_like(v)
        Az_ref = torch.zeros_like(v)
        P.precond_apply(v, z_ref, Az_ref, n_src)
        z = torch.full_like(v, float("nan"))
        Az = torch.full_like(v, float("nan"))
        P.precond_apply_noalloc(v, z, Az, n_src)
        zr, Azr, zn, Azn = host(z_ref), host(Az_ref), host(z), host(Az)
        print(f"n_src={n_src}: z {rel(zn, zr):.2e}, Az {rel(Azn, Azr):.2e}")
        assert np.all(np.isfinite(zn)) and np.all(np.isfinite(Azn))
        assert rel(zn, zr) <= 1e-6 and rel(Azn, Azr) <= 1e-6
        for k in range(nwl):
            for s in range(n_src):
                assert rel(zn[k, s], zr[k, s]) <= 1e-6


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    w = random_small(72, 192, 192, [64] * 3, [64] * 3, wavelengths=(1.0,), npml=12, k_coarse=1, block=16)
    ctx, P = make_gpu_problem(w)
    v = dev(np.zeros((1, 1, w.ny, w.nx), np.complex64))
    # 9 tiles x 300 000 right-hand sides need about 21 MB of queue: refused
    # before any kernel is launched, so the small buffers are never touched
    st = ctx.L.nosdd_precond_apply_noalloc(P.h, C.c_void_p(v.data_ptr()), C.c_void_p(v.data_ptr()),
                                           C.c_void_p(v.data_ptr()), 300000)
    assert st == -1
    assert b"scratch" in ctx.L.nosdd_last_error(ctx.h)
