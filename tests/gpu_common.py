"""Shared set-up for the GPU parity tests: builds a HIP-side problem and the
matching oracle objects from one seeded workload."""
from __future__ import annotations

import numpy as np

from paper_2509_03622_amd.workloads import Workload


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_gpu_problem(w: Workload, k_coarse=None, k_trial=None):
    import torch
    from paper_2509_03622_amd import nosdd
    ctx = nosdd.Context(0, nosdd.torch_stream_handle())
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths, w.pml_m, w.pml_lnR,
                      cores=w.cores)
    P.setup(k_coarse=w.k_coarse if k_coarse is None else k_coarse, k_trial=k_trial or w.k_trial)
    torch.cuda.synchronize()
    return ctx, P


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def oracle_fgmres_iterations(args):
    """Outer iterations of the oracle's Schwarz-FGMRES to 1e-6 for one
    (permittivity, wavelength, source) problem: a process-pool job, one BLAS
    thread, no GPU."""
    from threadpoolctl import threadpool_limits
    from oracle.schwarz import SchwarzProblem
    eps, lam, h, npml, core_x, core_y, overlap, k_coarse, k_trial, J = args
    with threadpool_limits(1):
        op = SchwarzProblem(eps, lam, h, npml, core_x, core_y, overlap, k_coarse=k_coarse, k_trial=k_trial)
        xo, it_o, hist_o, res_o = op.solve(J, tol=1e-6)
    return int(it_o)


def oracle_direct_field(args):
    """The FP64 direct solution of one (permittivity, wavelength, source)
    problem: a process-pool job (global sparse LU, one BLAS thread, no GPU)."""
    from threadpoolctl import threadpool_limits
    from oracle.fdfd import assemble_A, solve_direct, source_rhs
    eps, lam, h, npml, pml_m, pml_lnR, J = args
    with threadpool_limits(1):
        A = assemble_A(eps, lam, h, npml, pml_m, pml_lnR)
        return solve_direct(A, source_rhs(J, lam))


def oracle_fom_gradient_one(args):
    """The oracle's figure of merit and its gradient (direct LU of A and A^T)
    for one wavelength: a process-pool job, one BLAS thread, no GPU."""
    from threadpoolctl import threadpool_limits
    from oracle.adjoint import fom_and_gradient
    eps, lam, J, focal, h, npml = args
    with threadpool_limits(1):
        fom, grad, _ = fom_and_gradient(eps, [lam], [J], focal, h, npml)
    return fom, grad
