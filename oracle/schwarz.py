"""Global Schwarz-FGMRES driver (oracle, test infrastructure only).

Right-preconditioned flexible GMRES(restart) on the global system A x = b with
the two-level optimised restricted additive Schwarz preconditioner: one
preconditioner application is one sweep of all subdomain Robin solves
(Algorithm 3 loop body, which by the Robin identity equals x + M1^-1 (b - A x))
followed by the coarse correction.  Exact subdomain solves use sparse LU.
"""
from __future__ import annotations

import numpy as np

from .coarse import CoarseSpace, two_level_apply
from .fdfd import assemble_A, source_rhs
from .fgmres import fgmres
from .partition import Partition, build_local_problems


class SchwarzProblem:
    def __init__(self, eps, wavelength, h, npml, core_x, core_y, overlap,
                 k_coarse=0, k_trial=8, pml_m=2, pml_lnR=-30.0, rotation="svd", cores=None):
        self.eps = np.asarray(eps, dtype=np.float64)
        ny, nx = self.eps.shape
        self.wavelength, self.h = wavelength, h
        self.A = assemble_A(self.eps, wavelength, h, npml, pml_m, pml_lnR)
        if cores is not None:       # explicit core list (e.g. a quad-tree)
            self.part = Partition.from_cores(nx, ny, cores, overlap, npml)
        else:
            self.part = Partition(nx, ny, core_x, core_y, overlap, npml)
        self.locs = build_local_problems(self.part, self.A, self.eps, wavelength, h)
        self.cs = None
        if k_coarse > 0:
            self.cs = CoarseSpace(self.part, self.locs, self.A, self.eps, wavelength, h,
                                  k_coarse, k_trial, rotation)

    def precond(self, v):
        return two_level_apply(self.locs, self.A, self.cs, v)

    def solve(self, J, tol=1e-6, restart=30, max_iters=1000, x0=None):
        b = source_rhs(J, self.wavelength)
        return fgmres(lambda u: self.A @ u, b, self.precond, tol=tol,
                      restart=restart, max_iters=max_iters, x0=x0)
