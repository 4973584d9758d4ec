"""Figure-of-merit gradient for multi-wavelength inverse design (oracle; test
infrastructure only, imported by tests, smoke() and the CPU-baseline leg of the
benchmark, never by the library).

The paper optimises devices by the adjoint-variables method with implicit
differentiation of the converged field (inverse-design section of the
results).  Here the figure of merit is the field intensity summed over
wavelengths, sources and focal cells,

    FoM = sum_lambda sum_src sum_f |E(r_f)|^2,   A(eps) E = b = -i omega J,

and its gradient follows from the plain definitions, in FP64 with direct
sparse LU solves:

    dA/deps_p = -k0^2 e_p e_p^T   (only the mass term depends on eps),
    dE/deps_p = k0^2 E_p A^-1 e_p,
    dFoM/deps_p = sum 2 Re(conj(E_f) dE_f/deps_p) = 2 k0^2 Re(E_p lam_p),
    A^T lam = P conj(E)           (P: the focal cells),

with A^T factorised directly (the oracle does not use the symmetry of S A
that the GPU path relies on).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fdfd import assemble_A, pml_stretch, source_rhs


def figure_of_merit(eps, wavelengths, J_list, focal, h, npml, pml_m=2, pml_lnR=-30.0):
    """FoM only (direct solves); focal is a list of (ix, iy)."""
    ny, nx = eps.shape
    idx = [iy * nx + ix for ix, iy in focal]
    total = 0.0
    for lam in wavelengths:
        lu = spla.splu(assemble_A(eps, lam, h, npml, pml_m, pml_lnR).tocsc())
        for J in J_list:
            x = lu.solve(source_rhs(J, lam))
            total += float(np.sum(np.abs(x[idx]) ** 2))
    return total


def fom_and_gradient(eps, wavelengths, J_list, focal, h, npml, pml_m=2, pml_lnR=-30.0):
    """(FoM, dFoM/deps [ny][nx], forward fields {(wavelength index, source): E})."""
    ny, nx = eps.shape
    idx = np.array([iy * nx + ix for ix, iy in focal], dtype=np.int64)
    fom = 0.0
    grad = np.zeros(ny * nx)
    fields = {}
    for wi, lam in enumerate(wavelengths):
        k0 = 2.0 * np.pi / lam
        A = assemble_A(eps, lam, h, npml, pml_m, pml_lnR)
        lu = spla.splu(A.tocsc())
        luT = spla.splu(A.T.tocsc())
        for si, J in enumerate(J_list):
            x = lu.solve(source_rhs(J, lam))
            fields[(wi, si)] = x
            fom += float(np.sum(np.abs(x[idx]) ** 2))
            g = np.zeros(ny * nx, dtype=np.complex128)
            np.add.at(g, idx, np.conj(x[idx]))
            lam_adj = luT.solve(g)
            grad += 2.0 * k0 ** 2 * np.real(x * lam_adj)
    return fom, grad.reshape(ny, nx), fields


def centre_stretch_product(nx, ny, npml, wavelength, h, pml_m=2, pml_lnR=-30.0):
    """S = s_x(ix) s_y(iy) at cell centres, [ny][nx]."""
    k0 = 2.0 * np.pi / wavelength
    sx, _ = pml_stretch(nx, npml, pml_m, pml_lnR, k0, h)
    sy, _ = pml_stretch(ny, npml, pml_m, pml_lnR, k0, h)
    return np.outer(sy, sx)
