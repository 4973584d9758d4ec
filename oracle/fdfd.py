"""FDFD E_z operator with UPML stretching (oracle, test infrastructure only).

Units are normalised (c = eps0 = mu0 = eta0 = 1), so the angular frequency
equals the vacuum wavenumber, omega = k0 = 2*pi/wavelength.  The time
convention is exp(+i omega t), the one the paper's UPML stretch
s = 1 + sigma/(i omega eps0) is written in (Methods, UPML equations).

Grid: cells (ix, iy), spacing h, linear index iy*nx + ix (x fastest).
Field outside the grid is zero (Dirichlet wall behind the PML).

Operator (2D E_z form of Eq. 1, curl curl E - k0^2 eps E = -i omega J):

    (A u)[ix,iy] = -[(u[ix+1]-u[ix])/s_x(ix+1/2) - (u[ix]-u[ix-1])/s_x(ix-1/2)]
                     / (s_x(ix) h^2)
                   - (same in y)
                   - k0^2 eps[ix,iy] u[ix,iy]
    b = -i omega J.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def pml_depth(q, n, npml):
    """Fractional PML depth d(q) in [0, 1] at cell-unit position q.

    Cell centres sit at q = ix, faces at q = ix + 1/2.  The PML occupies the
    first and last ``npml`` cells; its outer faces (q = -1/2 and n - 1/2) have
    depth 1, the faces where it meets the interior have depth 0.
    """
    q = np.asarray(q, dtype=np.float64)
    if npml == 0:
        return np.zeros_like(q)
    d = np.maximum(npml - 0.5 - q, q - (n - npml - 0.5)) / npml
    return np.clip(d, 0.0, 1.0)


def pml_sigma_hat(k0, h, npml, m, lnR):
    """Normalised conductivity sigma_max / omega (Methods, UPML equations).

    sigma_max = -(m+1) ln R / (2 eta0 d) with d = npml*h the PML thickness,
    and s = 1 + sigma/(i omega) = 1 - i (sigma/omega); with omega = k0.
    """
    if npml == 0:
        return 0.0
    return (m + 1) * (-lnR) / (2.0 * k0 * npml * h)


def pml_stretch(n, npml, m, lnR, k0, h):
    """Return (s_centre[n], s_face[n+1]); s_face[f] is at position f - 1/2."""
    sh = pml_sigma_hat(k0, h, npml, m, lnR)
    qc = np.arange(n, dtype=np.float64)
    qf = np.arange(n + 1, dtype=np.float64) - 0.5
    sc = 1.0 - 1j * sh * pml_depth(qc, n, npml) ** m
    sf = 1.0 - 1j * sh * pml_depth(qf, n, npml) ** m
    return sc, sf


def _second_difference_1d(n, sc, sf, h):
    """1D matrix of -(1/s) d/dq (1/s') d/dq with zero Dirichlet outside."""
    main = (1.0 / sf[1:] + 1.0 / sf[:-1]) / (sc * h * h)
    upper = -1.0 / (sf[1:n] * sc[:n - 1] * h * h)   # row ix, column ix+1
    lower = -1.0 / (sf[1:n] * sc[1:] * h * h)       # row ix, column ix-1
    return sp.diags([lower, main, upper], [-1, 0, 1], shape=(n, n), format="csr")


def assemble_A(eps, wavelength, h, npml, pml_m=2, pml_lnR=-30.0):
    """Assemble the complex128 CSR FDFD operator for a [ny][nx] eps map."""
    eps = np.asarray(eps, dtype=np.float64)
    ny, nx = eps.shape
    k0 = 2.0 * np.pi / wavelength
    scx, sfx = pml_stretch(nx, npml, pml_m, pml_lnR, k0, h)
    scy, sfy = pml_stretch(ny, npml, pml_m, pml_lnR, k0, h)
    Dx = _second_difference_1d(nx, scx, sfx, h)
    Dy = _second_difference_1d(ny, scy, sfy, h)
    A = sp.kron(sp.identity(ny, format="csr"), Dx) + sp.kron(Dy, sp.identity(nx, format="csr"))
    A = A - sp.diags(k0 * k0 * eps.ravel())
    return A.tocsr().astype(np.complex128)


def source_rhs(J, wavelength):
    """b = -i omega J (Eq. 1 right-hand side, mu0 = 1)."""
    omega = 2.0 * np.pi / wavelength
    return (-1j * omega) * np.asarray(J, dtype=np.complex128).ravel()


def point_source(nx, ny, ix=None, iy=None):
    """Unit current in one cell; the centre of an even grid is (nx//2, ny//2)."""
    J = np.zeros((ny, nx), dtype=np.complex128)
    J[ny // 2 if iy is None else iy, nx // 2 if ix is None else ix] = 1.0
    return J


def solve_direct(A, b):
    """x* = A^-1 b by sparse LU (SuperLU), the reference for every field."""
    lu = spla.splu(A.tocsc())
    if b.ndim == 1:
        return lu.solve(b)
    return lu.solve(b)


def rel_residual(A, x, b):
    return np.linalg.norm(b - A @ x) / np.linalg.norm(b)
