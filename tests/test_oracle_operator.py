"""Pins of the oracle's FDFD operator, PML and direct solve (CPU only).

Each test checks the oracle against something other than itself: the discrete
plane-wave dispersion relation, the closed-form 2D Green's function
(exp(+i omega t) convention: -(omega h^2/4) H0^(2)(k0 r) for a unit cell current),
second-order convergence, reciprocity of the stretched operator and the
absorption of the PML.
"""
import numpy as np
import pytest
import scipy.special as special

from oracle.fdfd import assemble_A, pml_sigma_hat, pml_stretch, point_source, rel_residual, solve_direct, source_rhs


def test_sigma_hat_value():
    # m = 2, ln R = -30, 12 cells of h = 0.05 at wavelength 1: 3*30/(2*2pi*0.6)
    assert pml_sigma_hat(2 * np.pi, 0.05, 12, 2, -30.0) == pytest.approx(11.9366, rel=1e-4)


def test_pml_profile_ends():
    sc, sf = pml_stretch(40, 8, 2, -30.0, 2 * np.pi, 0.05)
    sh = pml_sigma_hat(2 * np.pi, 0.05, 8, 2, -30.0)
    # outer faces fully stretched, interior exactly 1, symmetric
    assert sf[0] == pytest.approx(1 - 1j * sh)
    assert sf[-1] == pytest.approx(1 - 1j * sh)
    assert np.all(sc[8:32] == 1.0)
    assert np.all(sf[8:33] == 1.0)
    np.testing.assert_allclose(sc, sc[::-1])
    np.testing.assert_allclose(sf, sf[::-1])
    # exp(+i omega t): the stretch has a negative imaginary part (decay of exp(-i k x~))
    assert np.all(sc.imag <= 0)


def test_plane_wave_dispersion_interior():
    """A discrete plane wave with the discrete wavenumber is annihilated away from the walls."""
    n, h, lam, eps0 = 48, 0.05, 1.0, 2.5
    k0 = 2 * np.pi / lam
    A = assemble_A(np.full((n, n), eps0), lam, h, npml=0)
    ang = 0.3
    # 4/h^2 (sin^2(kx h/2) + sin^2(ky h/2)) = k0^2 eps with (kx, ky) = kt (cos, sin)
    from scipy.optimize import brentq
    f = lambda kt: 4 / h**2 * (np.sin(kt * np.cos(ang) * h / 2) ** 2 + np.sin(kt * np.sin(ang) * h / 2) ** 2) - k0**2 * eps0
    kt = brentq(f, 0.5 * k0 * np.sqrt(eps0), 1.5 * k0 * np.sqrt(eps0))
    y, x = np.mgrid[0:n, 0:n]
    u = np.exp(-1j * kt * h * (np.cos(ang) * x + np.sin(ang) * y))
    r = (A @ u.ravel()).reshape(n, n)
    inner = r[1:-1, 1:-1]
    assert np.max(np.abs(inner)) < 1e-9 * k0**2 * eps0
    # and the Dirichlet wall rows are not annihilated (the wall is really there)
    assert np.max(np.abs(r[0])) > 1.0


def _green_error(cells_per_lambda):
    lam = 1.0
    h = lam / cells_per_lambda
    npml = int(round(0.6 * cells_per_lambda))
    half = 2 * cells_per_lambda           # 2 wavelengths from the centre to the PML
    n = 2 * (half + npml)
    A = assemble_A(np.ones((n, n)), lam, h, npml)
    x = solve_direct(A, source_rhs(point_source(n, n), lam)).reshape(n, n)
    k0 = 2 * np.pi / lam
    yy, xx = np.mgrid[0:n, 0:n]
    r = h * np.hypot(xx - n // 2, yy - n // 2)
    ring = (r >= 1.0 * lam) & (r <= 1.5 * lam)
    ref = -(k0 * h * h / 4) * special.hankel2(0, k0 * r[ring])
    return np.linalg.norm(x[ring] - ref) / np.linalg.norm(ref)


def test_green_function_and_second_order():
    e20, e40, e80 = _green_error(20), _green_error(40), _green_error(80)
    assert e20 < 0.1                      # dispersion error at 20 cells per wavelength
    assert 3.0 <= e20 / e40 <= 5.0
    assert 3.0 <= e40 / e80 <= 5.0


def test_reciprocity_with_pml():
    """S A is complex symmetric (S = diag(s_x s_y)), so s_a G_ab = s_b G_ba."""
    rng = np.random.default_rng(7)
    n, npml, lam, h = 40, 8, 1.0, 0.05
    eps = rng.uniform(1, 6, (n, n))
    A = assemble_A(eps, lam, h, npml)
    k0 = 2 * np.pi / lam
    sc, _ = pml_stretch(n, npml, 2, -30.0, k0, h)
    S = np.outer(sc, sc).ravel()         # [iy][ix] -> s_y(iy) s_x(ix)
    pts = [(20, 20), (13, 27), (3, 30), (25, 2), (36, 37)]     # interior and PML cells
    G = {}
    for (ix, iy) in pts:
        e = np.zeros(n * n, complex)
        e[iy * n + ix] = 1.0
        G[(ix, iy)] = solve_direct(A, e)
    for a in pts:
        for b in pts:
            ia, ib = a[1] * n + a[0], b[1] * n + b[0]
            lhs = S[ib] * G[a][ib]       # s_b (A^-1)_{b a}
            rhs = S[ia] * G[b][ia]
            assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1e-30)


def test_pml_absorbs():
    """Interior field is nearly unchanged when the PML is moved twice as far away."""
    lam, h, npml = 1.0, 0.05, 12
    rng = np.random.default_rng(3)
    core = rng.uniform(1, 4, (40, 40))
    fields = []
    for pad in (10, 50):
        n = 40 + 2 * (pad + npml)
        eps = np.ones((n, n))
        o = pad + npml
        eps[o:o + 40, o:o + 40] = core
        A = assemble_A(eps, lam, h, npml)
        J = point_source(n, n, o + 20, o + 20)
        x = solve_direct(A, source_rhs(J, lam)).reshape(n, n)
        fields.append(x[o:o + 40, o:o + 40])
    err = np.linalg.norm(fields[0] - fields[1]) / np.linalg.norm(fields[1])
    assert err < 1e-3


def test_direct_solve_residual():
    rng = np.random.default_rng(1)
    eps = rng.uniform(1, 12, (32, 32))
    A = assemble_A(eps, 1.0, 0.05, 6)
    b = source_rhs(point_source(32, 32), 1.0)
    x = solve_direct(A, b)
    assert rel_residual(A, x, b) < 1e-12
