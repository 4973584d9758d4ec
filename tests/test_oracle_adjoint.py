"""Pins of the oracle's figure-of-merit gradient (inverse design).

* Central finite differences of the FoM itself, in FP64, at cells in the
  interior, in the PML, on a focal cell and next to the source: the adjoint
  gradient must agree to 1e-6 relative (the O(delta^2) error of the central
  difference at delta = 1e-4 is far below that).
* The transpose identity the GPU adjoint relies on: S A is complex symmetric
  for S = diag(s_x s_y) at cell centres, so A^T = S A S^-1 (checked on the
  assembled matrix, PML included).
* Sum rule: the gradient summed over all cells equals the derivative of the
  FoM under the uniform shift eps -> eps + t (central difference in t).
"""
import numpy as np
import pytest

from oracle.adjoint import centre_stretch_product, figure_of_merit, fom_and_gradient
from oracle.fdfd import assemble_A

pytestmark = pytest.mark.filterwarnings("ignore")


def small_case(seed=3):
    rng = np.random.default_rng(seed)
    nx, ny, npml, h = 40, 34, 6, 0.05
    eps = np.ones((ny, nx))
    eps[10:24, 12:30] = rng.uniform(1, 12, (14, 18))
    J = np.zeros((ny, nx), dtype=np.complex128)
    J[9, 14:26] = 1.0                      # line source
    focal = [(20, 27), (24, 26)]
    return eps, [J], focal, h, npml


def test_gradient_matches_central_differences():
    eps, J, focal, h, npml = small_case()
    wls = (0.9, 1.3)
    fom, grad, _ = fom_and_gradient(eps, wls, J, focal, h, npml)
    assert fom > 0
    cells = [(20, 15), (2, 3), (20, 27), (15, 10), (33, 30), (7, 20)]   # interior, PML, focal, near source
    d = 1e-4
    for ix, iy in cells:
        ep, em = eps.copy(), eps.copy()
        ep[iy, ix] += d
        em[iy, ix] -= d
        fd = (figure_of_merit(ep, wls, J, focal, h, npml) - figure_of_merit(em, wls, J, focal, h, npml)) / (2 * d)
        assert abs(fd - grad[iy, ix]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(grad).max()), (ix, iy, fd, grad[iy, ix])


def test_uniform_perturbation_sum_rule():
    eps, J, focal, h, npml = small_case(4)
    wls = (1.1,)
    fom, grad, _ = fom_and_gradient(eps, wls, J, focal, h, npml)
    d = 1e-5
    fd = (figure_of_merit(eps + d, wls, J, focal, h, npml) - figure_of_merit(eps - d, wls, J, focal, h, npml)) / (2 * d)
    assert abs(fd - grad.sum()) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("lam", [0.8, 1.5])
def test_stretched_operator_is_complex_symmetric(lam):
    eps, J, focal, h, npml = small_case()
    ny, nx = eps.shape
    A = assemble_A(eps, lam, h, npml).tocsr()
    S = centre_stretch_product(nx, ny, npml, lam, h).ravel()
    SA = A.multiply(S[:, None]).tocsr()
    diff = abs(SA - SA.T).max()
    assert diff <= 1e-12 * abs(SA).max(), diff
    # and not symmetric without the scaling (the PML breaks it)
    assert abs(A - A.T).max() > 1e-3 * abs(A).max()
