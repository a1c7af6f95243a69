"""Pins of the oracle's gridding convolution function and grid correction (Sec. 3.2.3)."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import gcf


def test_alpha0_matches_scipy_prolate_angular_function():
    # For alpha = 0 the eigenfunction of the finite cosine transform is the prolate
    # spheroidal angular function S_00(c, x) (scipy's pro_ang1), up to normalisation.
    c = math.pi * 7 / 2
    x = np.linspace(-0.99, 0.99, 41)
    ours = gcf.pswf(x, 0.0, c) / gcf.pswf(0.0, 0.0, c)
    ref = np.array([special.pro_ang1(0, 0, c, xx)[0] for xx in x]) / special.pro_ang1(0, 0, c, 0.0)[0]
    assert np.max(np.abs(ours - ref)) < 1e-12


@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_eigen_equation_residual(alpha):
    # integral_{-1}^{1} (1-t^2)^alpha cos(c nu t) psi(t) dt = lambda psi(nu), checked with an
    # adaptive quadrature that is independent of the Nystrom nodes.
    c = math.pi * 7 / 2
    lam = gcf.pswf_eigenvalue(alpha, c)
    for nu in (0.0, 0.3, 0.77, 1.0):
        f = lambda t: (1 - t * t) ** alpha * math.cos(c * nu * t) * float(gcf.pswf(t, alpha, c))
        val, _ = integrate.quad(f, -1.0, 1.0, epsabs=1e-14, epsrel=1e-13, limit=200)
        assert abs(val - lam * float(gcf.pswf(nu, alpha, c))) < 1e-12 * abs(lam)


def test_table_shape_symmetry_and_edges():
    T = gcf.kernel_table(7, 128)
    assert len(T) == 897
    assert T[448] == 1.0
    assert np.array_equal(T, T[::-1])
    assert T[0] == 0.0 and T[-1] == 0.0          # (1 - eta^2)^alpha vanishes at |D| = W/2
    assert np.all(np.diff(T[448:]) < 0)           # monotone decreasing away from the centre


def test_correction_is_prolate_function_of_image_offset():
    # DTFT of the kernel at image offset x' is proportional to psi(2 x'/P) (Schwab's
    # optimality argument); the tabulated sum approximates the integral to quadrature error.
    for P in (64, 256, 2048):
        corr = gcf.correction(P)
        xp = np.arange(P) - P // 2
        psi = gcf.pswf(2.0 * xp / P) / gcf.pswf(0.0)
        assert np.max(np.abs(corr / corr[P // 2] - psi)) < 1e-7
        assert np.all(corr > 0)


def test_correction_against_direct_integral():
    # corr(x') ~ integral C(D) cos(2 pi D x'/P) dD with C normalised to C(0) = 1
    P = 128
    corr = gcf.correction(P)
    c0 = float(gcf.gcf(0.0))
    for xp in (0, 7, 40, 63):
        val, _ = integrate.quad(lambda d: float(gcf.gcf(d)) / c0 * math.cos(2 * math.pi * d * xp / P),
                                -3.5, 3.5, epsabs=1e-13, limit=200)
        assert abs(corr[P // 2 + xp] - val) < 1e-5 * corr[P // 2]
