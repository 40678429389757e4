"""Pins for the oracle's Matérn covariance (eq. (1), Section IV-B).

Each check uses mathematics that does not go through scipy's Bessel routine:
closed forms at half-integer smoothness, the integral representation of K_nu
evaluated by adaptive quadrature, the r -> 0 limit, the three-term recurrence
and the 1-D exponential-kernel (AR(1)) matrix.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import gamma

from oracle import matern, matern_matrix
from synthetic import jittered_grid, line_grid

X = np.concatenate([np.logspace(-6, 0, 25), np.linspace(1.1, 40.0, 40)])


@pytest.mark.parametrize("sigma2,beta", [(1.0, 0.1), (2.5, 0.03), (0.7, 0.3)])
def test_half_integer_closed_forms(sigma2, beta):
    # K_{1/2}, K_{3/2}, K_{5/2} are elementary; eq. (1) then reduces to
    # sigma2 e^-x, sigma2 (1+x) e^-x, sigma2 (1 + x + x^2/3) e^-x with x = r/beta.
    r = X * beta
    x = X
    closed = {
        0.5: sigma2 * np.exp(-x),
        1.5: sigma2 * (1.0 + x) * np.exp(-x),
        2.5: sigma2 * (1.0 + x + x * x / 3.0) * np.exp(-x),
    }
    for nu, want in closed.items():
        got = matern(r, sigma2, beta, nu)
        np.testing.assert_allclose(got, want, rtol=2e-14, atol=0)


def _k_integral(nu, x):
    # K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt  (DLMF 10.32.9)
    # the integrand is below e^-800 beyond t_max, so the tail is dropped
    t_max = math.acosh(max(800.0 / x, 2.0)) + 1.0
    val, err = quad(lambda t: math.exp(-x * math.cosh(t)) * math.cosh(nu * t), 0.0, t_max,
                    epsabs=0.0, epsrel=1e-13, limit=400)
    return val


@pytest.mark.parametrize("nu", [0.3, 0.73, 1.0, 1.37, 2.2])
def test_general_nu_against_integral_representation(nu):
    sigma2, beta = 1.3, 0.2
    for x in (1e-3, 0.05, 0.5, 1.0, 1.9, 2.1, 5.0, 12.0, 30.0):
        got = matern(np.array([x * beta]), sigma2, beta, nu)[0]
        want = sigma2 / (2.0 ** (nu - 1.0) * gamma(nu)) * x ** nu * _k_integral(nu, x)
        assert got == pytest.approx(want, rel=1e-11), (nu, x)


@pytest.mark.parametrize("nu", [0.5, 0.9, 1.0, 2.0])
def test_zero_distance_is_the_variance_limit(nu):
    sigma2 = 1.7
    assert matern(np.array([0.0]), sigma2, 0.1, nu)[0] == sigma2
    # continuity of x^nu K_nu(x) 2^(1-nu)/Gamma(nu) -> 1 at x -> 0
    near = matern(np.array([1e-9]), sigma2, 0.1, nu)[0]
    assert near == pytest.approx(sigma2, rel=1e-7)


@pytest.mark.parametrize("nu", [0.6, 1.3, 2.45])
def test_three_term_recurrence(nu):
    # K_{nu+1}(x) = K_{nu-1}(x) + (2 nu / x) K_nu(x), with K recovered from eq. (1)
    # and K_{-s} = K_s for a negative order.
    def k(order, x):
        order = abs(order)
        c = matern(np.array([x]), 1.0, 1.0, order)[0]
        return c * 2.0 ** (order - 1.0) * gamma(order) / x ** order

    for x in (0.2, 1.0, 3.0, 9.0):
        assert k(nu + 1, x) == pytest.approx(k(nu - 1, x) + 2 * nu / x * k(nu, x), rel=1e-13)


def test_matrix_is_symmetric_with_variance_diagonal():
    locs = jittered_grid(12, seed=5)
    s = matern_matrix(locs, (1.4, 0.1, 1.0))
    assert np.array_equal(s, s.T)
    assert np.all(np.diag(s) == 1.4)
    assert np.all(s > 0) and np.all(s <= 1.4)


def test_one_dimensional_exponential_is_ar1():
    # On points (i h, 0) with nu = 1/2: Sigma_ij = sigma2 rho^|i-j|, rho = exp(-h/beta).
    n, h, sigma2, beta = 60, 0.02, 1.3, 0.1
    s = matern_matrix(line_grid(n, h), (sigma2, beta, 0.5))
    rho = math.exp(-h / beta)
    i = np.arange(n)
    want = sigma2 * rho ** np.abs(i[:, None] - i[None, :])
    np.testing.assert_allclose(s, want, rtol=1e-13, atol=0)
