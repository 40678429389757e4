"""Pins for the oracle's factor, solve, log-determinant and eq. (2).

The exponential kernel on a regular 1-D grid is an AR(1) covariance whose
Cholesky factor, determinant and inverse have closed forms; tiny 2-D problems
are checked against an exact rational-arithmetic determinant and solve; the
reconstruction residual and permutation invariance hold at any size.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import cholesky_lower, loglik, matern_matrix, simulate_field
from oracle.likelihood import LOG_2PI, NotPositiveDefinite, loglik_parts
from synthetic import jittered_grid, line_grid, normals


def ar1_case(n=50, h=0.03, sigma2=1.7, beta=0.1, seed=7):
    locs = line_grid(n, h)
    z = normals(n, seed)
    rho = math.exp(-h / beta)
    return locs, z, (sigma2, beta, 0.5), rho


def test_ar1_cholesky_closed_form():
    locs, z, theta, rho = ar1_case()
    sigma = math.sqrt(theta[0])
    n = len(z)
    low = cholesky_lower(matern_matrix(locs, theta))
    want = np.zeros((n, n))
    for i in range(n):
        want[i, 0] = sigma * rho ** i
        for j in range(1, i + 1):
            want[i, j] = sigma * math.sqrt(1 - rho * rho) * rho ** (i - j)
    np.testing.assert_allclose(low, want, rtol=1e-12, atol=1e-15)


def test_ar1_logdet_quad_and_loglik_closed_form():
    locs, z, theta, rho = ar1_case()
    sigma2 = theta[0]
    n = len(z)
    out = loglik(locs, z, theta)
    logdet = n * math.log(sigma2) + (n - 1) * math.log(1 - rho * rho)
    # tridiagonal inverse of the AR(1) covariance
    quad = z[0] ** 2 / sigma2 + sum((z[i] - rho * z[i - 1]) ** 2 for i in range(1, n)) / (
        sigma2 * (1 - rho * rho))
    assert out["logdet"] == pytest.approx(logdet, rel=1e-13)
    assert out["quad"] == pytest.approx(quad, rel=1e-12)
    want = -0.5 * n * math.log(2 * math.pi) - 0.5 * logdet - 0.5 * quad
    assert out["loglik"] == pytest.approx(want, rel=1e-12)


def _exact_logdet_and_quad(a: np.ndarray, z: np.ndarray):
    """Exact determinant and z^T A^-1 z by Gaussian elimination over the rationals."""
    n = len(z)
    m = [[Fraction(float(a[i, j])) for j in range(n)] + [Fraction(float(z[i]))]
         for i in range(n)]
    det = Fraction(1)
    for c in range(n):
        piv = next(r for r in range(c, n) if m[r][c] != 0)
        if piv != c:
            m[c], m[piv] = m[piv], m[c]
            det = -det
        det *= m[c][c]
        for r in range(c + 1, n):
            f = m[r][c] / m[c][c]
            if f:
                for k in range(c, n + 1):
                    m[r][k] -= f * m[c][k]
    x = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        s = m[r][n] - sum(m[r][k] * x[k] for k in range(r + 1, n))
        x[r] = s / m[r][r]
    quad = sum(Fraction(float(z[i])) * x[i] for i in range(n))
    return math.log(det), float(quad)


@pytest.mark.parametrize("n,theta", [(4, (1.0, 0.1, 0.5)), (9, (1.3, 0.3, 1.0)),
                                     (12, (0.8, 0.05, 1.5)), (12, (1.0, 0.2, 0.73))])
def test_tiny_problems_against_exact_rational_arithmetic(n, theta):
    rng = np.random.default_rng(n)
    locs = rng.uniform(0, 1, size=(n, 2))
    z = normals(n, 11 + n)
    a = matern_matrix(locs, theta)
    logdet, quad = _exact_logdet_and_quad(a, z)
    out = loglik(locs, z, theta)
    cond = np.linalg.cond(a)
    assert out["logdet"] == pytest.approx(logdet, rel=1e-13 * cond, abs=1e-12 * cond)
    assert out["quad"] == pytest.approx(quad, rel=1e-13 * cond)
    want = -0.5 * n * LOG_2PI - 0.5 * logdet - 0.5 * quad
    assert out["loglik"] == pytest.approx(want, rel=1e-13 * cond)


def test_reconstruction_residual():
    locs = jittered_grid(20, seed=3)
    a = matern_matrix(locs, (1.0, 0.1, 1.0))
    low = cholesky_lower(a)
    n = a.shape[0]
    assert np.all(np.diag(low) > 0)
    assert np.array_equal(low, np.tril(low))
    res = np.linalg.norm(low @ low.T - a) / np.linalg.norm(a)
    assert res <= 10 * n * 2.0 ** -53


def test_permutation_invariance():
    locs = jittered_grid(15, seed=4)
    z = normals(len(locs), 5)
    theta = (1.0, 0.1, 0.5)
    base = loglik(locs, z, theta)["loglik"]
    perm = np.random.default_rng(0).permutation(len(z))
    assert loglik(locs[perm], z[perm], theta)["loglik"] == pytest.approx(base, rel=1e-12)


def test_identity_padding_leaves_logdet_and_quad_unchanged():
    locs = jittered_grid(10, seed=8)
    z = normals(len(locs), 9)
    a = matern_matrix(locs, (1.0, 0.2, 0.5))
    n, pad = a.shape[0], 7
    big = np.eye(n + pad)
    big[:n, :n] = a
    zz = np.concatenate([z, np.zeros(pad)])
    p1, p2 = loglik_parts(a, z), loglik_parts(big, zz)
    assert p2["logdet"] == pytest.approx(p1["logdet"], rel=1e-14, abs=1e-13)
    assert p2["quad"] == pytest.approx(p1["quad"], rel=1e-14)


def test_not_positive_definite_is_reported():
    a = np.eye(5)
    a[3, 3] = -1.0
    with pytest.raises(NotPositiveDefinite):
        cholesky_lower(a)


def test_simulated_field_has_the_model_covariance():
    # z = L eps: the sample covariance over many draws approaches Sigma.
    locs = jittered_grid(4, seed=1)
    theta = (1.0, 0.3, 0.5)
    eps = np.random.default_rng(2).standard_normal((16, 20000))
    low = cholesky_lower(matern_matrix(locs, theta))
    zs = low @ eps
    emp = zs @ zs.T / eps.shape[1]
    np.testing.assert_allclose(emp, matern_matrix(locs, theta), atol=0.05)
    z = simulate_field(locs, theta, eps[:, 0])
    np.testing.assert_allclose(z, zs[:, 0], rtol=1e-14)
