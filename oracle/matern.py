"""Matérn covariance, eq. (1) of Section IV-B — oracle (test infrastructure only).

C(r; theta) = theta1 / (2^(theta3-1) Gamma(theta3)) * (r/theta2)^theta3 * K_theta3(r/theta2)

theta1 > 0 is the variance, theta2 > 0 the range and theta3 > 0 the
smoothness.  The distance r is Euclidean (Section IV-B: Euclidean distance for
small areas).  At r = 0 the formula is 0 * inf; its limit is theta1 (because
x^nu K_nu(x) -> 2^(nu-1) Gamma(nu) as x -> 0), which is what Sigma_ii must be.
K is scipy's modified Bessel function of the second kind, used as a library
primitive; no closed forms are special-cased here, so the closed forms at
half-integer smoothness can pin this function in the tests.
"""
from __future__ import annotations

import numpy as np
from scipy.special import gamma, kv


def matern(r, sigma2: float, beta: float, nu: float) -> np.ndarray:
    """Eq. (1) evaluated element-wise on distances r >= 0 (float64)."""
    r = np.asarray(r, dtype=np.float64)
    x = r / beta
    out = np.full(x.shape, float(sigma2), dtype=np.float64)
    pos = x > 0.0
    if np.any(pos):
        xp = x[pos]
        scale = sigma2 / (2.0 ** (nu - 1.0) * gamma(nu))
        with np.errstate(under="ignore", over="ignore", invalid="ignore"):
            val = scale * xp ** nu * kv(nu, xp)
        # K_nu underflows to 0 far out; 0 is then the correct covariance.
        val = np.where(np.isnan(val), 0.0, val)
        out[pos] = val
    return out


def distances(locs: np.ndarray) -> np.ndarray:
    """Full n x n Euclidean distance matrix of n x 2 locations."""
    d0 = locs[:, 0][:, None] - locs[:, 0][None, :]
    d1 = locs[:, 1][:, None] - locs[:, 1][None, :]
    return np.sqrt(d0 * d0 + d1 * d1)


def cross_distances(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """len(a) x len(b) Euclidean distances."""
    d0 = a[:, 0][:, None] - b[:, 0][None, :]
    d1 = a[:, 1][:, None] - b[:, 1][None, :]
    return np.sqrt(d0 * d0 + d1 * d1)


def matern_matrix(locs: np.ndarray, theta) -> np.ndarray:
    """Sigma(theta) with entries Sigma_ab = C(||s_a - s_b||; theta) (Section IV-B)."""
    sigma2, beta, nu = theta
    return matern(distances(np.asarray(locs, dtype=np.float64)), sigma2, beta, nu)
