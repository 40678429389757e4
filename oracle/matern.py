"""Matérn covariance, eq. (1) of Section IV-B — oracle (test infrastructure only).

C(r; theta) = theta1 / (2^(theta3-1) Gamma(theta3)) * (r/theta2)^theta3 * K_theta3(r/theta2)

theta1 > 0 is the variance, theta2 > 0 the range and theta3 > 0 the
smoothness.  The distance r is Euclidean by default (Section IV-B: Euclidean
distance for small areas); metric="gcd" takes the locations as (longitude,
latitude) in degrees and r as the great-circle distance on a sphere of radius
6371 km (Section IV-B: great-circle distance for large areas; the radius is the
mean Earth radius, a reading), by the haversine formula.  At r = 0 the formula is 0 * inf; its limit is theta1 (because
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


EARTH_RADIUS_KM = 6371.0


def great_circle(lon1, lat1, lon2, lat2, radius: float = EARTH_RADIUS_KM):
    """Great-circle distance between points given in degrees (haversine formula):
    a = sin^2(dlat/2) + cos(lat1) cos(lat2) sin^2(dlon/2),  d = 2 R asin(sqrt(a))."""
    p1, p2 = np.radians(lat1), np.radians(lat2)
    dp = p2 - p1
    dl = np.radians(np.asarray(lon2, dtype=np.float64) - np.asarray(lon1, dtype=np.float64))
    a = np.sin(0.5 * dp) ** 2 + np.cos(p1) * np.cos(p2) * np.sin(0.5 * dl) ** 2
    return 2.0 * radius * np.arcsin(np.sqrt(np.minimum(a, 1.0)))


def cross_distances(a: np.ndarray, b: np.ndarray, metric: str = "euclidean") -> np.ndarray:
    """len(a) x len(b) distances: Euclidean, or great-circle for (lon, lat) in degrees."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if metric == "gcd":
        return great_circle(a[:, 0][:, None], a[:, 1][:, None], b[:, 0][None, :], b[:, 1][None, :])
    if metric != "euclidean":
        raise ValueError(metric)
    d0 = a[:, 0][:, None] - b[:, 0][None, :]
    d1 = a[:, 1][:, None] - b[:, 1][None, :]
    return np.sqrt(d0 * d0 + d1 * d1)


def distances(locs: np.ndarray, metric: str = "euclidean") -> np.ndarray:
    """Full n x n distance matrix of n x 2 locations."""
    return cross_distances(locs, locs, metric)


def matern_matrix(locs: np.ndarray, theta, metric: str = "euclidean") -> np.ndarray:
    """Sigma(theta) with entries Sigma_ab = C(d(s_a, s_b); theta) (Section IV-B)."""
    sigma2, beta, nu = theta
    return matern(distances(np.asarray(locs, dtype=np.float64), metric), sigma2, beta, nu)
