"""Gaussian log-likelihood, eq. (2) of Section IV-C — oracle (test infrastructure only).

l(theta) = -n/2 log(2 pi) - 1/2 log|Sigma(theta)| - 1/2 Z^T Sigma(theta)^-1 Z

evaluated the plain way: Sigma = L L^T with L lower triangular with positive
diagonal (Section V-A), y = L^-1 Z, log|Sigma| = 2 sum_i log L_ii and
Z^T Sigma^-1 Z = y^T y.  Everything is FP64; the two sums are correctly
rounded (math.fsum).  The natural logarithm is used throughout.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .matern import matern_matrix

LOG_2PI = math.log(2.0 * math.pi)


class NotPositiveDefinite(ArithmeticError):
    """Raised when the Cholesky factorisation meets a non-positive pivot."""


def cholesky_lower(a: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor of a symmetric positive-definite matrix (LAPACK)."""
    try:
        return np.linalg.cholesky(np.asarray(a, dtype=np.float64))
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite(str(exc)) from exc


def loglik_parts(a: np.ndarray, z: np.ndarray) -> dict:
    """logdet, quad and l of eq. (2) for a given covariance matrix and data vector."""
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[0]
    low = cholesky_lower(a)
    y = sla.solve_triangular(low, z, lower=True)
    logdet = 2.0 * math.fsum(np.log(np.diag(low)))
    quad = math.fsum(y * y)
    return {
        "loglik": -0.5 * n * LOG_2PI - 0.5 * logdet - 0.5 * quad,
        "logdet": logdet,
        "quad": quad,
        "L": low,
        "y": y,
    }


def loglik(locs: np.ndarray, z: np.ndarray, theta, metric: str = "euclidean") -> dict:
    """Eq. (2) at theta for locations locs (n x 2) and data z (n)."""
    return loglik_parts(matern_matrix(locs, theta, metric), z)


def simulate_field(locs: np.ndarray, theta, eps: np.ndarray, metric: str = "euclidean") -> np.ndarray:
    """A draw of the zero-mean Matérn field at locs: z = L eps with Sigma(theta) = L L^T.

    This is how synthetic measurements are produced from a parameter vector
    theta_0 (Section VIII-B.1): the standard normal vector eps is an input.
    """
    low = cholesky_lower(matern_matrix(locs, theta, metric))
    return low @ np.asarray(eps, dtype=np.float64)
