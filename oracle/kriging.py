"""Simple-kriging prediction — oracle (test infrastructure only).

The paper predicts held-out values from the fitted model and scores them by
the prediction mean squared error (Section VIII-D); it does not print the
predictor.  The reading used: simple kriging with the known zero mean of
Section IV-A,
    Zhat(s0) = Sigma(s0, S) Sigma(S, S)^-1 Z,
    var(s0)  = theta1 - Sigma(s0, S) Sigma(S, S)^-1 Sigma(S, s0).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .likelihood import cholesky_lower
from .matern import cross_distances, matern, matern_matrix


def krige(locs: np.ndarray, z: np.ndarray, theta, new_locs: np.ndarray,
          metric: str = "euclidean") -> dict:
    """Predictions and variances at new_locs (m x 2) from data z at locs (n x 2)."""
    sigma2, beta, nu = theta
    low = cholesky_lower(matern_matrix(locs, theta, metric))
    y = sla.solve_triangular(low, np.asarray(z, dtype=np.float64), lower=True)
    w = sla.solve_triangular(low.T, y, lower=False)          # Sigma^-1 Z
    c = matern(cross_distances(np.asarray(new_locs, dtype=np.float64),
                               np.asarray(locs, dtype=np.float64), metric), sigma2, beta, nu)
    pred = c @ w
    v = sla.solve_triangular(low, c.T, lower=True)           # L^-1 Sigma(S, s0)
    var = sigma2 - np.sum(v * v, axis=0)
    return {"pred": pred, "var": var}
