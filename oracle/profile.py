"""Profile log-likelihood in (theta2, theta3) — oracle (test infrastructure only).

Section IV-C: for fixed range theta2 and smoothness theta3, eq. (2) is maximised over the
variance theta1 in closed form.  Write Sigma(theta) = theta1 * R, with R the correlation
matrix (eq. (1) at theta1 = 1), and q = Z^T R^-1 Z.  Then
    l(theta1) = -n/2 log(2 pi) - n/2 log(theta1) - 1/2 log|R| - q / (2 theta1),
whose derivative in theta1 vanishes at theta1 = q / n, and substituting that value gives
    l_p(theta2, theta3) = -n/2 log(2 pi) - n/2 - n/2 log(q / n) - 1/2 log|R|.
The paper's printed profile equation has its trailing terms garbled (it would not equal
eq. (2) at the maximising variance); the form above is the one the substitution gives.
"""
from __future__ import annotations

import math

import numpy as np

from .likelihood import LOG_2PI, NotPositiveDefinite, loglik
from .mle import LOWER, START_SCALE, UPPER, nelder_mead


def profile_loglik(locs: np.ndarray, z: np.ndarray, beta: float, nu: float) -> dict:
    """l_p(beta, nu) with its parts: logdet = log|R|, quad = q, sigma2_hat = q / n."""
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[0]
    parts = loglik(locs, z, (1.0, beta, nu))
    q = parts["quad"]
    lp = -0.5 * n * LOG_2PI - 0.5 * n - 0.5 * n * math.log(q / n) - 0.5 * parts["logdet"]
    return {"loglik": lp, "logdet": parts["logdet"], "quad": q, "sigma2_hat": q / n}


def fit_mle_profile(locs: np.ndarray, z: np.ndarray, theta0, **nm_kwargs) -> dict:
    """Maximise l_p over (theta2, theta3) with the same Nelder-Mead as the full fit (log
    parameters, clamped to the same bounds, started at theta0 * START_SCALE); theta1 is then
    q / n at the maximiser."""
    def clamp(u):
        return tuple(min(max(math.exp(float(ui)), lo), hi)
                     for ui, lo, hi in zip(u, LOWER[1:], UPPER[1:]))

    def neg(u: np.ndarray) -> float:
        try:
            return -profile_loglik(locs, z, *clamp(u))["loglik"]
        except NotPositiveDefinite:
            return math.inf

    start = [min(max(t * s, lo), hi) for t, s, lo, hi in
             zip(theta0[1:], START_SCALE[1:], LOWER[1:], UPPER[1:])]
    res = nelder_mead(neg, np.log(start), **nm_kwargs)
    beta, nu = clamp(res["x"])
    best = profile_loglik(locs, z, beta, nu)
    return {"theta": (best["sigma2_hat"], beta, nu), "loglik": best["loglik"],
            "evals": res["evals"], "iters": res["iters"]}
