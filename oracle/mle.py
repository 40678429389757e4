"""Maximum-likelihood fit of theta by Nelder-Mead — oracle (test infrastructure only).

The paper maximises eq. (2) with a derivative-free optimiser at a 1e-3
tolerance and reports iteration counts (Sections IV-C and VIII-D-2); it does not
name the algorithm.  The reading used here is a plain Nelder-Mead simplex
search (reflection 1, expansion 2, contraction 1/2, shrink 1/2) on
u = log(theta), with theta clamped to box bounds, started at
theta0 * (1.5, 0.5, 1.2) with initial simplex steps of 0.1 in log units, and
stopped when the simplex spans less than xtol (log units, max-norm), or after
max_evals.  (A stop on small differences of the function values, ftol > 0, is
available but off: along the flat sigma2-range ridge of the Matérn likelihood it
ends the search while theta is still far from the maximum.)
"""
from __future__ import annotations

import math
from typing import Callable, Sequence

import numpy as np

from .likelihood import NotPositiveDefinite, loglik

LOWER = (0.01, 0.001, 0.1)
UPPER = (10.0, 2.0, 3.0)
START_SCALE = (1.5, 0.5, 1.2)


def nelder_mead(f: Callable[[np.ndarray], float], x0: Sequence[float], step: float = 0.1,
                xtol: float = 1e-6, ftol: float = 0.0, max_evals: int = 1000) -> dict:
    """Minimise f from x0 with the standard Nelder-Mead moves; returns x, f, evals, iters."""
    x0 = np.asarray(x0, dtype=np.float64)
    d = x0.size
    simplex = [x0.copy()]
    for i in range(d):
        v = x0.copy()
        v[i] += step
        simplex.append(v)
    fv = [f(v) for v in simplex]
    evals = d + 1
    iters = 0
    while evals < max_evals:
        order = sorted(range(d + 1), key=lambda i: fv[i])
        simplex = [simplex[i] for i in order]
        fv = [fv[i] for i in order]
        span = max(np.max(np.abs(v - simplex[0])) for v in simplex[1:])
        if span < xtol or (ftol > 0 and abs(fv[-1] - fv[0]) <= ftol * abs(fv[0])):
            break
        iters += 1
        centroid = np.mean(simplex[:-1], axis=0)
        worst = simplex[-1]
        xr = centroid + (centroid - worst)
        fr = f(xr)
        evals += 1
        if fr < fv[0]:
            xe = centroid + 2.0 * (centroid - worst)
            fe = f(xe)
            evals += 1
            if fe < fr:
                simplex[-1], fv[-1] = xe, fe
            else:
                simplex[-1], fv[-1] = xr, fr
            continue
        if fr < fv[-2]:
            simplex[-1], fv[-1] = xr, fr
            continue
        if fr < fv[-1]:
            xc = centroid + 0.5 * (xr - centroid)        # outside contraction
            fc = f(xc)
            evals += 1
            if fc <= fr:
                simplex[-1], fv[-1] = xc, fc
                continue
        else:
            xc = centroid + 0.5 * (worst - centroid)     # inside contraction
            fc = f(xc)
            evals += 1
            if fc < fv[-1]:
                simplex[-1], fv[-1] = xc, fc
                continue
        for i in range(1, d + 1):                        # shrink towards the best
            simplex[i] = simplex[0] + 0.5 * (simplex[i] - simplex[0])
            fv[i] = f(simplex[i])
            evals += 1
    best = int(np.argmin(fv))
    return {"x": simplex[best], "f": fv[best], "evals": evals, "iters": iters}


def clamp_theta(u: np.ndarray) -> tuple:
    """theta = exp(u), clamped component-wise to [LOWER, UPPER]."""
    return tuple(min(max(math.exp(float(ui)), lo), hi)
                 for ui, lo, hi in zip(u, LOWER, UPPER))


def fit_mle(locs: np.ndarray, z: np.ndarray, theta0, **nm_kwargs) -> dict:
    """Maximise eq. (2) over theta; returns theta_hat, loglik, evals and iterations."""
    def neg_loglik(u: np.ndarray) -> float:
        try:
            return -loglik(locs, z, clamp_theta(u))["loglik"]
        except NotPositiveDefinite:
            return math.inf

    start = [min(max(t * s, lo), hi) for t, s, lo, hi in
             zip(theta0, START_SCALE, LOWER, UPPER)]
    res = nelder_mead(neg_loglik, np.log(start), **nm_kwargs)
    return {"theta": clamp_theta(res["x"]), "loglik": -res["f"],
            "evals": res["evals"], "iters": res["iters"]}
