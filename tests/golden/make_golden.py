"""Writes the stored expected values under tests/golden/ using only the oracle.

    python tests/golden/make_golden.py mle_small mle_profile_small

mle_small.json: maximum-likelihood fit (Nelder-Mead of the oracle) for the n = 1,600
jittered-grid workload (theta_0 = (1, 0.1, 0.5)), with z = L eps drawn by the oracle.
mle_profile_small.json: the same data fitted through the profile likelihood in
(theta2, theta3) (two-dimensional Nelder-Mead; theta1 = q / n at the maximiser).
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synthetic import SMALL  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def mle_small():
    w = SMALL
    locs = w.locations()
    z = oracle.simulate_field(locs, w.theta, w.eps())
    t0 = time.time()
    fit = oracle.fit_mle(locs, z, w.theta)
    out = {
        "workload": w.name,
        "n": w.n,
        "theta_true": list(w.theta),
        "theta_hat": list(fit["theta"]),
        "loglik_hat": fit["loglik"],
        "evals": fit["evals"],
        "iters": fit["iters"],
        "seconds": time.time() - t0,
        "source": "oracle.fit_mle (Nelder-Mead on eq. (2)); z = oracle.simulate_field",
    }
    with open(os.path.join(HERE, "mle_small.json"), "w") as f:
        json.dump(out, f, indent=2)
    print(json.dumps(out, indent=2))


def mle_profile_small():
    w = SMALL
    locs = w.locations()
    z = oracle.simulate_field(locs, w.theta, w.eps())
    t0 = time.time()
    fit = oracle.fit_mle_profile(locs, z, w.theta)
    out = {
        "workload": w.name,
        "n": w.n,
        "theta_true": list(w.theta),
        "theta_hat": list(fit["theta"]),
        "loglik_hat": fit["loglik"],
        "evals": fit["evals"],
        "iters": fit["iters"],
        "seconds": time.time() - t0,
        "source": "oracle.fit_mle_profile (Nelder-Mead on the profile of eq. (2)); "
                  "z = oracle.simulate_field",
    }
    with open(os.path.join(HERE, "mle_profile_small.json"), "w") as f:
        json.dump(out, f, indent=2)
    print(json.dumps(out, indent=2))


if __name__ == "__main__":
    for name in sys.argv[1:] or ["mle_small"]:
        globals()[name]()
