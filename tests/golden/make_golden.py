"""Writes the stored expected values under tests/golden/ using only the oracle.

    python tests/golden/make_golden.py mle_small mle_profile_small

mle_small.json: maximum-likelihood fit (Nelder-Mead of the oracle) for the n = 1,600
jittered-grid workload (theta_0 = (1, 0.1, 0.5)), with z = L eps drawn by the oracle.
mle_profile_small.json: the same data fitted through the profile likelihood in
(theta2, theta3) (two-dimensional Nelder-Mead; theta1 = q / n at the maximiser).
small_z.txt: the data z = L eps of the n = 1,600 workload drawn by the oracle (one value per
line, 17 significant digits), the input of the fits above, for the benchmark's fit beside them.
sweep_n40000.json: for each of the six n = 40,000 band-sweep fields, eq. (2) at the true theta
with z = L eps drawn by the oracle's FP64 factor (so y = L^-1 z is eps up to rounding): logdet,
quad and l.  Sigma is filled in row blocks of the oracle's own eq. (1), one block at a time
(the whole-matrix form of the oracle would hold several 12.8 GB temporaries at once; the Bessel
routine is not safe to call from several threads at general smoothness); the factorization and
the forward substitution are LAPACK's through PyTorch on the CPU, the steps of the oracle's
eq. (2).  Three to six minutes per field, 26 GB.
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synthetic import SMALL, SWEEP  # noqa: E402

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


def small_z():
    w = SMALL
    z = oracle.simulate_field(w.locations(), w.theta, w.eps())
    with open(os.path.join(HERE, "small_z.txt"), "w") as f:
        f.write("".join(f"{float(v)!r}\n" for v in z))


def _matern_matrix_blocked(locs, theta, blocks=256):
    import numpy as np
    n = len(locs)
    sig = np.empty((n, n))
    for rows in np.array_split(np.arange(n), blocks):
        sig[rows] = oracle.matern(oracle.cross_distances(locs[rows], locs), *theta)
    return sig


def sweep_n40000():
    import math

    import numpy as np
    import torch
    rows = []
    for w in SWEEP:
        t0 = time.time()
        locs = w.locations()
        eps = w.eps()
        sig = _matern_matrix_blocked(locs, w.theta)
        # Cholesky and forward substitution by PyTorch's CPU LAPACK (MKL): OpenBLAS's threaded
        # Cholesky faulted at this size, in numpy's and scipy's builds alike
        low_t = torch.linalg.cholesky(torch.from_numpy(sig))
        del sig
        low = low_t.numpy()
        z = (low_t @ torch.from_numpy(eps)).numpy()     # oracle.simulate_field, factor reused
        y = torch.linalg.solve_triangular(low_t, torch.from_numpy(z)[:, None], upper=False)[:, 0].numpy()
        logdet = 2.0 * math.fsum(np.log(np.diag(low)))
        quad = math.fsum(y * y)
        del low, low_t
        row = {"field": w.name, "n": w.n, "theta": list(w.theta), "loc_seed": w.loc_seed,
               "z_seed": w.z_seed, "logdet": logdet, "quad": quad,
               "loglik": -0.5 * w.n * oracle.likelihood.LOG_2PI - 0.5 * logdet - 0.5 * quad,
               "seconds": time.time() - t0}
        rows.append(row)
        print(json.dumps(row), flush=True)
    out = {"source": "oracle eq. (2) at the true theta, z = L eps with the oracle's FP64 factor",
           "fields": rows}
    with open(os.path.join(HERE, "sweep_n40000.json"), "w") as f:
        json.dump(out, f, indent=2)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["mle_small"]:
        globals()[name]()
