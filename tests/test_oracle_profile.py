"""Pins for the oracle's profile likelihood in (theta2, theta3) (Section IV-C)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from synthetic import SMALL, jittered_grid, line_grid, normals


def test_profile_equals_eq2_at_the_maximising_variance():
    # substituting theta1 = q/n into eq. (2) must give the profile value, and any other
    # variance must give less (eq. (2) is concave in log theta1)
    locs = jittered_grid(12, seed=5)
    z = normals(len(locs), 6)
    beta, nu = 0.15, 0.8
    prof = oracle.profile_loglik(locs, z, beta, nu)
    full = oracle.loglik(locs, z, (prof["sigma2_hat"], beta, nu))["loglik"]
    assert prof["loglik"] == pytest.approx(full, rel=1e-12, abs=1e-9)
    for f in (0.97, 0.995, 1.005, 1.03):
        assert oracle.loglik(locs, z, (prof["sigma2_hat"] * f, beta, nu))["loglik"] < prof["loglik"]


def test_profile_ar1_closed_form():
    # 1-D regular grid, nu = 1/2: R = rho^|i-j|, log|R| = (n-1) log(1 - rho^2),
    # q = z_1^2 + sum_{i>=2} (z_i - rho z_{i-1})^2 / (1 - rho^2)
    n, h, beta = 40, 0.03, 0.2
    rho = math.exp(-h / beta)
    locs = line_grid(n, h)
    z = normals(n, 9)
    q = z[0] ** 2 + sum((z[i] - rho * z[i - 1]) ** 2 for i in range(1, n)) / (1 - rho * rho)
    logdet = (n - 1) * math.log(1 - rho * rho)
    want = -0.5 * n * math.log(2 * math.pi) - 0.5 * n - 0.5 * n * math.log(q / n) - 0.5 * logdet
    got = oracle.profile_loglik(locs, z, beta, 0.5)
    assert got["loglik"] == pytest.approx(want, rel=1e-12)
    assert got["sigma2_hat"] == pytest.approx(q / n, rel=1e-12)


def test_profile_scale_equivariance():
    # Z -> c Z multiplies q by c^2, so l_p drops by n log c; eq. (2) itself has no such law
    locs = jittered_grid(10, seed=7)
    z = normals(len(locs), 8)
    a = oracle.profile_loglik(locs, z, 0.1, 0.5)["loglik"]
    b = oracle.profile_loglik(locs, 3.0 * z, 0.1, 0.5)["loglik"]
    assert b == pytest.approx(a - len(z) * math.log(3.0), rel=1e-12)


def test_stored_profile_fit_agrees_with_the_full_fit():
    # both searches maximise the same function of theta: the profile maximiser, completed
    # with theta1 = q/n, is the maximiser of eq. (2) (stored fits, each to its own tolerance)
    here = os.path.join(os.path.dirname(__file__), "golden")
    full = json.load(open(os.path.join(here, "mle_small.json")))
    prof = json.load(open(os.path.join(here, "mle_profile_small.json")))
    np.testing.assert_allclose(prof["theta_hat"], full["theta_hat"], rtol=1e-3)
    assert abs(prof["loglik_hat"] - full["loglik_hat"]) <= 1e-6 * abs(full["loglik_hat"])
    # the stored profile optimum is eq. (2) at its own theta_hat
    locs = SMALL.locations()
    z = oracle.simulate_field(locs, SMALL.theta, SMALL.eps())
    ll = oracle.loglik(locs, z, tuple(prof["theta_hat"]))["loglik"]
    assert ll == pytest.approx(prof["loglik_hat"], rel=1e-10)
