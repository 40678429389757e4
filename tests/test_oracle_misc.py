"""Pins for the oracle's Morton ordering, kriging and Nelder-Mead."""
import math

import numpy as np
import pytest

from oracle import krige, morton_keys, morton_order, nelder_mead
from oracle.morton import morton_key
from synthetic import jittered_grid, line_grid, normals


def test_morton_hand_computed_keys():
    # q = floor(c * 65536): x bits go to even positions, y bits to odd ones.
    assert morton_key(0.0, 0.0) == 0
    assert morton_key(1.0 / 65536, 0.0) == 0b01          # qx = 1
    assert morton_key(0.0, 1.0 / 65536) == 0b10          # qy = 1
    assert morton_key(3.0 / 65536, 5.0 / 65536) == 0b100111  # qx=011, qy=101 -> y2 x2 y1 x1 y0 x0
    assert morton_key(0.5, 0.0) == 1 << 30                # qx = 2^15
    assert morton_key(0.0, 0.5) == 1 << 31
    assert morton_key(1.0, 1.0) == 0xFFFFFFFF             # clamped to 2^16 - 1
    assert morton_key(-0.2, 2.0) == 0xAAAAAAAA            # qx = 0, qy = 65535


def test_morton_order_sorts_and_is_a_bijection():
    locs = jittered_grid(30, seed=12)
    perm = morton_order(locs)
    assert sorted(perm.tolist()) == list(range(len(locs)))
    keys = morton_keys(locs)[perm]
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)


def test_morton_ties_keep_input_order():
    locs = np.array([[0.5, 0.5], [0.1, 0.1], [0.5, 0.5], [0.1, 0.1]])
    assert morton_order(locs).tolist() == [1, 3, 0, 2]


def test_kriging_interpolates_observed_sites():
    locs = jittered_grid(8, seed=2)
    z = normals(len(locs), 3)
    out = krige(locs, z, (1.0, 0.1, 1.0), locs[[3, 17, 40]])
    np.testing.assert_allclose(out["pred"], z[[3, 17, 40]], rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(out["var"], 0.0, atol=1e-8)


def test_kriging_ou_bridge_closed_form():
    # 1-D exponential kernel = Ornstein-Uhlenbeck process: the prediction between
    # two neighbours s_k < x < s_k+1 depends on those two only.
    sigma2, beta, h = 1.4, 0.2, 0.05
    locs = line_grid(30, h)
    z = normals(30, 4)
    xs = np.array([0.3 * h, 7.5 * h, 21.9 * h])
    new = np.stack([xs, np.zeros_like(xs)], axis=1)
    out = krige(locs, z, (sigma2, beta, 0.5), new)
    for x, pred, var in zip(xs, out["pred"], out["var"]):
        k = int(x // h)
        s0, s1 = k * h, (k + 1) * h
        den = math.sinh((s1 - s0) / beta)
        w1, w2 = math.sinh((s1 - x) / beta) / den, math.sinh((x - s0) / beta) / den
        assert pred == pytest.approx(w1 * z[k] + w2 * z[k + 1], rel=1e-10)
        v = sigma2 * (1 - w1 * math.exp(-(x - s0) / beta) - w2 * math.exp(-(s1 - x) / beta))
        assert var == pytest.approx(v, rel=1e-8)


def test_nelder_mead_finds_known_minima():
    quadratic = lambda x: float(np.sum((x - np.array([0.3, -1.2, 2.0])) ** 2 * np.array([1, 10, 3])))
    res = nelder_mead(quadratic, [0, 0, 0], step=0.5, xtol=1e-9, ftol=0, max_evals=5000)
    np.testing.assert_allclose(res["x"], [0.3, -1.2, 2.0], atol=1e-7)

    def rosen(x):
        return float(sum(100 * (x[i + 1] - x[i] ** 2) ** 2 + (1 - x[i]) ** 2 for i in range(2)))

    res = nelder_mead(rosen, [-1.0, 1.5, 0.5], step=0.5, xtol=1e-10, ftol=0, max_evals=20000)
    np.testing.assert_allclose(res["x"], [1, 1, 1], atol=1e-6)


def test_stored_mle_is_a_profile_maximum():
    # For fixed (range, smoothness) eq. (2) is maximised over the variance by
    # sigma2 = Z^T Sigma~^-1 Z / n (Sigma~ at unit variance).  The stored oracle fit must
    # satisfy this closed form to the optimiser's tolerance.
    import json
    import os

    from oracle import loglik, simulate_field
    from synthetic import SMALL
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mle_small.json")))
    s2, beta, nu = gold["theta_hat"]
    locs = SMALL.locations()
    z = simulate_field(locs, SMALL.theta, SMALL.eps())
    q = loglik(locs, z, (1.0, beta, nu))["quad"]
    assert abs(s2 - q / len(z)) / s2 <= 1e-4
    assert abs(loglik(locs, z, (s2, beta, nu))["loglik"] - gold["loglik_hat"]) <= 1e-8 * abs(gold["loglik_hat"])
