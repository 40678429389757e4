"""Pins for the oracle's great-circle distance (Section IV-B, large regions) and the
matching Morton key normalisation."""
import math

import numpy as np
import pytest

import oracle
from oracle.matern import EARTH_RADIUS_KM as R, great_circle
from oracle.morton import morton_keys
from synthetic import lonlat_grid, normals


def test_great_circle_special_values():
    assert great_circle(0.0, 0.0, 90.0, 0.0) == pytest.approx(math.pi * R / 2, rel=1e-15)
    assert great_circle(0.0, 90.0, 0.0, -90.0) == pytest.approx(math.pi * R, rel=1e-15)
    assert great_circle(17.0, 0.0, 197.0, 0.0) == pytest.approx(math.pi * R, rel=1e-15)  # antipodal
    assert great_circle(3.0, 0.0, 3.0, 1.0) == pytest.approx(R * math.pi / 180, rel=1e-14)
    assert great_circle(-40.0, 60.0, -40.0, 60.0) == 0.0
    # along a parallel at latitude 60 degrees, 1 degree of longitude: the chord of the small
    # circle of radius R cos 60 subtends the great-circle arc 2 R asin(cos60 sin(0.5 deg))
    want = 2 * R * math.asin(math.cos(math.radians(60)) * math.sin(math.radians(0.5)))
    assert great_circle(0.0, 60.0, 1.0, 60.0) == pytest.approx(want, rel=1e-13)


def _vincenty(lon1, lat1, lon2, lat2):
    # the atan2 form of the central angle (a different textbook formula, accurate everywhere)
    p1, p2, dl = math.radians(lat1), math.radians(lat2), math.radians(lon2 - lon1)
    num = math.hypot(math.cos(p2) * math.sin(dl),
                     math.cos(p1) * math.sin(p2) - math.sin(p1) * math.cos(p2) * math.cos(dl))
    den = math.sin(p1) * math.sin(p2) + math.cos(p1) * math.cos(p2) * math.cos(dl)
    return R * math.atan2(num, den)


def test_great_circle_agrees_with_the_atan2_formula():
    rng = np.random.default_rng(3)
    for _ in range(500):
        lon1, lon2 = rng.uniform(-180, 180, 2)
        lat1, lat2 = rng.uniform(-89, 89, 2)
        d = great_circle(lon1, lat1, lon2, lat2)
        assert d == pytest.approx(_vincenty(lon1, lat1, lon2, lat2), rel=1e-10, abs=1e-9)


def test_great_circle_small_distance_limit_and_metric_axioms():
    # at short range the sphere is locally flat: d ~ R sqrt(dlat^2 + (cos lat dlon)^2)
    lat0 = 25.0
    d = great_circle(40.0, lat0, 40.01, lat0 + 0.02)
    flat = R * math.hypot(math.radians(0.02), math.cos(math.radians(lat0 + 0.01)) * math.radians(0.01))
    assert d == pytest.approx(flat, rel=1e-7)
    pts = lonlat_grid(6, 4)
    dm = oracle.distances(pts, "gcd")
    assert np.allclose(dm, dm.T, rtol=0, atol=1e-9)
    assert np.all(np.diag(dm) == 0.0)
    n = len(pts)
    for a in range(n):
        assert np.all(dm[a][:, None] <= dm[a][None, :] + dm + 1e-9)   # triangle inequality


def test_gcd_morton_keys():
    pts = np.array([[-180.0, -90.0], [180.0, 90.0], [0.0, 0.0], [-90.0, 0.0]])
    keys = morton_keys(pts, "gcd")
    assert keys[0] == 0
    assert keys[1] == 0xFFFFFFFF
    assert keys[2] == (1 << 30) | (1 << 31)        # (0.5, 0.5): bit 15 of both coordinates
    assert keys[3] == (1 << 31) | (1 << 28)        # (0.25, 0.5): qx = 2^14, qy = 2^15


def test_gcd_likelihood_of_a_tiny_problem_by_brute_force():
    # eq. (2) with great-circle distances on 6 sites against the determinant and inverse
    # computed independently (numpy det / solve on the same Sigma)
    pts = lonlat_grid(3, 9)[:6]
    theta = (1.2, 300.0, 0.5)
    z = normals(6, 10)
    sig = np.array([[theta[0] * math.exp(-great_circle(a[0], a[1], b[0], b[1]) / theta[1])
                     for b in pts] for a in pts])
    sign, logdet = np.linalg.slogdet(sig)
    quad = float(z @ np.linalg.solve(sig, z))
    want = -3 * math.log(2 * math.pi) - 0.5 * logdet - 0.5 * quad
    got = oracle.loglik(pts, z, theta, "gcd")
    assert sign > 0
    assert got["loglik"] == pytest.approx(want, rel=1e-12)
