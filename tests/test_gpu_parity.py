"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances:
  * all-FP64 path:       |dl| / |l| <= 1e-10 (also logdet and quad);
  * FP64/FP32 band path: |dl| / |l| <= 1e-5 where l is well away from zero (the n = 1,600
    workload: |l| ~ 1,200 at every theta), |dl| / max(|l|, n) <= 1e-5 for the small random
    problems whose l can pass through zero;
  * third tier (FP16 operands): |dl| / |l| <= 1e-5; BF16 where its FP32 width makes it;
  * Morton permutation:  bit-exact;
  * covariance entries:  FP64 tiles within 1e-13 relative of the oracle for nu = 1/2 (both
    sides elementary) and 5e-13 for general nu (the oracle's Bessel routine itself is good
    to about 1e-13 near x = 2); FP32 tiles within one FP32 ulp of the oracle value.
"""
import ctypes
import functools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from synthetic import SMALL, jittered_grid, line_grid, lonlat_grid, normals, perturbed_thetas

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@functools.lru_cache(maxsize=None)
def small_case():
    locs = SMALL.locations()
    z = oracle.simulate_field(locs, SMALL.theta, SMALL.eps())
    return locs, z


@functools.lru_cache(maxsize=None)
def small_oracle(theta):
    locs, z = small_case()
    out = oracle.loglik(locs, z, theta)
    return {k: out[k] for k in ("loglik", "logdet", "quad")}


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def small_ds(lib, ctx):
    locs, z = small_case()
    ds = lib.Dataset(ctx, locs, z)
    yield ds
    ds.close()


def rel(a, b):
    return abs(a - b) / abs(b)


def test_morton_permutation_is_bit_exact(small_ds):
    locs, _ = small_case()
    assert np.array_equal(small_ds.perm(), oracle.morton_order(locs))


@pytest.mark.parametrize("theta,band", [((1.0, 0.1, 0.5), 2), ((1.3, 0.2, 0.73), 1),
                                        ((0.9, 0.05, 1.0), 0), ((1.0, 0.1, 1.5), -1),
                                        ((1.0, 0.1, 0.3), -1), ((0.8, 0.3, 2.2), -1),
                                        ((1.1, 0.02, 0.49), 2)])
def test_covariance_entries(small_ds, theta, band):
    locs, _ = small_case()
    tile = SMALL.tile
    got = small_ds.covariance(theta, tile, band)
    want = oracle.matern_matrix(locs[small_ds.perm()], theta)
    n = want.shape[0]
    ti = np.arange(n) // tile
    dist = ti[:, None] - ti[None, :]
    lower = np.tril(np.ones((n, n), dtype=bool))
    fp64 = lower & ((dist <= band) if band >= 0 else True)
    fp32 = lower & ~fp64
    tol = 1e-13 if theta[2] in (0.5, 1.5, 2.5) else 5e-13
    err64 = np.abs(got[fp64] - want[fp64]) / np.maximum(np.abs(want[fp64]), 1e-300)
    assert err64.max() <= tol
    if fp32.any():
        w32 = want[fp32].astype(np.float32)
        ulp = np.spacing(np.abs(w32)).astype(np.float64)
        assert np.all(np.abs(got[fp32] - w32.astype(np.float64)) <= ulp)
        assert np.all(got[fp32] == got[fp32].astype(np.float32))   # stored as FP32


@pytest.mark.parametrize("theta", [SMALL.theta] + perturbed_thetas(SMALL.theta))
def test_fp64_path_matches_oracle(small_ds, theta):
    want = small_oracle(tuple(theta))
    got = small_ds.loglik(theta, SMALL.tile, -1)
    assert rel(got["loglik"], want["loglik"]) <= 1e-10
    assert rel(got["logdet"], want["logdet"]) <= 1e-10
    assert rel(got["quad"], want["quad"]) <= 1e-10


@pytest.mark.parametrize("band", [2, 1, 0])
@pytest.mark.parametrize("theta", [SMALL.theta] + perturbed_thetas(SMALL.theta))
def test_band_path_matches_oracle(small_ds, theta, band):
    want = small_oracle(tuple(theta))
    got = small_ds.loglik(theta, SMALL.tile, band)
    assert rel(got["loglik"], want["loglik"]) <= 1e-5


def test_one_shot_equals_resident_dataset(lib, ctx, small_ds):
    locs, z = small_case()
    a = ctx.loglik(locs, z, SMALL.theta, SMALL.tile, SMALL.band64)
    b = small_ds.loglik(SMALL.theta, SMALL.tile, SMALL.band64)
    assert a["loglik"] == b["loglik"] and a["logdet"] == b["logdet"]


def test_device_inputs(lib, ctx, small_ds):
    import torch
    locs, z = small_case()
    dl = torch.from_numpy(locs).to("cuda:0")
    dz = torch.from_numpy(z).to("cuda:0")
    a = ctx.loglik(dl, dz, SMALL.theta, SMALL.tile, SMALL.band64)
    b = small_ds.loglik(SMALL.theta, SMALL.tile, SMALL.band64)
    assert a["loglik"] == b["loglik"]


def test_factor_and_forward_solve_entries(small_ds):
    locs, z = small_case()
    theta = (1.0, 0.1, 1.0)
    small_ds.loglik(theta, SMALL.tile, -1)
    perm = small_ds.perm()
    s = oracle.matern_matrix(locs[perm], theta)
    low = oracle.cholesky_lower(s)
    got = small_ds.matrix()
    assert np.max(np.abs(np.tril(got) - low)) <= 1e-11 * np.max(np.abs(low))
    y = sla.solve_triangular(low, z[perm], lower=True)
    np.testing.assert_allclose(small_ds.solution(), y, rtol=0, atol=1e-10 * np.max(np.abs(y)))


@pytest.mark.parametrize("n,tile", [(50, 7), (50, 16), (77, 32), (77, 50), (64, 64), (130, 33)])
@pytest.mark.parametrize("band", [-1, 0, 1])
def test_ar1_closed_form_ragged_tiles(lib, ctx, n, tile, band):
    h, sigma2, beta = 0.007, 1.6, 0.05
    locs = line_grid(n, h)
    z = normals(n, 3 + n)
    rho = math.exp(-h / beta)
    logdet = n * math.log(sigma2) + (n - 1) * math.log(1 - rho * rho)
    quad = z[0] ** 2 / sigma2 + sum((z[i] - rho * z[i - 1]) ** 2 for i in range(1, n)) / (
        sigma2 * (1 - rho * rho))
    got = ctx.loglik(locs, z, (sigma2, beta, 0.5), tile, band)
    if band < 0 or band >= (n + tile - 1) // tile - 1:      # every tile FP64
        assert rel(got["logdet"], logdet) <= 1e-11
        assert rel(got["quad"], quad) <= 1e-11
    else:
        want = -0.5 * n * math.log(2 * math.pi) - 0.5 * logdet - 0.5 * quad
        assert abs(got["loglik"] - want) / max(abs(want), n) <= 1e-5


def _exact_loglik(a, z):
    from fractions import Fraction
    n = len(z)
    m = [[Fraction(float(a[i, j])) for j in range(n)] + [Fraction(float(z[i]))] for i in range(n)]
    det = Fraction(1)
    for c in range(n):
        det *= m[c][c]
        for r in range(c + 1, n):
            f = m[r][c] / m[c][c]
            for k in range(c, n + 1):
                m[r][k] -= f * m[c][k]
    x = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        x[r] = (m[r][n] - sum(m[r][k] * x[k] for k in range(r + 1, n))) / m[r][r]
    quad = float(sum(Fraction(float(z[i])) * x[i] for i in range(n)))
    logdet = math.log(det)
    return -0.5 * n * math.log(2 * math.pi) - 0.5 * logdet - 0.5 * quad


@pytest.mark.parametrize("n", [5, 9, 12])
@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6])
def test_tiny_problems_every_band(lib, ctx, n, tile):
    rng = np.random.default_rng(100 * n + tile)
    locs = rng.uniform(0, 1, size=(n, 2))
    z = normals(n, n + tile)
    theta = (1.2, 0.3, 0.8)
    perm = oracle.morton_order(locs)
    want = _exact_loglik(oracle.matern_matrix(locs[perm], theta), z[perm])
    p = (n + tile - 1) // tile
    for band in list(range(p)) + [-1]:
        got = ctx.loglik(locs, z, theta, tile, band)["loglik"]
        if band < 0 or band >= p - 1:
            assert rel(got, want) <= 1e-10, (band, got, want)
        else:
            assert abs(got - want) / max(abs(want), n) <= 1e-5, (band, got, want)


def _block_banded_spd(n, tile, width, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n))
    a = (a + a.T) / 2
    ti = np.arange(n) // tile
    a[np.abs(ti[:, None] - ti[None, :]) > width] = 0.0
    a += np.eye(n) * (np.abs(a).sum(axis=1).max() + 1.0)    # diagonally dominant -> SPD
    return a


def test_block_banded_matrix_is_exact_for_every_wider_band(lib, ctx):
    n, tile, width = 200, 32, 2
    a = _block_banded_spd(n, tile, width, 5)
    z = normals(n, 6)
    want = oracle.likelihood.loglik_parts(a, z)
    results = [ctx.factor_dense(a, z, tile, band) for band in (width, width + 1, 5, -1)]
    for r in results:
        assert r["loglik"] == results[0]["loglik"]
        assert r["logdet"] == results[0]["logdet"]
    assert rel(results[0]["logdet"], want["logdet"]) <= 1e-12
    assert rel(results[0]["quad"], want["quad"]) <= 1e-12


def test_factor_dense_matches_oracle_on_random_spd(lib, ctx):
    from synthetic import random_spd
    a = random_spd(300, 9)
    z = normals(300, 10)
    want = oracle.likelihood.loglik_parts(a, z)
    got = ctx.factor_dense(a, z, 64, -1)
    assert rel(got["loglik"], want["loglik"]) <= 1e-10
    got = ctx.factor_dense(a, z, 64, 0)
    assert abs(got["loglik"] - want["loglik"]) / max(abs(want["loglik"]), 300) <= 1e-5


@pytest.mark.parametrize("col", [0, 37, 63])
def test_not_positive_definite_reports_failing_column(lib, ctx, col):
    n = 64
    a = np.eye(n) * 2.0
    a[col, col] = -1.0
    with pytest.raises(lib.MpgeoError) as exc:
        ctx.factor_dense(a, None, 16, -1)
    assert exc.value.status == lib.MPGEO_E_NOT_SPD
    assert exc.value.info == col


def test_permutation_invariance_of_fp64_path(lib, ctx):
    locs, z = small_case()
    perm = np.random.default_rng(1).permutation(len(z))
    a = ctx.loglik(locs, z, SMALL.theta, SMALL.tile, -1, morton=False)
    b = ctx.loglik(locs[perm], z[perm], SMALL.theta, SMALL.tile, -1, morton=False)
    assert rel(a["loglik"], b["loglik"]) <= 1e-12


@pytest.mark.parametrize("band", [-1, 2])
def test_kriging_matches_oracle(lib, ctx, band):
    locs = jittered_grid(24, 41)
    theta = (1.0, 0.1, 0.5)
    z = oracle.simulate_field(locs, theta, normals(len(locs), 42))
    new = np.random.default_rng(43).uniform(0, 1, size=(40, 2))
    want = oracle.krige(locs, z, theta, new)
    ds = lib.Dataset(ctx, locs, z)
    ds.loglik(theta, 96, band)
    pred, var = ds.krige(new, variance=True)
    tol = 1e-9 if band < 0 else 1e-4
    assert np.max(np.abs(pred - want["pred"])) <= tol * np.max(np.abs(want["pred"]))
    assert np.max(np.abs(var - want["var"])) <= tol * theta[0]
    # interpolation at observed sites (FP64 path)
    if band < 0:
        at = ds.krige(locs[[3, 100, 500]])
        np.testing.assert_allclose(at, z[[3, 100, 500]], atol=1e-8)
    ds.close()


@pytest.mark.parametrize("band", [-1, 2])
def test_field_sampler_matches_oracle(lib, ctx, band):
    # z = P^T L P eps: the oracle draws the same field in the ordered frame
    locs = jittered_grid(30, 51)
    eps = normals(len(locs), 52)
    theta = (1.1, 0.08, 0.5)
    ds = lib.Dataset(ctx, locs, None)
    z = ds.simulate(theta, eps, 128, band)
    perm = ds.perm()
    ds.close()
    want = np.empty(len(locs))
    want[perm] = oracle.simulate_field(locs[perm], theta, eps[perm])
    tol = 1e-11 if band < 0 else 1e-5
    assert np.max(np.abs(z - want)) <= tol * np.max(np.abs(want))


def test_argument_validation(lib, ctx, small_ds):
    with pytest.raises(lib.MpgeoError) as e:
        small_ds.loglik((1.0, -0.1, 0.5), 160, 2)
    assert e.value.status == lib.MPGEO_E_ARG
    with pytest.raises(lib.MpgeoError) as e:
        small_ds.loglik((1.0, 0.1, float("nan")), 160, 2)
    assert e.value.status == lib.MPGEO_E_ARG
    with pytest.raises(lib.MpgeoError) as e:
        small_ds.loglik((1.0, 0.1, 0.5), 1024, 2)
    assert e.value.status == lib.MPGEO_E_ARG
    with pytest.raises(lib.MpgeoError) as e:
        small_ds.loglik((1.0, 0.1, 0.5), 160, -2)
    assert e.value.status == lib.MPGEO_E_ARG


@pytest.mark.parametrize("band", [2, -1])
def test_mle_matches_oracle(lib, small_ds, band):
    gold = json.load(open(os.path.join(HERE, "golden", "mle_small.json")))
    start = [min(max(t * s, lo), hi) for t, s, lo, hi in
             zip(SMALL.theta, oracle.mle.START_SCALE, oracle.mle.LOWER, oracle.mle.UPPER)]
    fit = small_ds.mle(start, SMALL.tile, band)
    for got, want in zip(fit["theta"], gold["theta_hat"]):
        assert abs(got - want) / abs(want) <= 1e-3, (fit, gold)


def test_mle_trace_is_the_search(lib, small_ds):
    # the recorded trajectory is the search itself: same fit as mpgeo_dataset_mle, one entry per
    # evaluation starting at the start point, the fit's log-likelihood its best entry, and each
    # entry the log-likelihood a separate evaluation of that theta gives, bit for bit
    start = [min(max(t * s, lo), hi) for t, s, lo, hi in
             zip(SMALL.theta, oracle.mle.START_SCALE, oracle.mle.LOWER, oracle.mle.UPPER)]
    fit = small_ds.mle(start, SMALL.tile, 2, xtol=1e-4)
    tr = small_ds.mle_trace(start, SMALL.tile, 2, xtol=1e-4)
    assert tr["theta"] == fit["theta"] and tr["loglik"] == fit["loglik"] and tr["evals"] == fit["evals"]
    assert len(tr["trace"]) == tr["evals"] and tr["evals"] >= 4
    assert np.allclose(tr["trace"][0], start, rtol=1e-14, atol=0)
    best = int(np.argmax(tr["trace_loglik"]))
    assert tr["trace_loglik"][best] == fit["loglik"]
    assert np.allclose(tr["trace"][best], fit["theta"], rtol=1e-14, atol=0)
    for e in (0, tr["evals"] // 2, tr["evals"] - 1):
        assert small_ds.loglik(tr["trace"][e], SMALL.tile, 2)["loglik"] == tr["trace_loglik"][e]
    with pytest.raises(lib.MpgeoError):
        small_ds.mle_trace(start, SMALL.tile, 2, max_evals=3)


# ---- third precision tier (16-bit operands for the farthest tiles) -------------------------
# Bar: the mixed paths' 1e-5 on |dl| / |l|.  FP16 (u = 2^-11 per operand) meets it at every FP32
# width here; BF16 (u = 2^-8) needs FP32 tiles beyond the band (width >= 2): with width 0 its
# error reaches 2e-5 at some of the nine theta, a reported row, held only to the derived worst
# case 20u of a BF16 operand tier (each far-tile update errs by at most 2u of
# sum |L_ik||L_jk| <= theta1, entering l through tr(Sigma^-1 dSigma) and the quadratic form).
LOWP_BAR = 1e-5
LOWP_WORST = {"fp16": 20 * 2.0 ** -11, "bf16": 20 * 2.0 ** -8}


@pytest.mark.parametrize("lowp", ["fp16", "bf16"])
@pytest.mark.parametrize("band32", [0, 2, 5])
@pytest.mark.parametrize("theta", [SMALL.theta] + perturbed_thetas(SMALL.theta))
def test_three_tier_matches_oracle(small_ds, theta, lowp, band32):
    want = small_oracle(tuple(theta))
    got = small_ds.loglik(theta, SMALL.tile, 2, band32=band32, lowp=lowp)
    err = rel(got["loglik"], want["loglik"])
    asserted = lowp == "fp16" or band32 >= 2
    print(f"three-tier {lowp} band64=2 band32={band32} theta={theta}: |dl|/|l| = {err:.3e}"
          f"{'' if asserted else ' (reported row)'}")
    assert err <= (LOWP_BAR if asserted else LOWP_WORST[lowp])
    # the two-tier path is the c -> infinity limit: more FP32 tiles never hurts much
    two = small_ds.loglik(theta, SMALL.tile, 2)
    assert rel(two["loglik"], want["loglik"]) <= max(err, 1e-6)


@pytest.mark.parametrize("lowp", ["fp16", "bf16"])
def test_three_tier_block_banded_is_exact(lib, ctx, lowp):
    # far tiles exactly zero: their 16-bit copies are exact zeros, so every tier gives the
    # FP64 result bit for bit
    n, tile, width = 256, 32, 1
    a = _block_banded_spd(n, tile, width, 15)
    z = normals(n, 16)
    ref = ctx.factor_dense(a, z, tile, -1)
    got = ctx.factor_dense(a, z, tile, width, band32=0, lowp=lowp)
    assert got["loglik"] == ref["loglik"]
    assert got["logdet"] == ref["logdet"]


@pytest.mark.parametrize("band64,band32,lowp", [(-1, -1, None), (2, -1, None), (2, 4, "fp16"),
                                                 (2, 4, "bf16")])
def test_row_scaling_by_powers_of_two_is_exact(lib, ctx, band64, band32, lowp):
    # Scaling the rows and columns of Sigma by powers of two, D Sigma D with D = diag(2^e_r), and
    # the data by D scales every entry of the factor exactly (binary floating point, no
    # overflow or underflow here), and each tile row's 16-bit scale follows from its own
    # diagonal, so l(D Sigma D, D y) + sum_r log d_r must equal l(Sigma, y) up to the rounding
    # of the logarithms.  A scale shared by all rows would flush the rows scaled by 2^-20 to
    # zero in FP16.
    n, tile = 1024, 64
    locs = jittered_grid(32, 51)
    sigma = oracle.matern_matrix(locs[oracle.morton_order(locs)], (1.0, 0.1, 0.5))
    y = normals(n, 52)
    e = ((np.arange(n) // tile) % 5 - 2) * 10.0          # 2^-20 .. 2^20 by tile row
    d = np.exp2(e)
    ref = ctx.factor_dense(sigma, y, tile, band64, band32=band32, lowp=lowp)
    got = ctx.factor_dense(sigma * d[:, None] * d[None, :], y * d, tile, band64, band32=band32, lowp=lowp)
    shift = float(np.sum(e) * np.log(2.0))
    err = abs(got["loglik"] + shift - ref["loglik"]) / max(abs(ref["loglik"]), n)
    print(f"band64={band64} band32={band32} lowp={lowp}: l = {ref['loglik']:.10f}, scaled + shift "
          f"= {got['loglik'] + shift:.10f}, rel {err:.2e}")
    assert err <= 1e-12
    assert got["quad"] == ref["quad"]


def test_three_tier_bits_do_not_depend_on_pass_grouping(lib, ctx):
    # n = 40,000, tile 256: up to about 140 far tiles per column, more than one wave of the
    # 16-bit pass on part of the GPU.  A context that leaves compute units to the critical path
    # (MPGEO_RESERVED_CUS) sizes the waves differently, so the layout groups the far tiles'
    # panels into different passes (and runs all bulk updates on one stream); each element
    # still takes the same FP32 accumulation sequence, so l must agree bit for bit.
    m = 200
    locs = jittered_grid(m, 41)
    z = normals(m * m, 42)
    theta = (1.0, 0.1, 0.5)
    plan = dict(band32=8, lowp="fp16")
    ds = lib.Dataset(ctx, locs, z)
    try:
        ref = ds.loglik(theta, 256, 2, **plan)
    finally:
        ds.close()
    os.environ["MPGEO_RESERVED_CUS"] = "100"
    try:
        ctx2 = lib.Context(0)
    finally:
        del os.environ["MPGEO_RESERVED_CUS"]
    try:
        ds2 = lib.Dataset(ctx2, locs, z)
        try:
            got = ds2.loglik(theta, 256, 2, **plan)
        finally:
            ds2.close()
    finally:
        ctx2.close()
    print(f"three-tier n={m * m}: l = {ref['loglik']!r} (reserved compute units: {got['loglik']!r})")
    assert got["loglik"] == ref["loglik"]
    assert got["logdet"] == ref["logdet"]


def test_three_tier_plan_validation(lib, small_ds):
    for band32, lowp in [(2, None), (-1, "fp16")]:
        with pytest.raises(lib.MpgeoError) as e:
            small_ds.loglik(SMALL.theta, SMALL.tile, 2, band32=band32, lowp=lowp)
        assert e.value.status == lib.MPGEO_E_ARG


# ---- profile likelihood in (theta2, theta3) ---------------------------------------------------
@pytest.mark.parametrize("band,tol", [(-1, 1e-10), (2, 1e-5)])
@pytest.mark.parametrize("theta", [SMALL.theta, (0.7, 0.13, 0.62)])
def test_profile_likelihood_matches_oracle(small_ds, theta, band, tol):
    locs, z = small_case()
    want = oracle.profile_loglik(locs, z, theta[1], theta[2])
    got = small_ds.loglik(theta, SMALL.tile, band, profile=True)   # theta1 is ignored
    assert abs(got["loglik"] - want["loglik"]) / max(abs(want["loglik"]), len(z)) <= tol
    assert rel(got["quad"], want["quad"]) <= (1e-10 if band < 0 else 1e-4)
    # eq. (2) through the library at the variance estimate q/n equals the profile value
    full = small_ds.loglik((got["quad"] / len(z), theta[1], theta[2]), SMALL.tile, band)
    assert abs(full["loglik"] - got["loglik"]) / max(abs(got["loglik"]), len(z)) <= tol


def test_profile_kriging_uses_the_variance_estimate(lib, ctx):
    locs = jittered_grid(20, 61)
    theta = (1.4, 0.1, 0.5)
    z = oracle.simulate_field(locs, theta, normals(len(locs), 62))
    new = np.random.default_rng(63).uniform(0, 1, size=(25, 2))
    ds = lib.Dataset(ctx, locs, z)
    r = ds.loglik(theta, 80, -1, profile=True)
    s2 = r["quad"] / len(z)
    pred, var = ds.krige(new, variance=True)
    ds.close()
    want = oracle.krige(locs, z, (s2, theta[1], theta[2]), new)
    assert np.max(np.abs(pred - want["pred"])) <= 1e-9 * np.max(np.abs(want["pred"]))
    assert np.max(np.abs(var - want["var"])) <= 1e-9 * s2


@pytest.mark.parametrize("band", [2, -1])
def test_profile_mle_matches_oracle(lib, small_ds, band):
    gold = json.load(open(os.path.join(HERE, "golden", "mle_profile_small.json")))
    start = [min(max(t * s, lo), hi) for t, s, lo, hi in
             zip(SMALL.theta, oracle.mle.START_SCALE, oracle.mle.LOWER, oracle.mle.UPPER)]
    fit = small_ds.mle(start, SMALL.tile, band, profile=True)
    for got, want in zip(fit["theta"], gold["theta_hat"]):
        assert abs(got - want) / abs(want) <= 1e-3, (fit, gold)


def test_profile_rejected_where_it_has_no_meaning(lib, small_ds):
    # a field draw needs the variance: simulate refuses the profile flag
    eps = np.zeros(small_ds.n)
    out = np.zeros(small_ds.n)
    st = lib.LIB.mpgeo_dataset_simulate(small_ds.handle, lib.Theta(*SMALL.theta),
                                        lib.make_plan(SMALL.tile, 2, lib.MPGEO_PROFILE),
                                        eps.ctypes.data, out.ctypes.data)
    assert st == lib.MPGEO_E_ARG


# ---- great-circle distance ((lon, lat) in degrees) -----------------------------------------
GCD_THETA = (1.0, 150.0, 0.5)     # range 150 km on a 20 x 20 degree box (~2,000 km)


@functools.lru_cache(maxsize=None)
def gcd_case(m=30, seed=71):
    locs = lonlat_grid(m, seed)
    z = oracle.simulate_field(locs, GCD_THETA, normals(len(locs), seed + 1), "gcd")
    return locs, z


def test_gcd_morton_permutation_is_bit_exact(lib, ctx):
    locs, z = gcd_case()
    ds = lib.Dataset(ctx, locs, z, gcd=True)
    assert np.array_equal(ds.perm(), oracle.morton_order(locs, "gcd"))
    ds.close()


@pytest.mark.parametrize("theta", [GCD_THETA, (1.3, 90.0, 1.1)])
def test_gcd_covariance_entries(lib, ctx, theta):
    locs, z = gcd_case()
    ds = lib.Dataset(ctx, locs, z, gcd=True)
    got = ds.covariance(theta, 128, -1)
    perm = ds.perm()
    ds.close()
    want = oracle.matern_matrix(locs[perm], theta, "gcd")
    low = np.tril_indices(len(z))
    tol = 1e-13 if theta[2] == 0.5 else 5e-13
    np.testing.assert_allclose(got[low], want[low], rtol=tol, atol=0)


@pytest.mark.parametrize("band,tol", [(-1, 1e-10), (1, 1e-5)])
def test_gcd_loglik_and_kriging_match_oracle(lib, ctx, band, tol):
    locs, z = gcd_case()
    want = oracle.loglik(locs, z, GCD_THETA, "gcd")
    got = ctx.loglik(locs, z, GCD_THETA, 128, band, gcd=True)
    assert abs(got["loglik"] - want["loglik"]) / max(abs(want["loglik"]), len(z)) <= tol
    new = lonlat_grid(6, 77)
    kr = oracle.krige(locs, z, GCD_THETA, new, "gcd")
    ds = lib.Dataset(ctx, locs, z, gcd=True)
    ds.loglik(GCD_THETA, 128, band)
    pred, var = ds.krige(new, variance=True)
    ds.close()
    ktol = 1e-9 if band < 0 else 1e-4
    assert np.max(np.abs(pred - kr["pred"])) <= ktol * np.max(np.abs(kr["pred"]))
    assert np.max(np.abs(var - kr["var"])) <= ktol * GCD_THETA[0]


# ---- dropped tiles (diagonal super tile: tiles beyond band0 taken as zero) -----------------
def test_dropped_tiles_are_exact_on_a_block_banded_matrix(lib, ctx):
    # a matrix of tile bandwidth w has a Cholesky factor of the same bandwidth, so dropping
    # the tiles beyond any band0 >= w changes nothing (bitwise: only exact zeros are skipped)
    n, tile, width = 200, 32, 2
    a = _block_banded_spd(n, tile, width, 5)
    z = normals(n, 6)
    full = ctx.factor_dense(a, z, tile, -1)
    for band0 in (width, width + 1, 6):
        for band in (-1, 1):
            r = ctx.factor_dense(a, z, tile, band, band0=band0)
            ref = full if band < 0 else ctx.factor_dense(a, z, tile, band)
            assert r["loglik"] == ref["loglik"], (band0, band)
            assert r["logdet"] == ref["logdet"], (band0, band)


@pytest.mark.parametrize("theta,band0", [((1.0, 0.1, 0.5), 0), ((1.0, 0.1, 0.5), 3),
                                         ((1.0, 0.1, 0.5), 6), ((1.0, 0.03, 0.5), 1),
                                         ((1.0, 0.03, 0.5), 2), ((1.0, 0.03, 0.5), 5)])
@pytest.mark.parametrize("band,tol", [(-1, 1e-10), (1, 1e-5)])
def test_dropped_tiles_match_the_truncated_matrix(small_ds, theta, band0, band, tol):
    # the oracle's definition: Sigma in the ordered frame with every entry of a tile farther
    # than band0 from the diagonal set to zero, then eq. (2); it may not be positive definite,
    # in which case the library must say so
    locs, z = small_case()
    perm = oracle.morton_order(locs)
    sig = oracle.matern_matrix(locs[perm], theta)
    ti = np.arange(len(z)) // SMALL.tile
    sig[np.abs(ti[:, None] - ti[None, :]) > band0] = 0.0
    try:
        want = oracle.likelihood.loglik_parts(sig, z[perm])
    except oracle.likelihood.NotPositiveDefinite:
        want = None
    st, got = small_ds.try_loglik(theta, SMALL.tile, band, band0=band0)
    if want is None:
        assert st == 2, (st, got)       # MPGEO_E_NOT_SPD
        return
    assert st == 0
    assert abs(got["loglik"] - want["loglik"]) / max(abs(want["loglik"]), len(z)) <= tol
    # dropped tiles read back as zero
    if band0 < 2:
        far = small_ds.entries(np.array([len(z) - 1]), np.array([0]))
        assert far[0] == 0.0


@pytest.mark.parametrize("lowp", ["fp16", "bf16"])
@pytest.mark.parametrize("band0", [4, 6])
def test_dropped_tiles_with_a_16bit_tier(small_ds, lowp, band0):
    # three tiers under a dropped band: FP64 for i - j <= 1, FP32 for 2, 16-bit operands for
    # 3 .. band0, zero beyond.  The 16-bit tiles take their earlier panels in one pass that
    # skips the dropped panels (k < i - band0); the truncated matrix of the oracle decides.
    theta = (1.0, 0.03, 0.5)
    locs, z = small_case()
    perm = oracle.morton_order(locs)
    sig = oracle.matern_matrix(locs[perm], theta)
    ti = np.arange(len(z)) // SMALL.tile
    sig[np.abs(ti[:, None] - ti[None, :]) > band0] = 0.0
    want = oracle.likelihood.loglik_parts(sig, z[perm])   # positive definite at this range
    got = small_ds.loglik(theta, SMALL.tile, 1, band32=1, lowp=lowp, band0=band0)
    err = rel(got["loglik"], want["loglik"])
    print(f"dropped tiles beyond {band0}, three tiers {lowp}: |dl|/|l| = {err:.3e}")
    assert err <= LOWP_BAR


# ---- precision map drawn from distances -----------------------------------------------------
def _tile_box_distances(ordered, tile):
    p = -(-len(ordered) // tile)
    boxes = []
    for i in range(p):
        blk = ordered[i * tile:(i + 1) * tile]
        boxes.append((blk[:, 0].min(), blk[:, 0].max(), blk[:, 1].min(), blk[:, 1].max()))
    d = np.zeros((p, p))
    for i in range(p):
        for j in range(p):
            a, b = boxes[i], boxes[j]
            dx = max(0.0, a[0] - b[1], b[0] - a[1])
            dy = max(0.0, a[2] - b[3], b[2] - a[3])
            d[i, j] = math.hypot(dx, dy)
    return d


@pytest.mark.parametrize("dist64", [0.02, 0.1, 0.3])
def test_distance_map_tiers_follow_tile_distances(small_ds, dist64):
    locs, z = small_case()
    perm = small_ds.perm()
    x = locs[perm]
    tile = SMALL.tile
    got = small_ds.covariance(SMALL.theta, tile, -1, dist64=dist64)
    want = oracle.matern_matrix(x, SMALL.theta)
    d = _tile_box_distances(x, tile)
    p = d.shape[0]
    n64 = 0
    for i in range(p):
        for j in range(i + 1):
            g = got[i * tile:(i + 1) * tile, j * tile:(j + 1) * tile]
            w = want[i * tile:(i + 1) * tile, j * tile:(j + 1) * tile]
            if i == j:
                g, w = np.tril(g), np.tril(w)
            if i == j or d[i, j] <= dist64:
                n64 += 1
                np.testing.assert_allclose(g, w, rtol=1e-13, atol=0)
            else:
                np.testing.assert_array_equal(g, w.astype(np.float32).astype(np.float64))
    assert n64 >= p


@pytest.mark.parametrize("dist64,tol", [(0.05, 1e-5), (0.2, 1e-5), (10.0, 1e-10)])
def test_distance_map_matches_oracle(small_ds, dist64, tol):
    want = small_oracle(SMALL.theta)
    got = small_ds.loglik(SMALL.theta, SMALL.tile, -1, dist64=dist64)
    assert abs(got["loglik"] - want["loglik"]) / max(abs(want["loglik"]), SMALL.n) <= tol
    if dist64 >= 10.0:   # every tile FP64: the all-FP64 path
        full = small_ds.loglik(SMALL.theta, SMALL.tile, -1)
        assert rel(got["loglik"], full["loglik"]) <= 1e-12


@pytest.mark.parametrize("lowp", ["fp16", "bf16"])
def test_distance_map_three_tiers(small_ds, lowp):
    want = small_oracle(SMALL.theta)
    got = small_ds.loglik(SMALL.theta, SMALL.tile, -1, lowp=lowp, dist64=0.05, dist32=0.2)
    err = rel(got["loglik"], want["loglik"])
    print(f"distance map, three tiers {lowp}: |dl|/|l| = {err:.3e}")
    assert err <= LOWP_BAR, err


def test_distance_map_plan_validation(lib, ctx, small_ds):
    bad = [dict(dist64=0.1, band0=2), dict(dist64=-1.0), dict(dist64=0.1, dist32=0.2),
           dict(dist64=0.2, dist32=0.1, lowp="fp16"), dict(dist32=0.1)]
    for kw in bad:
        res = lib.Result()
        plan = lib.make_plan(SMALL.tile, -1, 0, -1, kw.get("lowp"), kw.get("band0", -1),
                             kw.get("dist64", 0.0), kw.get("dist32", 0.0))
        st = lib.LIB.mpgeo_dataset_loglik(small_ds.handle, lib.Theta(*SMALL.theta), plan,
                                          ctypes.byref(res))
        assert st == lib.MPGEO_E_ARG, kw
    # the map needs sites: not available for a caller's matrix
    from synthetic import random_spd
    a = np.asfortranarray(random_spd(64, 1))
    res = lib.Result()
    st = lib.LIB.mpgeo_factor_dense(ctx.handle, 64, a.ctypes.data, 64, None,
                                    lib.make_plan(32, -1, 0, -1, None, -1, 0.1, 0.0),
                                    ctypes.byref(res))
    assert st == lib.MPGEO_E_ARG
