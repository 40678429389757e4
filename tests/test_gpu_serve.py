"""Serving loop: every result equals the same evaluation done alone, whatever the mix, the
lane it ran on or an eviction and re-admission of its dataset in between."""
import numpy as np
import pytest

import oracle
from synthetic import jittered_grid, normals

pytestmark = pytest.mark.gpu


def test_served_results_equal_isolated_evaluations(lib):
    ctx = lib.Context(0)
    sizes = [300, 700, 1100, 1500]
    data = [(jittered_grid(int(np.ceil(np.sqrt(n))), 40 + q)[:n].copy(), normals(n, 50 + q))
            for q, n in enumerate(sizes)]
    foot = sorted(lib.mpgeo_footprint_bytes(n, 128, 1) for n in sizes)
    srv = lib.Server(ctx, hbm_budget_bytes=foot[-1] + foot[-2], lanes=3)   # two resident at most
    ids = [srv.add_dataset(locs, z, 128, 1) for locs, z in data]
    rng = np.random.default_rng(3)
    reqs = []
    for q in range(14):
        d = int(rng.integers(0, len(sizes)))
        theta = (float(np.exp(rng.normal(0, 0.2))), float(0.1 * np.exp(rng.normal(0, 0.2))), 0.5)
        t = srv.submit(ids[d], theta, 0.02 * q)
        reqs.append((t, d, theta))
    st, out = srv.run()
    assert st == 0
    for t, d, theta in reqs:
        r = out[t]
        assert r["info"] == -1
        assert r["arrival_s"] <= r["start_s"] + 1e-9 and r["start_s"] <= r["finish_s"]
        ds = lib.Dataset(ctx, *data[d])
        alone = ds.loglik(theta, 128, 1)
        ds.close()
        assert r["loglik"] == alone["loglik"] and r["logdet"] == alone["logdet"], (t, d)
        want = oracle.loglik(data[d][0], data[d][1], theta)["loglik"]
        assert abs(r["loglik"] - want) / max(abs(want), sizes[d]) <= 1e-5
    # a dataset larger than the whole budget is refused up front
    with pytest.raises(lib.MpgeoError) as e:
        big = jittered_grid(60, 9)
        srv.add_dataset(big, normals(len(big), 9), 128, -1)
    assert e.value.status == lib.MPGEO_E_NOMEM
    srv.close()
    ctx.close()


def test_kriging_requests_in_the_mix(lib):
    # likelihood and kriging requests of different sizes interleaved: every kriging request's
    # predictions and variances equal a dataset's own evaluation followed by kriging, bit for
    # bit, and match the oracle's simple kriging
    ctx = lib.Context(0)
    sizes = [400, 900, 1300]
    data = [(jittered_grid(int(np.ceil(np.sqrt(n))), 60 + q)[:n].copy(), normals(n, 70 + q))
            for q, n in enumerate(sizes)]
    srv = lib.Server(ctx, hbm_budget_bytes=1 << 34, lanes=2)
    ids = [srv.add_dataset(locs, z, 128, -1) for locs, z in data]
    new = [jittered_grid(7, 80 + q) * 0.9 + 0.05 for q in range(len(sizes))]   # 49 new sites
    rng = np.random.default_rng(5)
    reqs = []
    for q in range(9):
        d = q % len(sizes)
        theta = (float(np.exp(rng.normal(0, 0.2))), float(0.1 * np.exp(rng.normal(0, 0.2))), 0.5)
        if q % 2 == 0:
            t = srv.submit_krige(ids[d], theta, new[d], 0.01 * q, variance=(q % 4 == 0))
        else:
            t = srv.submit(ids[d], theta, 0.01 * q)
        reqs.append((t, d, theta, q % 2 == 0, q % 4 == 0))
    st, out = srv.run()
    assert st == 0
    for t, d, theta, kriging, variance in reqs:
        r = out[t]
        ds = lib.Dataset(ctx, *data[d])
        alone = ds.loglik(theta, 128, -1)
        assert r["loglik"] == alone["loglik"]
        if kriging:
            got = ds.krige(new[d], variance=variance)
            pred, var = got if variance else (got, None)
            assert np.array_equal(r["pred"], pred), t
            want = oracle.krige(data[d][0], data[d][1], theta, new[d])
            assert np.max(np.abs(r["pred"] - want["pred"])) <= 1e-9 * max(1.0, np.max(np.abs(want["pred"])))
            if variance:
                assert np.array_equal(r["var"], var), t
                assert np.max(np.abs(r["var"] - want["var"])) <= 1e-9 * theta[0]
        else:
            assert "pred" not in r
        ds.close()
    srv.close()
    ctx.close()


def test_three_tier_served_results_equal_isolated_evaluations(lib):
    # the serving lanes run the three-tier plan (FP64 band 1, FP32 for 2 more tiles, FP16
    # operands beyond) with two streams each; every result equals the dataset's own evaluation
    # bit for bit and the oracle within the third tier's bar
    ctx = lib.Context(0)
    sizes = [1500, 3100]
    data = [(jittered_grid(int(np.ceil(np.sqrt(n))), 90 + q)[:n].copy(), normals(n, 95 + q))
            for q, n in enumerate(sizes)]
    srv = lib.Server(ctx, hbm_budget_bytes=1 << 34, lanes=2)
    ids = [srv.add_dataset(locs, z, 128, 1, 2, "fp16") for locs, z in data]
    rng = np.random.default_rng(9)
    reqs = []
    for q in range(6):
        d = q % len(sizes)
        theta = (float(np.exp(rng.normal(0, 0.2))), float(0.1 * np.exp(rng.normal(0, 0.2))), 0.5)
        reqs.append((srv.submit(ids[d], theta, 0.01 * q), d, theta))
    st, out = srv.run()
    assert st == 0
    for t, d, theta in reqs:
        r = out[t]
        ds = lib.Dataset(ctx, *data[d])
        alone = ds.loglik(theta, 128, 1, band32=2, lowp="fp16")
        ds.close()
        assert r["loglik"] == alone["loglik"] and r["logdet"] == alone["logdet"], (t, d)
        want = oracle.loglik(data[d][0], data[d][1], theta)["loglik"]
        assert abs(r["loglik"] - want) / max(abs(want), sizes[d]) <= 20 * 2.0 ** -11
    srv.close()
    ctx.close()


def test_queued_requests_batch_in_one_launch_and_equal_alone(lib):
    # small datasets registered for the persistent queue: their ready likelihood requests are
    # batched into queue launches beside the lanes' evaluations of the other datasets.  Every
    # queued result equals the same problem queued alone (each problem's tasks have a fixed
    # order whatever else is in the launch), bit for bit, and the oracle within the band bar;
    # kriging requests on a queued dataset run on a lane (the factor stays resident there)
    ctx = lib.Context(0)
    sizes = [250, 600, 1000, 1400, 2600]
    data = []
    for q, n in enumerate(sizes):
        locs = jittered_grid(int(np.ceil(np.sqrt(n))), 110 + q)[:n].copy()
        data.append((locs, oracle.simulate_field(locs, (1.0, 0.1, 0.5), normals(n, 120 + q))))
    srv = lib.Server(ctx, hbm_budget_bytes=1 << 34, lanes=2)
    queued = [True, True, True, True, False]
    bands = [1, -1, 2, 1, 1]
    ids = [srv.add_dataset(locs, z, 128, b, queue=qd) for (locs, z), b, qd in zip(data, bands, queued)]
    new = jittered_grid(6, 130) * 0.9 + 0.05
    rng = np.random.default_rng(11)
    reqs = []
    for q in range(16):
        d = int(rng.integers(0, len(sizes)))
        theta = (float(np.exp(rng.normal(0, 0.15))), float(0.1 * np.exp(rng.normal(0, 0.15))), 0.5)
        if q in (5, 11):
            d = 1
            reqs.append((srv.submit_krige(ids[d], theta, new, 0.002 * (q // 4)), d, theta, True))
        else:
            reqs.append((srv.submit(ids[d], theta, 0.002 * (q // 4)), d, theta, False))  # bursts of 4
    st, out = srv.run()
    assert st == 0
    for t, d, theta, kriging in reqs:
        r = out[t]
        assert r["info"] == -1
        if queued[d] and not kriging:
            st1, alone, _ = ctx.batch_loglik([(data[d][0], data[d][1], theta)], tile=128, band64=bands[d],
                                             queue=True)
            assert st1 == 0
            assert r["loglik"] == alone[0]["loglik"] and r["logdet"] == alone[0]["logdet"], (t, d)
        else:
            ds = lib.Dataset(ctx, *data[d])
            alone = ds.loglik(theta, 128, bands[d])
            assert r["loglik"] == alone["loglik"], (t, d)
            if kriging:
                assert np.array_equal(r["pred"], ds.krige(new)), t
            ds.close()
        want = oracle.loglik(data[d][0], data[d][1], theta)["loglik"]
        assert abs(r["loglik"] - want) / abs(want) <= 1e-5
    # plans the queue does not run are refused for a queued dataset
    with pytest.raises(lib.MpgeoError):
        srv.add_dataset(data[0][0], data[0][1], 128, 1, 2, "fp16", queue=True)
    srv.close()
    ctx.close()
