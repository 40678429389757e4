"""Batched evaluation of independent problems (many small and medium likelihoods in one call)
against the oracle and against one-at-a-time evaluation through the same C-ABI."""
import numpy as np
import pytest

import oracle
from synthetic import batch_instances, jittered_grid, normals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def problems():
    # data drawn from each problem's own field (white noise would put the quadratic form on
    # the smallest eigenvalues, where the FP32 tiers of the mixed plan are amplified)
    out = []
    for locs, eps, theta in batch_instances(14, 7, n_min=20, n_max=1500):
        out.append((locs, oracle.simulate_field(locs, theta, eps), theta))
    return out


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)


def test_fixed_tile_matches_oracle_and_single_calls(ctx, problems):
    st, res, tiles = ctx.batch_loglik(problems, tile=128, band64=-1)
    assert st == 0 and tiles == [128] * len(problems)
    for (locs, z, theta), r in zip(problems, res):
        want = oracle.loglik(locs, z, theta)
        assert _rel(r["loglik"], want["loglik"]) <= 1e-10, (len(z), theta)
        assert _rel(r["logdet"], want["logdet"]) <= 1e-10
        one = ctx.loglik(locs, z, theta, 128, -1)
        assert r["loglik"] == one["loglik"] and r["logdet"] == one["logdet"]   # same kernels


def test_autotuned_tiles_and_band_plan(ctx, problems):
    st, res, tiles = ctx.batch_loglik(problems, tile=0, band64=-1)
    assert st == 0
    # one tile per half-octave of n: a standard size, or the whole of some problem of that class
    classes = {}
    for (locs, z, theta), t in zip(problems, tiles):
        classes.setdefault(int(np.floor(2 * np.log2(len(z)))), []).append((len(z), t))
    for members in classes.values():
        assert len({t for _, t in members}) == 1
        t = members[0][1]
        assert t in (128, 256, 384, 512) or t in {min(n, 512) for n, _ in members}
    for (locs, z, theta), r in zip(problems, res):
        assert _rel(r["loglik"], oracle.loglik(locs, z, theta)["loglik"]) <= 1e-10
    # mixed precision: identical to single calls with the same tile, within the band bar of the oracle
    st, res, tiles = ctx.batch_loglik(problems, tile=0, band64=1)
    assert st == 0
    for (locs, z, theta), r, t in zip(problems, res, tiles):
        one = ctx.loglik(locs, z, theta, t, 1)
        assert r["loglik"] == one["loglik"]
        want = oracle.loglik(locs, z, theta)["loglik"]
        assert abs(r["loglik"] - want) / max(abs(want), len(z)) <= 1e-5


def test_failure_is_reported_per_instance(lib, ctx):
    # with tiles beyond band0 = 3 dropped, the n = 1,600 workload is not positive definite
    # (the oracle's truncated matrix fails too); one-tile instances are untouched by band0
    from synthetic import SMALL
    big_locs = SMALL.locations()
    big_z = oracle.simulate_field(big_locs, SMALL.theta, SMALL.eps())
    good = jittered_grid(10, 3)
    probs = [(good, normals(100, 1), (1.0, 0.1, 0.5)), (big_locs, big_z, SMALL.theta),
             (good, normals(100, 3), (1.2, 0.2, 1.5))]
    st, res, _ = ctx.batch_loglik(probs, tile=160, band64=-1, band0=3)
    assert st == lib.MPGEO_E_NOT_SPD
    assert res[0]["info"] == -1 and res[2]["info"] == -1 and res[1]["info"] >= 0
    for q in (0, 2):
        assert _rel(res[q]["loglik"], oracle.loglik(*probs[q])["loglik"]) <= 1e-10


def test_empty_and_invalid_batches(lib, ctx):
    assert ctx.batch_loglik([], tile=64)[0] == 0
    with pytest.raises(lib.MpgeoError):
        ctx.batch_loglik([(jittered_grid(4, 1), normals(16, 1), (1.0, -0.1, 0.5))], tile=64)
