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


def test_three_tier_plan_through_the_lanes(ctx, problems):
    # the third tier through the batched lanes (tile 64, FP64 band 1, FP32 for 1 more tile,
    # FP16 operands beyond): identical to single calls, within the third tier's bar of the oracle
    st, res, tiles = ctx.batch_loglik(problems, tile=64, band64=1, band32=1, lowp="fp16")
    assert st == 0 and tiles == [64] * len(problems)
    for (locs, z, theta), r in zip(problems, res):
        one = ctx.loglik(locs, z, theta, 64, 1, band32=1, lowp="fp16")
        assert r["loglik"] == one["loglik"] and r["logdet"] == one["logdet"]
        want = oracle.loglik(locs, z, theta)["loglik"]
        assert abs(r["loglik"] - want) / max(abs(want), len(z)) <= 20 * 2.0 ** -11


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


# ---- one persistent kernel over a device task queue (MPGEO_BATCH_QUEUE) ----------------------
def test_queue_matches_oracle_and_lanes(lib, ctx, problems):
    st, res, tiles = ctx.batch_loglik(problems, tile=0, band64=-1, queue=True)
    assert st == 0 and tiles == [128] * len(problems)
    _, lanes, _ = ctx.batch_loglik(problems, tile=128, band64=-1)
    for (locs, z, theta), r, l in zip(problems, res, lanes):
        want = oracle.loglik(locs, z, theta)
        assert _rel(r["loglik"], want["loglik"]) <= 1e-10, (len(z), theta)
        assert _rel(r["logdet"], want["logdet"]) <= 1e-10
        assert _rel(r["quad"], want["quad"]) <= 1e-10
        assert r["info"] == -1
        # same tiles and operations, products summed in another order
        assert _rel(r["loglik"], l["loglik"]) <= 1e-11
    # deterministic: every task's arithmetic has a fixed order
    st2, res2, _ = ctx.batch_loglik(problems, tile=128, band64=-1, queue=True)
    assert st2 == 0 and [r["loglik"] for r in res2] == [r["loglik"] for r in res]


def test_queue_medium_problems_and_groups(lib, ctx):
    # n up to 6,000 (47 tile rows): long left-looking chains, many tasks per column
    probs = []
    for locs, eps, theta in batch_instances(12, 23, n_min=2000, n_max=6000):
        probs.append((locs, oracle.simulate_field(locs, theta, eps), theta))
    st, res, _ = ctx.batch_loglik(probs, tile=0, band64=-1, queue=True)
    assert st == 0
    _, lanes, _ = ctx.batch_loglik(probs, tile=128, band64=-1)
    for r, l in zip(res, lanes):
        assert _rel(r["loglik"], l["loglik"]) <= 1e-11
    q = int(np.argmin([len(z) for _, z, _ in probs]))
    assert _rel(res[q]["loglik"], oracle.loglik(*probs[q])["loglik"]) <= 1e-10


def test_queue_profile_and_great_circle(lib, ctx):
    from synthetic import lonlat_grid
    locs = jittered_grid(30, 5)
    theta = (1.0, 0.1, 1.5)
    z = oracle.simulate_field(locs, theta, normals(len(locs), 6))
    st, res, _ = ctx.batch_loglik([(locs, z, (7.0, 0.1, 1.5))], tile=0, profile=True, queue=True)
    want = oracle.profile_loglik(locs, z, theta[1], theta[2])
    assert st == 0 and _rel(res[0]["loglik"], want["loglik"]) <= 1e-10
    ll = lonlat_grid(25, 8)
    th = (1.0, 300.0, 0.5)
    zz = oracle.simulate_field(ll, th, normals(len(ll), 9), metric="gcd")
    st, res, _ = ctx.batch_loglik([(ll, zz, th)], tile=0, gcd=True, queue=True)
    assert st == 0 and _rel(res[0]["loglik"], oracle.loglik(ll, zz, th, metric="gcd")["loglik"]) <= 1e-10


def _storage_perturbation(locs, z, theta, tile, band):
    """|l(Sigma') - l(Sigma)| / |l| with Sigma' = Sigma whose tiles farther than `band` from the
    diagonal (in the Z-order the library factors in) are rounded to FP32: the part of a two-tier
    plan's error that no FP32 arithmetic can avoid, computed exactly by the oracle."""
    perm = oracle.morton_order(locs)
    sigma = oracle.matern_matrix(locs[perm], theta)
    blk = np.arange(len(z)) // tile
    far = np.abs(blk[:, None] - blk[None, :]) > band
    rounded = np.where(far, sigma.astype(np.float32).astype(np.float64), sigma)
    base = oracle.loglik_parts(sigma, z[perm])["loglik"]
    return abs(oracle.loglik_parts(rounded, z[perm])["loglik"] - base) / abs(base)


@pytest.mark.parametrize("band", [0, 1, 3])
def test_queue_two_tier_plans(lib, ctx, problems, band):
    # FP64 within `band` tiles of 128, FP32 beyond, in the persistent queue.  Bar per problem:
    # the band path's 1e-5 of |l|, or ten times the plan's own FP32 storage perturbation where
    # that is larger (the smoothest fields here, nu = 1.5 with beta ~ 0.15 on a few hundred
    # sites, lose a few 1e-6 to the rounding of Sigma alone at bands 0 and 1, and the FP32
    # factorization rounds each far tile once per panel on top of it; such a plan misses the
    # stated bar, which is what the band tuner below is for).  Also: close to the same plan
    # through the lanes (FP32 products summed in another order), deterministic, reported with
    # its band.
    st, res, _ = ctx.batch_loglik(problems, tile=128, band64=band, queue=True)
    assert st == 0
    _, lanes, _ = ctx.batch_loglik(problems, tile=128, band64=band)
    worst = 0.0
    for (locs, z, theta), r, l in zip(problems, res, lanes):
        want = oracle.loglik(locs, z, theta)["loglik"]
        bar = max(1e-5, 10 * _storage_perturbation(locs, z, theta, 128, band))
        err = abs(r["loglik"] - want) / abs(want)
        errl = abs(l["loglik"] - want) / abs(want)
        worst = max(worst, err)
        print(f"n {len(z)} theta {theta}: queue {err:.2e}, lanes {errl:.2e}, bar {bar:.1e}")
        assert err <= bar, (len(z), theta, err, bar)
        assert errl <= bar, (len(z), theta, errl, bar)
        p = -(-len(z) // 128)
        assert r["band64"] == (band if band < p - 1 else -1)
    print(f"queue band {band}: max |dl|/|l| vs oracle = {worst:.2e}")
    st2, res2, _ = ctx.batch_loglik(problems, tile=128, band64=band, queue=True)
    assert [r["loglik"] for r in res2] == [r["loglik"] for r in res]


def _tune_class(n, theta):
    # the tuner's class: half-octave of n, smoothness to a quarter, half-octave of the range
    return (int(np.floor(2 * np.log2(n))), int(round(4 * theta[2])), int(round(2 * np.log2(theta[1]))))


def _terms(n, logdet, quad):
    # half the summed sizes of eq. (2)'s terms: the scale the tuner measures its error on
    return 0.5 * (n * np.log(2 * np.pi) + abs(logdet) + abs(quad))


def _check_tuned(lib, problems, res, fp64):
    # one band per class among the problems left at their tuned band; the others all-FP64,
    # either re-evaluated for accuracy (one escalation, the all-FP64 result bit for bit) or with
    # a band that covers their matrix; every result within the band path's 1e-5 of the oracle
    classes = {}
    for (locs, z, theta), r, f in zip(problems, res, fp64):
        want = oracle.loglik(locs, z, theta)["loglik"]
        assert abs(r["loglik"] - want) / abs(want) <= 1e-5
        if r["escalations"] > 0:
            assert r["band64"] == -1 and r["loglik"] == f["loglik"]
        elif r["band64"] >= 0:
            classes.setdefault(_tune_class(len(z), theta), set()).add(r["band64"])
    assert all(len(b) == 1 for b in classes.values())
    return classes


def test_band_tuner(lib, problems):
    # MPGEO_TUNE_BAND: one band per class (narrowest within 1e-7 of all-FP64, relative to the
    # size of eq. (2)'s terms, on the class's first two problems), deterministic across contexts
    c1, c2 = lib.Context(0), lib.Context(0)
    try:
        st, res, _ = c1.batch_loglik(problems, tile=128, queue=True, tune_band=True)
        assert st == 0
        st2, res2, _ = c2.batch_loglik(problems, tile=128, queue=True, tune_band=True)
        assert [r["band64"] for r in res2] == [r["band64"] for r in res]
        assert [r["loglik"] for r in res2] == [r["loglik"] for r in res]
        _, fp64, _ = c1.batch_loglik(problems, tile=128, band64=-1, queue=True)
        classes = _check_tuned(lib, problems, res, fp64)
        print("tuned bands per class:", {k: sorted(v) for k, v in classes.items()},
              "re-evaluated:", sum(r["escalations"] for r in res))
        # the lanes probe their classes themselves (their products are summed in another order,
        # so a band at the edge of the bar may come out differently)
        st, lanes, tiles = c1.batch_loglik(problems, tile=128, tune_band=True)
        assert st == 0 and tiles == [128] * len(problems)
        _, fp64l, _ = c1.batch_loglik(problems, tile=128, band64=-1)
        _check_tuned(lib, problems, lanes, fp64l)
    finally:
        c1.close()
        c2.close()


@pytest.mark.parametrize("queue", [True, False])
def test_band_tuner_reevaluates_cancelling_loglik(lib, queue):
    # l passes through zero where its terms cancel, and a mixed band's rounding error, a small
    # fraction of those terms, is then no longer small against l: such a problem is evaluated
    # again all-FP64.  Two probes of one class (same sites, smoothness and range) fix a mixed
    # band; the third problem is the first scaled so that l = 0 (z -> c z, sigma2 -> c^2 sigma2
    # shifts l by -n log c, with c = exp(l / n)), which leaves its class and its relative
    # rounding unchanged
    locs = jittered_grid(40, 21)
    theta = (1.0, 0.02, 0.5)
    z = oracle.simulate_field(locs, theta, normals(1600, 22))
    l0 = oracle.loglik(locs, z, theta)["loglik"]
    c = np.exp(l0 / len(z))
    zero = (locs, c * z, (c * c, theta[1], theta[2]))
    probs = [(locs, z, theta), (locs, 1.5 * z, (2.25, theta[1], theta[2])), zero]
    want = oracle.loglik(*zero)
    terms = _terms(len(z), want["logdet"], want["quad"])
    assert abs(want["loglik"]) < 1e-9 * terms
    ctx = lib.Context(0)
    try:
        st, res, _ = ctx.batch_loglik(probs, tile=128, queue=queue, tune_band=True)
        assert st == 0
        print("bands", [r["band64"] for r in res], "escalations", [r["escalations"] for r in res])
        assert res[0]["band64"] >= 0 and res[1]["band64"] == res[0]["band64"]
        assert res[0]["escalations"] == res[1]["escalations"] == 0
        assert res[2]["band64"] == -1 and res[2]["escalations"] == 1
        _, fp64, _ = ctx.batch_loglik([zero], tile=128, band64=-1, queue=queue)
        assert res[2]["loglik"] == fp64[0]["loglik"]
        assert abs(res[2]["loglik"] - want["loglik"]) <= 1e-10 * terms
        # the same problem at the class's band, without the tuner: its error against l
        _, mixed, _ = ctx.batch_loglik([zero], tile=128, band64=res[0]["band64"], queue=queue)
        print(f"at band {res[0]['band64']}: |dl| = {abs(mixed[0]['loglik'] - want['loglik']):.2e}, "
              f"terms {terms:.3e}, l {want['loglik']:.2e}")
    finally:
        ctx.close()


def test_queue_escalation(lib, ctx):
    # a problem positive definite in FP64 but not with FP32 tiles (nu = 5/2, beta = 0.3 on 900
    # sites: condition number 3e10) beside an easy one: with MPGEO_ESCALATE the failed problem
    # runs again at the widened FP64 band until it factors, the easy one is untouched; the
    # escalated result equals the queue at the final band, bit for bit, and the oracle
    hard_locs = jittered_grid(30, 3)
    hard_theta = (1.0, 0.3, 2.5)
    hard = (hard_locs, oracle.simulate_field(hard_locs, hard_theta, normals(900, 4)), hard_theta)
    easy_locs = jittered_grid(20, 5)
    easy = (easy_locs, oracle.simulate_field(easy_locs, (1.0, 0.05, 0.5), normals(400, 6)), (1.0, 0.05, 0.5))
    st, res, _ = ctx.batch_loglik([hard, easy], tile=128, band64=0, queue=True)
    assert st == lib.MPGEO_E_NOT_SPD and res[0]["info"] >= 0 and res[1]["info"] == -1
    st, res, _ = ctx.batch_loglik([hard, easy], tile=128, band64=0, queue=True, escalate=True)
    assert st == lib.MPGEO_OK
    assert res[0]["escalations"] >= 1 and res[1]["escalations"] == 0 and res[1]["band64"] == 0
    ladder = [0, 1, 3, -1]                                  # b -> 2b + 1, p = 8 tile rows
    assert res[0]["band64"] == ladder[res[0]["escalations"]]
    st1, alone, _ = ctx.batch_loglik([hard], tile=128, band64=res[0]["band64"], queue=True)
    assert st1 == lib.MPGEO_OK and alone[0]["loglik"] == res[0]["loglik"]
    # against the oracle: two FP64 factorizations of a matrix of condition number 3e10 differ by
    # their roundings amplified by it (9e-10 measured for the all-FP64 plan), hence 1e-8 here
    want = oracle.loglik(*hard)["loglik"]
    bar = 1e-8 if res[0]["band64"] < 0 else 1e-5
    assert abs(res[0]["loglik"] - want) / abs(want) <= bar
    print(f"escalated to band {res[0]['band64']} after {res[0]['escalations']} widenings")
    # the lanes do not escalate
    with pytest.raises(lib.MpgeoError):
        ctx.batch_loglik([easy], tile=128, band64=0, escalate=True)


def test_queue_rejects_what_it_does_not_cover(lib, ctx, problems):
    assert ctx.batch_loglik([], tile=0, queue=True)[0] == 0
    for kw in (dict(band64=1, band32=1, lowp="fp16"), dict(tile=256), dict(band0=2)):
        args = dict(tile=0, band64=-1)
        args.update(kw)
        with pytest.raises(lib.MpgeoError):
            ctx.batch_loglik(problems[:2], queue=True, **args)
    big = jittered_grid(129, 2)                      # n = 16,641 > 16,384
    with pytest.raises(lib.MpgeoError):
        ctx.batch_loglik([(big, normals(len(big), 1), (1.0, 0.1, 0.5))], tile=0, queue=True)
