"""MPGEO_GRAPH: the factorization replayed as a captured HIP graph.  Every replay must equal the
plain launch sequence bit for bit (the graph holds the same kernels with the same arguments and
dependencies), with the program's own eager evaluations and synchronisations between replays,
across theta, plans (a new plan captures again), the profile likelihood, the blocked diagonal
factorization of 256/512 tiles and the 16-bit pass."""
import numpy as np
import pytest

import oracle
from synthetic import jittered_grid, normals

pytestmark = pytest.mark.gpu

# The first GPU run of these tests ended the process with a segmentation fault inside the first
# captured evaluation; its cause was not found, so the capture path is switched off (MPGEO_GRAPH
# returns MPGEO_E_UNSUPPORTED) and the tests of the replay stay skipped.
OFF = pytest.mark.skip(reason="graph capture of the factorization is switched off: its first GPU run "
                              "ended in a host segmentation fault whose cause was not found")

THETA0 = (1.0, 0.1, 0.5)


def _same(a, b):
    return a["loglik"] == b["loglik"] and a["logdet"] == b["logdet"] and a["quad"] == b["quad"]


@pytest.fixture(scope="module")
def small(lib):
    locs = jittered_grid(40, 101)
    z = oracle.simulate_field(locs, THETA0, normals(1600, 102))
    ctx = lib.Context(0)
    ds = lib.Dataset(ctx, locs, z)
    yield locs, z, ds
    ds.close()
    ctx.close()


@OFF
def test_graph_replays_equal_the_plain_path(small):
    locs, z, ds = small
    thetas = [THETA0] + [tuple(t * f for t, f in zip(THETA0, fs))
                         for fs in ((1.1, 0.9, 1.1), (0.9, 1.1, 0.9), (1.1, 1.1, 1.1), (0.9, 0.9, 0.9))]
    for rep in range(2):
        for th in thetas:
            g = ds.loglik(th, 160, 2, graph=True)
            plain = ds.loglik(th, 160, 2)          # eager work between the replays
            assert _same(g, plain), (rep, th, g, plain)
            g2 = ds.loglik(th, 160, 2, graph=True)
            assert _same(g2, plain)
    want = oracle.loglik(locs, z, THETA0)["loglik"]
    got = ds.loglik(THETA0, 160, 2, graph=True)["loglik"]
    assert abs(got - want) / abs(want) <= 1e-5


@OFF
def test_graph_recaptures_for_each_plan(small):
    locs, z, ds = small
    plans = [dict(tile=160, band64=2), dict(tile=160, band64=-1), dict(tile=64, band64=1, band32=2, lowp="fp16"),
             dict(tile=160, band64=2, profile=True), dict(tile=64, band64=0), dict(tile=160, band64=2)]
    for pl in plans + plans[::-1]:
        kw = dict(pl)
        tile, band = kw.pop("tile"), kw.pop("band64")
        g = ds.loglik(THETA0, tile, band, graph=True, **kw)
        plain = ds.loglik(THETA0, tile, band, **kw)
        assert _same(g, plain), (pl, g, plain)
    # with per-kernel timing the flag is ignored (the events need the plain launches)
    t = ds.loglik(THETA0, 160, 2, graph=True, timing=True)
    assert _same(t, ds.loglik(THETA0, 160, 2))


@OFF
@pytest.mark.parametrize("tile,plan", [(512, dict(band64=2)), (256, dict(band64=2, band32=2, lowp="fp16")),
                                       (256, dict(band64=-1))])
def test_graph_on_production_kernels(lib, tile, plan):
    # n = 4,900: tiles of 512 and 256 factored blocked (one-workgroup 128-column blocks and
    # their products), the 128 x 128 products and, in the three-tier plan, the 256 x 256 16-bit pass
    locs = jittered_grid(70, 201)
    theta = (1.0, 0.05, 0.5)
    z = oracle.simulate_field(locs, theta, normals(4900, 202))
    ctx = lib.Context(0)
    try:
        ds = lib.Dataset(ctx, locs, z)
        for th in (theta, (1.2, 0.04, 0.6), theta):
            g = ds.loglik(th, tile, plan["band64"], graph=True, **{k: v for k, v in plan.items() if k != "band64"})
            plain = ds.loglik(th, tile, plan["band64"], **{k: v for k, v in plan.items() if k != "band64"})
            assert _same(g, plain), (tile, plan, th)
        ds.close()
        rest = {k: v for k, v in plan.items() if k != "band64"}
        one = ctx.loglik(locs, z, theta, tile, plan["band64"], graph=True, **rest)   # the one-shot call
        assert _same(one, ctx.loglik(locs, z, theta, tile, plan["band64"], **rest))
    finally:
        ctx.close()


@OFF
def test_graph_maximum_likelihood_is_the_same_search(lib):
    locs = jittered_grid(20, 301)
    z = oracle.simulate_field(locs, THETA0, normals(400, 302))
    ctx = lib.Context(0)
    try:
        ds = lib.Dataset(ctx, locs, z)
        a = ds.mle((1.5, 0.05, 0.6), 64, 1, xtol=1e-5)
        b = ds.mle((1.5, 0.05, 0.6), 64, 1, xtol=1e-5, graph=True)
        assert a == b
        ds.close()
    finally:
        ctx.close()


def test_graph_flag_is_rejected(lib, small):
    locs, z, ds = small
    with pytest.raises(lib.MpgeoError):
        ds.loglik(THETA0, 160, 2, graph=True)
    with pytest.raises(lib.MpgeoError):
        ds.mle((1.5, 0.05, 0.6), 160, 2, graph=True)
    assert ds.loglik(THETA0, 160, 2)["info"] == -1   # the dataset is unharmed
