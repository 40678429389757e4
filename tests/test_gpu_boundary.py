"""The C-ABI's argument checks, HBM budget and escalation on the GPU.

  * non-finite locations, data, kriging sites, normal draws and matrix entries are rejected
    with MPGEO_E_ARG, host inputs and device inputs alike, in every entry point that takes
    them; a NaN in the strict upper triangle of a matrix that mpgeo_factor_dense does not
    read is not an error;
  * a context's HBM budget: a plan whose tiles exceed it returns MPGEO_E_NOMEM before any
    work, a budget equal to the footprint gives the unbudgeted result bit for bit;
  * MPGEO_ESCALATE: a plan that loses positive definiteness in reduced precision (Section
    VIII-D-1) is repeated with wider bands; the result equals a direct call with the bands it
    reports, bit for bit, and every narrower plan on the ladder fails.
"""
import numpy as np
import pytest

import oracle
from synthetic import SMALL, jittered_grid, normals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def small(lib):
    locs = SMALL.locations()
    z = oracle.simulate_field(locs, SMALL.theta, SMALL.eps())
    return locs, z


def _status(lib, fn):
    with pytest.raises(lib.MpgeoError) as e:
        fn()
    return e.value.status


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_non_finite_host_inputs_are_rejected(lib, ctx, small, bad):
    locs, z = small
    l2 = locs.copy()
    l2[123, 1] = bad
    z2 = z.copy()
    z2[77] = bad
    assert _status(lib, lambda: ctx.loglik(l2, z, SMALL.theta, 160, 2)) == lib.MPGEO_E_ARG
    assert _status(lib, lambda: ctx.loglik(locs, z2, SMALL.theta, 160, 2)) == lib.MPGEO_E_ARG
    assert _status(lib, lambda: lib.Dataset(ctx, l2, z)) == lib.MPGEO_E_ARG
    assert _status(lib, lambda: lib.Dataset(ctx, locs, z2)) == lib.MPGEO_E_ARG
    ds = lib.Dataset(ctx, locs, z)
    try:
        ds.loglik(SMALL.theta, 160, 2)
        sites = np.array([[0.5, 0.5], [bad, 0.2]])
        assert _status(lib, lambda: ds.krige(sites)) == lib.MPGEO_E_ARG
        eps = normals(len(z), 5)
        eps[9] = bad
        assert _status(lib, lambda: ds.simulate(SMALL.theta, eps, 160, 2)) == lib.MPGEO_E_ARG
        # the dataset is still usable after rejected calls
        ok = ds.loglik(SMALL.theta, 160, 2)
        assert np.isfinite(ok["loglik"])
    finally:
        ds.close()
    # batched problems and the serving loop check their host copies
    st = _status(lib, lambda: ctx.batch_loglik([(locs[:300], z[:300], SMALL.theta), (l2, z, SMALL.theta)],
                                               tile=128))
    assert st == lib.MPGEO_E_ARG
    srv = lib.Server(ctx, 1 << 30, lanes=2)
    try:
        assert _status(lib, lambda: srv.add_dataset(locs, z2, 160, 2)) == lib.MPGEO_E_ARG
        d = srv.add_dataset(locs, z, 160, 2)
        sites = np.array([[0.5, bad]])
        assert _status(lib, lambda: srv.submit_krige(d, SMALL.theta, sites, 0.0)) == lib.MPGEO_E_ARG
    finally:
        srv.close()


def test_non_finite_device_inputs_are_rejected(lib, ctx, small):
    import torch
    locs, z = small
    dl = torch.from_numpy(locs).to("cuda:0")
    dz = torch.from_numpy(z).to("cuda:0")
    ref = ctx.loglik(dl, dz, SMALL.theta, 160, 2)
    bad_z = dz.clone()
    bad_z[1599] = float("nan")
    bad_l = dl.clone()
    bad_l[0, 0] = float("inf")
    assert _status(lib, lambda: ctx.loglik(dl, bad_z, SMALL.theta, 160, 2)) == lib.MPGEO_E_ARG
    assert _status(lib, lambda: ctx.loglik(bad_l, dz, SMALL.theta, 160, 2)) == lib.MPGEO_E_ARG
    assert _status(lib, lambda: lib.Dataset(ctx, bad_l, dz)) == lib.MPGEO_E_ARG
    ds = lib.Dataset(ctx, dl, dz)
    try:
        got = ds.loglik(SMALL.theta, 160, 2)
        assert got["loglik"] == ref["loglik"]
        sites = torch.tensor([[0.25, 0.75], [0.5, float("nan")]], dtype=torch.float64, device="cuda:0")
        assert _status(lib, lambda: ds.krige(sites)) == lib.MPGEO_E_ARG
    finally:
        ds.close()


def test_factor_dense_reads_only_the_lower_triangle(lib, ctx):
    import torch
    from synthetic import random_spd
    n = 200
    a = random_spd(n, 21)
    z = normals(n, 22)
    ref = ctx.factor_dense(a, z, 64, -1)
    upper = a.copy()
    upper[3, 150] = np.nan                       # strict upper triangle: never read
    assert ctx.factor_dense(upper, z, 64, -1)["loglik"] == ref["loglik"]
    lower = a.copy()
    lower[150, 3] = np.inf
    assert _status(lib, lambda: ctx.factor_dense(lower, z, 64, -1)) == lib.MPGEO_E_ARG
    z2 = z.copy()
    z2[0] = np.nan
    assert _status(lib, lambda: ctx.factor_dense(a, z2, 64, -1)) == lib.MPGEO_E_ARG
    # device matrices: the same checks by a reduction on the device; the library reads a
    # column-major matrix, which is the storage of the row-major transpose
    da = torch.from_numpy(np.ascontiguousarray(upper.T)).to("cuda:0")
    dz = torch.from_numpy(z).to("cuda:0")
    assert ctx.factor_dense(da, dz, 64, -1)["loglik"] == ref["loglik"]
    dl = torch.from_numpy(np.ascontiguousarray(lower.T)).to("cuda:0")
    assert _status(lib, lambda: ctx.factor_dense(dl, dz, 64, -1)) == lib.MPGEO_E_ARG


@pytest.mark.parametrize("plan", [dict(band64=-1), dict(band64=2), dict(band64=2, band32=2, lowp="fp16")])
def test_hbm_budget(lib, small, plan):
    locs, z = small
    b64 = plan["band64"]
    kw = {k: v for k, v in plan.items() if k != "band64"}
    need = lib.mpgeo_footprint_bytes(len(z), 160, b64, kw.get("band32", -1), kw.get("lowp"))
    assert need > 0
    free = lib.Context(0)
    tight = lib.Context(0, hbm_budget_bytes=need)
    short = lib.Context(0, hbm_budget_bytes=need - 1)
    try:
        want = free.loglik(locs, z, SMALL.theta, 160, b64, **kw)
        got = tight.loglik(locs, z, SMALL.theta, 160, b64, **kw)
        assert got["loglik"] == want["loglik"]
        assert _status(lib, lambda: short.loglik(locs, z, SMALL.theta, 160, b64, **kw)) == lib.MPGEO_E_NOMEM
        ds = lib.Dataset(short, locs, z)       # creation allocates no tiles
        try:
            assert _status(lib, lambda: ds.loglik(SMALL.theta, 160, b64, **kw)) == lib.MPGEO_E_NOMEM
            # a plan that fits the budget still runs on the same dataset
            assert lib.mpgeo_footprint_bytes(len(z), 160, 0) < need - 1
            assert np.isfinite(ds.loglik(SMALL.theta, 160, 0)["loglik"])
        finally:
            ds.close()
    finally:
        for c in (free, tight, short):
            c.close()


def test_hbm_budget_batch_queue(lib, small):
    locs, z = small
    probs = [(locs[:1000], z[:1000], SMALL.theta), (locs[:300], z[:300], SMALL.theta)]
    p = -(-1000 // 128)
    need = p * (p + 1) // 2 * 128 * 128 * 8     # FP64 tiles of the larger problem
    ok = lib.Context(0, hbm_budget_bytes=need)
    short = lib.Context(0, hbm_budget_bytes=need - 1)
    ref = lib.Context(0)
    try:
        st, res, _ = ok.batch_loglik(probs, tile=128, queue=True)
        st_ref, res_ref, _ = ref.batch_loglik(probs, tile=128, queue=True)
        assert st == st_ref == lib.MPGEO_OK
        assert [r["loglik"] for r in res] == [r["loglik"] for r in res_ref]
        assert _status(lib, lambda: short.batch_loglik(probs, tile=128, queue=True)) == lib.MPGEO_E_NOMEM
    finally:
        for c in (ok, short, ref):
            c.close()


# A strongly correlated smooth field (range 0.3, smoothness 2): Sigma is positive definite
# (condition number about 6e9, well inside FP64) but with its far tiles rounded to FP32 its
# smallest eigenvalue turns negative for bands 0 and 1 (-8.8e-8 and -2.8e-8, against 1.7e-7
# for Sigma), so those plans must fail.
HARD_THETA = (1.0, 0.3, 2.0)


def test_escalation_widens_the_band_until_the_factor_exists(lib, small):
    locs, z = small
    ctx = lib.Context(0)
    ds = lib.Dataset(ctx, locs, z)
    try:
        st, r0 = ds.try_loglik(HARD_THETA, 160, 0)
        assert st == lib.MPGEO_E_NOT_SPD and r0["info"] >= 0
        got = ds.loglik(HARD_THETA, 160, 0, escalate=True)
        assert got["escalations"] >= 1
        ladder = [0, 1, 3, 7, -1]
        assert got["band64"] == ladder[got["escalations"]]
        for b in ladder[:got["escalations"]]:            # every narrower plan fails
            st, _ = ds.try_loglik(HARD_THETA, 160, b)
            assert st == lib.MPGEO_E_NOT_SPD, b
        direct = ds.loglik(HARD_THETA, 160, got["band64"])
        assert direct["escalations"] == 0 and direct["band64"] == got["band64"]
        assert got["loglik"] == direct["loglik"] and got["logdet"] == direct["logdet"]
        want = oracle.loglik(locs, z, HARD_THETA)
        print(f"escalated to band64={got['band64']} after {got['escalations']} failures: "
              f"l = {got['loglik']:.6f}, oracle {want['loglik']:.6f}")
        # the same through the one-shot call and Algorithm 1 on the matrix itself
        one = ctx.loglik(locs, z, HARD_THETA, 160, 0, escalate=True)
        assert one["loglik"] == got["loglik"] and one["escalations"] == got["escalations"]
        perm = ds.perm()
        sigma = oracle.matern_matrix(locs[perm], HARD_THETA)
        dense = ctx.factor_dense(sigma, z[perm], 160, 0, escalate=True)
        assert dense["escalations"] >= 1 and dense["band64"] == ladder[dense["escalations"]]
        # a plan that needs no escalation reports its own bands
        easy = ds.loglik(SMALL.theta, 160, 2, escalate=True)
        assert easy["escalations"] == 0 and easy["band64"] == 2
    finally:
        ds.close()
        ctx.close()


def test_escalation_is_refused_where_it_is_not_supported(lib, ctx, small):
    locs, z = small
    plan = lib.make_plan(128, 0, lib.MPGEO_ESCALATE)
    inst = (lib.Instance * 1)()
    inst[0] = lib.Instance(300, locs.ctypes.data, z.ctypes.data, lib.Theta(*SMALL.theta))
    res = (lib.Result * 1)()
    assert lib.LIB.mpgeo_batch_loglik(ctx.handle, 1, inst, plan, res, None) == lib.MPGEO_E_UNSUPPORTED
