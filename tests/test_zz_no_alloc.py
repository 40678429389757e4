"""The allocation-free batched entry point, mpgeo_batch_loglik_noalloc, against the allocating
persistent-queue batch it is a variant of (mpgeo_batch_loglik with MPGEO_BATCH_QUEUE): the same
kernels over the same tiles, so the same bits, on two calls in a row, the second with smaller
problems (the fixed device array keeps the first call's contents, so anything not cleared
would show), plus the oracle on the smallest problems and the size limit of the array."""
import numpy as np
import pytest

import oracle
from synthetic import batch_instances, jittered_grid, normals

pytestmark = pytest.mark.gpu


def _problems(count, seed, n_min, n_max, nu=None):
    out = []
    for locs, eps, theta in batch_instances(count, seed, n_min=n_min, n_max=n_max):
        if nu is not None:
            theta = (theta[0], theta[1], nu)
        out.append((locs, oracle.simulate_field(locs, theta, eps), theta))
    return out


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def test_noalloc_matches_the_queue_twice(lib, ctx):
    # nu = 1/2 for the large ones: the smoothest fields of the batch distribution are not
    # positive definite in FP32 beyond a band of 2 at these sizes
    large = _problems(6, 61, 3000, 6000, nu=0.5)   # several groups in the fixed array
    small = _problems(9, 62, 20, 900)        # then smaller problems into the same array
    for probs, band in ((large, 2), (large, -1), (small, -1), (small, 1)):
        st_q, want, _ = ctx.batch_loglik(probs, tile=128, band64=band, queue=True)
        st_n, got = ctx.batch_loglik_noalloc(probs, band64=band)
        assert st_q == st_n == lib.MPGEO_OK
        for (locs, z, theta), w, g in zip(probs, want, got):
            assert g["loglik"] == w["loglik"], (len(z), theta, band)
            assert g["logdet"] == w["logdet"] and g["quad"] == w["quad"]
            assert g["info"] == -1 and g["band64"] == w["band64"]
        print(f"band {band}: {len(probs)} problems, n {min(len(p[1]) for p in probs)}.."
              f"{max(len(p[1]) for p in probs)}: bit-identical to the allocating queue")
    # the oracle on the small all-FP64 problems
    _, got = ctx.batch_loglik_noalloc(small, band64=-1)
    for (locs, z, theta), g in zip(small, got):
        want = oracle.loglik(locs, z, theta)
        assert abs(g["loglik"] - want["loglik"]) / max(abs(want["loglik"]), 1.0) <= 1e-10


def test_noalloc_limits(lib, ctx):
    # a problem whose buffers exceed the array is refused before any work; the plans the
    # queue does not run and the band tuner are refused too; an empty batch is a no-op
    big = jittered_grid(95, 3)                        # n = 9,025 > 8,960 all-FP64
    with pytest.raises(lib.MpgeoError) as e:
        ctx.batch_loglik_noalloc([(big, normals(len(big), 4), (1.0, 0.1, 0.5))], band64=-1)
    assert e.value.status == lib.MPGEO_E_TOO_LARGE
    st, res = ctx.batch_loglik_noalloc([], band64=-1)
    assert st == lib.MPGEO_OK and res == []
    small = _problems(2, 63, 100, 300)
    with pytest.raises(lib.MpgeoError):
        ctx.batch_loglik_noalloc([(small[0][0], small[0][1], (1.0, -0.1, 0.5))], band64=-1)
    # after the refusals the array still serves a call
    st, got = ctx.batch_loglik_noalloc(small, band64=-1)
    assert st == lib.MPGEO_OK
    for (locs, z, theta), g in zip(small, got):
        want = oracle.loglik(locs, z, theta)["loglik"]
        assert abs(g["loglik"] - want) / max(abs(want), 1.0) <= 1e-10
