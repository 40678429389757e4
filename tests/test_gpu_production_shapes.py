"""Parity with the oracle at the tile shapes the benchmark runs: tiles of 512 and 256.

n = 16,900 (130 x 130 jittered grid; 16,900 = 33 * 512 + 4 = 66 * 256 + 4, so the last tile row
is a ragged 4 rows), theta = (1, 0.1, 0.5), z a draw of the field by the oracle's own factor.
At these tile sizes every update runs in the kernels of the n ~ 1e5 workload: the 128 x 128 FP64
and FP32 tile products, the 256 x 256 direct-to-LDS 16-bit left-looking pass (tile rows that are
multiples of 256) and the 128 x 64 one-panel 16-bit column update.  The oracle evaluates eq. (2)
here on the host in about 12 s.

Bars, on the stated metric |dl| / |l| (|l| = 2,511 here, well away from zero):
  * all-FP64 path:               1e-10 (also logdet and quad);
  * two tiers, FP64 band 2:      1e-5;
  * three tiers, band 2, FP32 width 8, FP16 operands beyond: 1e-5;
  * BF16 operands: 1e-5 where the FP32 width makes it (tile 512, width 16); the plans that miss
    it (tile 512 width 8, tile 256 width 16) are reported rows, printed with their error;
  * kriging at 200 held-out sites: FP64 1e-9 (of max |pred|, and of theta1 for variances),
    two tiers 1e-4, three tiers 1e-3 (a 16-bit operand carries 2^-11 relative error; the
    weights Sigma^-1 Z amplify it by the conditioning of Sigma).
"""
import functools

import numpy as np
import pytest

import oracle
from synthetic import jittered_grid, normals, uniform_sites

pytestmark = pytest.mark.gpu

M = 130
THETA = (1.0, 0.1, 0.5)


@functools.lru_cache(maxsize=None)
def workload():
    locs = jittered_grid(M, 131)
    z = oracle.simulate_field(locs, THETA, normals(M * M, 132))
    ref = oracle.loglik(locs, z, THETA)
    return locs, z, {k: ref[k] for k in ("loglik", "logdet", "quad")}


@functools.lru_cache(maxsize=None)
def kriging_ref():
    locs, z, _ = workload()
    new = uniform_sites(200, 133)
    return new, oracle.krige(locs, z, THETA, new)


@pytest.fixture(scope="module")
def ds(lib):
    locs, z, _ = workload()
    ctx = lib.Context(0)
    d = lib.Dataset(ctx, locs, z)
    yield d
    d.close()
    ctx.close()


def rel(got, want):
    return abs(got - want) / abs(want)


@pytest.mark.parametrize("tile", [512, 256])
def test_fp64_path(ds, tile):
    _, _, ref = workload()
    got = ds.loglik(THETA, tile, -1)
    assert rel(got["loglik"], ref["loglik"]) <= 1e-10
    assert rel(got["logdet"], ref["logdet"]) <= 1e-10
    assert rel(got["quad"], ref["quad"]) <= 1e-10


@pytest.mark.parametrize("tile", [512, 256])
@pytest.mark.parametrize("band", [2, 0])
def test_two_tier_path(ds, tile, band):
    _, _, ref = workload()
    got = ds.loglik(THETA, tile, band)
    err = rel(got["loglik"], ref["loglik"])
    print(f"tile {tile} band {band}: |dl|/|l| = {err:.3e}")
    assert err <= 1e-5


CASES = [  # (tile, band32, format, asserted at 1e-5)
    (512, 8, "fp16", True), (256, 8, "fp16", True),
    (512, 16, "bf16", True), (512, 8, "bf16", False), (256, 16, "bf16", False),
]


@pytest.mark.parametrize("tile,band32,lowp,asserted", CASES)
def test_three_tier_path(ds, tile, band32, lowp, asserted):
    _, _, ref = workload()
    got = ds.loglik(THETA, tile, 2, band32=band32, lowp=lowp)
    err = rel(got["loglik"], ref["loglik"])
    print(f"tile {tile} band64 2 band32 {band32} {lowp}: |dl|/|l| = {err:.3e}"
          f"{'' if asserted else ' (reported; misses the 1e-5 bar)'}")
    assert np.isfinite(got["loglik"])
    assert rel(got["logdet"], ref["logdet"]) <= 1e-5
    if asserted:
        assert err <= 1e-5
    else:
        assert err <= 20 * 2.0 ** -8      # the derived worst case of a BF16 operand tier


@pytest.mark.parametrize("tile,plan,tol", [
    (512, dict(band64=-1), 1e-9), (512, dict(band64=2), 1e-4),
    (512, dict(band64=2, band32=8, lowp="fp16"), 1e-3),
    (256, dict(band64=2, band32=8, lowp="fp16"), 1e-3)])
def test_kriging_from_the_factor(ds, tile, plan, tol):
    new, want = kriging_ref()
    kw = dict(plan)
    b64 = kw.pop("band64")
    ds.loglik(THETA, tile, b64, **kw)
    pred, var = ds.krige(new, variance=True)
    dp = np.max(np.abs(pred - want["pred"])) / np.max(np.abs(want["pred"]))
    dv = np.max(np.abs(var - want["var"])) / THETA[0]
    pmse_gap = abs(np.mean((pred - want["pred"]) ** 2))
    print(f"tile {tile} {plan}: max|dpred|/max|pred| = {dp:.2e}, max|dvar| = {dv:.2e}, "
          f"mean dpred^2 = {pmse_gap:.2e}")
    assert dp <= tol and dv <= tol
