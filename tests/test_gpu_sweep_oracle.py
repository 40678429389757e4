"""The n = 40,000 band-sweep fields (200 x 200 jittered grids, tile 512, p = 79 with a ragged
last tile of 64 rows) against the oracle's eq. (2) at the true theta, stored in
tests/golden/sweep_n40000.json by tests/golden/make_golden.py (oracle only).

The stored values use the oracle's draw z = L eps; the library draws z with its own FP64 factor
from the same eps, equal to rounding.  The log-determinant does not depend on z: it is held to
the FP64 bar 1e-10.  For both draws y = L^-1 z is eps up to rounding, so the quadratic forms
agree with eps^T eps (and each other) to the solve's rounding, amplified by the conditioning of
L (up to about 1e-9 relative for the smoothest field); l is held to 1e-9.
"""
import json
import os

import numpy as np
import pytest

from synthetic import SWEEP

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sweep_n40000.json")


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("field", range(len(SWEEP)))
def test_fp64_path_against_stored_oracle(lib, ctx, field):
    import torch
    gold = {f["field"]: f for f in json.load(open(GOLD))["fields"]}
    w = SWEEP[field]
    want = gold[w.name]
    assert want["loc_seed"] == w.loc_seed and want["z_seed"] == w.z_seed and want["n"] == w.n
    dev = torch.device("cuda:0")
    locs = torch.from_numpy(w.locations()).to(dev)
    eps = w.eps()
    gen = lib.Dataset(ctx, locs, None)
    z = gen.simulate(w.theta, torch.from_numpy(eps).to(dev), w.tile, -1)
    gen.close()
    ds = lib.Dataset(ctx, locs, z)
    got = ds.loglik(w.theta, w.tile, -1)
    ds.close()
    ee = float(np.dot(eps, eps))
    dlogdet = abs(got["logdet"] - want["logdet"]) / abs(want["logdet"])
    dl = abs(got["loglik"] - want["loglik"]) / abs(want["loglik"])
    print(f"{w.name}: dlogdet {dlogdet:.2e}, dl {dl:.2e}, quad/eps'eps - 1: library "
          f"{got['quad'] / ee - 1:.2e}, oracle {want['quad'] / ee - 1:.2e}")
    assert dlogdet <= 1e-10
    assert abs(want["quad"] / ee - 1) <= 1e-9 and abs(got["quad"] / ee - 1) <= 1e-9
    assert dl <= 1e-9
