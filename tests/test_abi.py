"""The C-ABI library loads and exports every entry point include/mpgeo.h declares (no GPU needed)."""
import ctypes
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpgeo.h")
LIB = os.path.join(ROOT, "paper_2003_05324_amd", "libmpgeo.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpgeo_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmpgeo.so is not built (python paper_2003_05324_amd/build.py)")
    import torch  # noqa: F401  (same HIP runtime as the binding)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mpgeo_loglik", "mpgeo_dataset_loglik", "mpgeo_dataset_krige",
                 "mpgeo_factor_dense", "mpgeo_ctx_create", "mpgeo_dataset_mle"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_python_binding_names_match_header():
    import paper_2003_05324_amd as mp
    assert sorted(mp.EXPORTED) == declared_functions()


def test_host_only_entry_points(lib):
    import paper_2003_05324_amd as mp
    assert mp.status_string(mp.MPGEO_E_NOT_SPD) == "matrix is not positive definite"
    # footprint: FP64 band tiles + FP32 far tiles of the physical (padded) tiles
    p, nb = 196, 512
    band = 2
    n64 = sum(1 for i in range(p) for j in range(i + 1) if i - j <= band)
    n32 = p * (p + 1) // 2 - n64
    assert mp.mpgeo_footprint_bytes(99856, nb, band) == (n64 * 8 + n32 * 4) * nb * nb
    assert mp.mpgeo_footprint_bytes(99856, nb, -1) == p * (p + 1) // 2 * 8 * nb * nb
    # tile 160 is padded to 160 (a multiple of 32); tile 100 to 128
    assert mp.mpgeo_footprint_bytes(1000, 100, -1) == 55 * 8 * 128 * 128
    assert mp.mpgeo_footprint_bytes(10, 0, -1) == 0          # invalid plan


def test_argument_errors_need_no_gpu(lib):
    import paper_2003_05324_amd as mp
    res = mp.Result()
    # a NULL context is rejected before any device call
    st = mp.LIB.mpgeo_loglik(None, 10, None, None, mp.Theta(1, 0.1, 0.5), mp.make_plan(4, 0),
                             ctypes.byref(res))
    assert st == mp.MPGEO_E_ARG
    assert mp.LIB.mpgeo_ctx_destroy(None) == mp.MPGEO_OK
    assert mp.LIB.mpgeo_dataset_destroy(None) == mp.MPGEO_OK


def _tiers_by_enumeration(n, nb, band64, band32, band0):
    """Tile counts and per-tier update / TRSM / POTRF flops of Algorithm 1, tile by tile."""
    p = -(-n // nb)
    rows = [min(nb, n - i * nb) for i in range(p)]
    z = p if band0 < 0 or band0 > p else band0
    b = min(p if band64 < 0 or band64 > p else band64, z)
    e = min(p if band32 < 0 or b + band32 > p else b + band32, z)

    def tier(i, j):
        d = i - j
        return 3 if d > z else (0 if d <= b else (1 if d <= e else 2))

    tiles = [0, 0, 0, 0]
    for i in range(p):
        for j in range(i + 1):
            tiles[tier(i, j)] += 1
    upd = [0.0, 0.0, 0.0]
    trsm = [0.0, 0.0]
    for k in range(p):
        for i in range(k + 1, p):
            if i - k > z:
                continue
            trsm[0 if i - k <= b else 1] += rows[i] * rows[k] ** 2
            for j in range(k + 1, i + 1):
                t = tier(i, j)
                if t == 3:
                    continue
                f = rows[j] * (rows[j] + 1) if i == j else 2 * rows[i] * rows[j]
                upd[t] += f * rows[k]
    potrf = sum(r ** 3 / 3.0 for r in rows)
    return tiles, upd, trsm, potrf


@pytest.mark.parametrize("n,nb,b,c,z", [(99856, 512, 2, 8, -1), (99856, 512, 2, -1, -1),
                                         (5000, 300, 1, 3, -1), (5000, 300, 2, -1, 6),
                                         (5000, 300, 2, 2, 4), (777, 100, -1, -1, 2), (50, 7, 0, 1, 3)])
def test_plan_tiers_match_a_tile_by_tile_enumeration(n, nb, b, c, z):
    import paper_2003_05324_amd as mp
    lowp = "fp16" if c >= 0 else None
    got = mp.plan_tiers(n, nb, b, c, lowp, z)
    tiles, upd, trsm, potrf = _tiers_by_enumeration(n, nb, b, c, z)
    assert got["tiles"] == tiles
    np.testing.assert_allclose(got["update_flops"], upd, rtol=1e-12)
    np.testing.assert_allclose(got["trsm_flops"], trsm, rtol=1e-12)
    assert got["potrf_flops"] == pytest.approx(potrf, rel=1e-12)
    # storage: FP64 tiers at 8 bytes, FP32 and 16-bit-operand tiers at 4, one shared zero tile,
    # and with a 16-bit tier the 16-bit copy of the factor (one 2-byte slot per lower tile)
    nbp = -(-nb // 32) * 32
    p = -(-n // nb)
    q16 = p * (p + 1) // 2 * 2 if tiles[2] else 0
    want_bytes = (tiles[0] * 8 + (tiles[1] + tiles[2] + (1 if tiles[3] else 0)) * 4 + q16) * nbp * nbp
    assert got["footprint_bytes"] == want_bytes


def test_plan_tiers_headline_split():
    # the n = 99,856, tile 512 three-tier plan: about 3.8% / 11.4% / 84.0% of the Cholesky flops
    # in the FP64 / FP32 / 16-bit tiers (trailing updates), as the tier geometry predicts
    import paper_2003_05324_amd as mp
    t = mp.plan_tiers(99856, 512, 2, 8, "fp16")
    total = sum(t["update_flops"]) + sum(t["trsm_flops"]) + t["potrf_flops"]
    assert total == pytest.approx(99856 ** 3 / 3, rel=2e-3)
    shares = [f / total for f in t["update_flops"]]
    assert shares[0] == pytest.approx(0.0378, abs=5e-4)
    assert shares[2] == pytest.approx(0.840, abs=2e-3)
