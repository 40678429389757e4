"""The C-ABI library loads and exports every entry point include/mpgeo.h declares (no GPU needed)."""
import ctypes
import os
import re

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
