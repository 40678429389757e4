"""Host logic: the factorization schedule of the tile layout (no GPU work).

The C++ check in schedule_check.hip includes the library's layout code, builds the schedules of
several plans and verifies them (panel order and completeness of the 16-bit tier's left-looking
passes, wave filling, the split of each step's FP64/FP32 update lists); it is compiled with
hipcc and linked against the in-tree library.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.join(os.path.dirname(HERE), "paper_2003_05324_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_schedule_is_consistent():
    lib = os.path.join(PKG, "libmpgeo.so")
    if not os.path.exists(lib):
        pytest.skip("libmpgeo.so is not built")
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc is not available")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "schedule_check")
        cmd = [HIPCC, "-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", os.path.join(HERE, "schedule_check.hip"), "-o", exe,
               "-L", PKG, "-lmpgeo", f"-Wl,-rpath,{PKG}"]
        build = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert build.returncode == 0, build.stderr[-2000:]
        run = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(run.stdout)
        assert run.returncode == 0, run.stdout[-2000:]


def test_blocked_diagonal_factorization_plan():
    # the plan of the blocked 256/512-column diagonal-tile factorization (potrf_plan.h): bounds of
    # every product and of the device kernel's indices, job counts per launch, independence of
    # the products of a launch, and the plan replayed in FP64 against a plain Cholesky factor
    # and inverse (tests/potrf_plan_check.cpp, host code only)
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ is not available")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "potrf_plan_check")
        build = subprocess.run([gxx, "-O2", "-std=c++17", os.path.join(HERE, "potrf_plan_check.cpp"), "-o", exe],
                               capture_output=True, text=True, timeout=300)
        assert build.returncode == 0, build.stderr[-2000:]
        run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        print(run.stdout)
        assert run.returncode == 0, run.stdout[-2000:]


def test_band_tuner_policy():
    # the FP64-band tuner's policy (tune_policy.h): the terms scale of eq. (2), the class key, the
    # candidate bands, the choice from the probes' results and the all-FP64 re-evaluation of a
    # problem whose l cancels (tests/tune_policy_check.cpp, host code only)
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ is not available")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "tune_policy_check")
        build = subprocess.run([gxx, "-O2", "-std=c++17", "-Wall", os.path.join(HERE, "tune_policy_check.cpp"),
                                "-o", exe], capture_output=True, text=True, timeout=300)
        assert build.returncode == 0, build.stderr[-2000:]
        run = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(run.stdout)
        assert run.returncode == 0, run.stdout[-2000:]
