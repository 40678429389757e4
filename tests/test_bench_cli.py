"""The benchmark's command line on a machine without a GPU: it refuses more than one GPU in
every mode before touching a device, and its help names the modes (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


@pytest.mark.parametrize("mode", [[], ["--batch", "4"], ["--serve", "2"], ["--sweep"], ["--small"]])
def test_more_than_one_gpu_is_refused_in_every_mode(mode):
    res = run_bench("--gpus", "2", *mode)
    assert res.returncode == 2
    assert "one GPU only" in res.stderr
    assert res.stdout == ""   # no JSON line


def test_help_lists_the_modes():
    res = run_bench("--help")
    assert res.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--batch", "--serve", "--sweep", "--lowp", "--small", "--legs"):
        assert flag in res.stdout
