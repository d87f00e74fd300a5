"""The benchmark's command-line contract, checked without a GPU: more than one GPU is
refused with a message, a host without a HIP device fails loudly, and the flags parse."""
import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_flags_parse():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--no-forms", "--no-cpu", "--no-trace", "--copy-calibration",
                 "--forms-only"):
        assert flag in r.stdout


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the host without a HIP device")
def test_no_device_fails_loudly():
    r = _run("--steps", "1", "--warmup", "0")
    assert r.returncode != 0
    assert "HIP device" in r.stderr
    assert r.stdout.strip() == ""
