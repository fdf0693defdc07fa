"""The FP64 tiles' table-driven exponential (Tang's method, in kmap64.h) on the
host against long-double exp: compiled from the same header with hipcc and run
on the CPU."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not found")


def test_scaled_exp_and_kernel_maps_within_a_few_ulps(tmp_path):
    exe = tmp_path / "exp64_check"
    cmd = [_hipcc(), "-O2", "-std=c++17", "--offload-arch=gfx950", "-x", "hip",
           os.path.join(ROOT, "tests", "exp64_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    print(out)
    vals = {line.split()[0]: float(line.split()[1]) for line in out.splitlines()}
    assert vals["exp_ulps"] <= 3.0
    assert vals["rbf_ulps"] <= 4.0
    # Matern: error over (4 + 3 t) ulps, t the rounded argument of exp
    assert vals["m32_per_bound"] <= 1.0
    assert vals["m52_per_bound"] <= 1.0
