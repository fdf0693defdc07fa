"""Device helpers compiled with hipcc for the host and run on the CPU: the FP64
tiles' table-driven exponential (Tang's method, in kmap64.h) against
long-double exp, and the random block rule (ap_internal.h) against the
oracle's implementation."""
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


def test_library_random_rule_matches_oracle(tmp_path):
    """The library's random block rule (device code, compiled here for the
    host) against the oracle's separate SplitMix64 implementation."""
    import ctypes

    import numpy as np
    from oracle import apo

    exe = tmp_path / "random_check"
    cmd = [_hipcc(), "-O2", "-std=c++17", "--offload-arch=gfx950", "-x", "hip",
           "-I", os.path.join(ROOT, "paper_2310_17137_amd", "csrc"),
           os.path.join(ROOT, "tests", "random_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    rows = [tuple(int(v) for v in line.split()) for line in out.splitlines()]
    assert len(rows) == 4 * 6 * 5
    ell = np.ones(1)
    lib = apo._load()
    for seed, u, m, blk in rows:
        # a bare config of m one-point blocks (the rule reads only n, b, seed)
        c = apo._Cfg(m, 1, 1, 1, apo.RBF, ell.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     1.0, 0.1, apo.RANDOM, 1e-2, 0, 1, seed)
        assert 0 <= blk < m
        assert lib.apo_select_random(ctypes.byref(c), u) == blk, (seed, u, m)
