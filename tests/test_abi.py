"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point include/ap.h declares, and sizes workspaces from the layout rules."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_2310_17137_amd import ap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ap.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ap_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(ap.SYMBOLS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = ap.load()
    for name in _declared():
        assert hasattr(lib, name), name
    raw = ctypes.CDLL(ap.LIB_PATH)
    for name in _declared():
        getattr(raw, name)


def test_library_shares_torchs_hip_runtime():
    ap.load()
    runtimes = ap._hip_runtimes()
    assert len(runtimes) == 1, runtimes
    assert ap.last_error() == ""  # nothing failed on this thread


def test_status_strings():
    assert ap.status_str(ap.OK) == "ok"
    assert "positive definite" in ap.status_str(ap.ERR_NOT_PD)
    assert ap.status_str(42) == "unknown status"


def _ws(**over):
    kw = dict(n=10000, d=3, l=8, b=512, kernel=ap.RBF, lengthscale=0.5)
    kw.update(over)
    return ap.workspace_bytes(**kw)


def test_workspace_holds_the_block_inverses():
    n, b = 10000, 512
    m = (n + b - 1) // b
    need = _ws(n=n, b=b)
    assert need >= m * b * b * 8
    # b rounded up to 64 for the FP64 tiles
    m2 = (n + 500 - 1) // 500
    assert _ws(n=n, b=500) >= m2 * 512 * 512 * 8
    assert _ws(n=2 * n, b=b) > need
    assert _ws(tile=ap.TILE_BF16) > 0


@pytest.mark.parametrize("over", [
    dict(n=0), dict(d=0), dict(l=0), dict(b=0), dict(b=20000), dict(kernel=7), dict(order=3),
    dict(tile=4), dict(tile=-1), dict(outputscale=0.0), dict(noise=-1.0), dict(lengthscale=0.0),
    dict(lengthscale=float("nan")), dict(tol=-1.0), dict(max_epochs=0), dict(min_epochs=-1),
    dict(refine_every=-2),
])
def test_invalid_configs_have_no_workspace(over):
    assert _ws(**over) == 0


@pytest.mark.parametrize("over", [dict(d=21), dict(l=33), dict(b=4097, n=100000)])
def test_sizes_beyond_this_build(over):
    assert _ws(**over) == 0
