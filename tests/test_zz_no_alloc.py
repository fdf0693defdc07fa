"""The allocation-free true residual (ap_residual_noalloc) against ap_residual
through the C ABI: same kernels, so R_out and the column ratios are bitwise
equal; two calls in a row, the second on a smaller problem, so the shared
static scratch is reused; sizes above its limit are refused before any
launch."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import apo
from paper_2310_17137_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2310_17137_amd import ap  # noqa: E402


def _case(w, epochs):
    print(f"[noalloc] n={w.n} d={w.d} l={w.l} kernel={w.kernel}", flush=True)
    s, B, W, R = ap.from_workload(w, device="cuda:0", tile=ap.TILE_FP64)
    s.reset(B, W, R)
    s.epoch(B, W, R, epochs)
    ref = torch.empty_like(R)
    cols_ref = s.residual(B, W, R, R_out=ref)
    got = torch.full_like(R, float("nan"))
    cols = ap.residual_noalloc(s.X, B, W, got, kernel=w.kernel, lengthscale=w.lengthscale,
                               outputscale=w.outputscale, noise=w.noise)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert np.array_equal(cols, cols_ref)
    return got, cols


def test_noalloc_residual_equals_handle_residual_twice():
    big = gen.small(21, 70000, 3, 7, 512, kernel=apo.RBF, noise=0.01, ell=0.2)
    small = gen.small(22, 1234, 5, 3, 100, kernel=apo.MATERN52, noise=0.05, ell=0.7)
    got, cols = _case(big, 2)
    # the second call reuses the scratch the first one left behind
    _case(small, 1)
    assert np.all(np.isfinite(cols)) and got.abs().max().item() > 0


def test_noalloc_refuses_sizes_beyond_its_scratch():
    n = ap.NOALLOC_MAX_N + 1
    X = torch.zeros((n, 1), dtype=torch.float32, device="cuda:0")
    B = torch.zeros((n, 1), dtype=torch.float32, device="cuda:0")
    W = torch.zeros((n, 1), dtype=torch.float64, device="cuda:0")
    R = torch.zeros((n, 1), dtype=torch.float32, device="cuda:0")
    with pytest.raises(ap.ApError) as e:
        ap.residual_noalloc(X, B, W, R, kernel=ap.RBF, lengthscale=1.0)
    assert e.value.code == ap.ERR_UNSUPPORTED
    assert "AP_NOALLOC_MAX_N" in ap.last_error()
