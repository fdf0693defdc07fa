"""Posterior mean at test points (ap_predict) against the FP64 oracle's
K(X*, X) W, element by element. Both sides compute FP64 kernel values and FP64
sums, in different orders, so the bound is relative to sum_j |k(x*, x_j)||W_j|:
1e-12 of it (2^-53 per operation over a few thousand terms, with room)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import apo
from paper_2310_17137_amd import gen
from tests.helpers import to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2310_17137_amd import ap  # noqa: E402

# (seed, n, d, l, b, kernel, noise, ell, ns)
CASES = [
    (0, 1000, 3, 1, 100, gen.RBF, 0.1, 0.3, 333),       # vector-unit path, ragged ns
    (1, 777, 5, 7, 128, gen.MATERN32, 0.05, 0.6, 129),
    (2, 1536, 8, 16, 512, gen.MATERN52, 0.01, 1.2, 256),  # matrix cores, one half
    (3, 700, 11, 32, 256, gen.RBF, 0.02, 0.9, 1),          # both halves, one test point
    (4, 300, 16, 3, 300, gen.MATERN52, 0.1, 2.0, 77),
]


def _bound(p, W, Xs):
    absw = np.abs(W)
    out = np.zeros((Xs.shape[0], p.l))
    for r in range(Xs.shape[0]):
        k = np.array([apo.kernel(p, Xs[r], p.X[j]) for j in range(p.n)])
        out[r] = np.abs(k) @ absw
    return out


@pytest.mark.parametrize("case", CASES)
def test_predict_matches_oracle(case):
    seed, n, d, l, b, kern, noise, ell, ns = case
    w = gen.small(seed, n, d, l, b, kernel=kern, noise=noise, ell=ell)
    print(f"[predict-case] seed={seed} n={n} d={d} l={l} ns={ns} kernel={kern}", flush=True)
    s, B, W, R = ap.from_workload(w, tile=ap.TILE_FP64)
    s.reset(B, W, R)
    s.epoch(B, W, R, 2)  # weights of a partial solve
    rng = np.random.default_rng(50 + seed)
    Xs = rng.uniform(0.0, 1.0, size=(ns, d)).astype(np.float32)
    mean = s.predict(W, torch.from_numpy(Xs).cuda()).cpu().numpy()
    p = to_oracle(w)
    Wc = W.cpu().numpy()
    ref = apo.predict(p, Wc, Xs.astype(np.float64))
    err = np.abs(mean - ref)
    bound = 1e-12 * _bound(p, Wc, Xs.astype(np.float64)) + 1e-300
    print(f"[predict] worst err/bound {np.max(err / bound):.3e}", flush=True)
    assert np.all(err <= bound)


def test_predict_at_training_points_is_b_minus_noise_times_w():
    """Property that holds at any size: at the training points, K W = K^ W -
    sigma^2 W, so B - mean = R_true + sigma^2 W with the FP64 true residual."""
    w = gen.small(7, 2000, 4, 5, 256, kernel=gen.MATERN32, noise=0.03, ell=0.5)
    s, B, W, R = ap.from_workload(w, tile=ap.TILE_FP64)
    s.reset(B, W, R)
    s.epoch(B, W, R, 3)
    X = torch.from_numpy(w.X).cuda()
    mean = s.predict(W, X).cpu().numpy()
    p = to_oracle(w)
    Wc = W.cpu().numpy()
    rtrue = apo.residual(p, Wc)
    lhs = p.B - mean
    np.testing.assert_allclose(lhs, rtrue + 0.03 * Wc, rtol=0,
                               atol=1e-11 * float(np.abs(p.B).max() + np.abs(Wc).max()))


@pytest.mark.parametrize("l", [32, 1])
def test_predict_fullsize_sampled_test_points(l):
    """The n = 2M workload: 48 test points drawn from the same mixture, weights
    W ~ N(0, 1) in FP64, against the oracle point by point."""
    w = gen.c3(l=l)
    print(f"[predict-fullsize] n={w.n} l={l}", flush=True)
    s, B, W, R = ap.from_workload(w, tile=ap.TILE_FP64)
    rng = np.random.default_rng(3)
    Wc = rng.standard_normal((w.n, w.l))
    W.copy_(torch.from_numpy(Wc))
    Xs = gen.c3(n=4096, l=1, seed=9).X[rng.choice(4096, size=48, replace=False)]
    mean = s.predict(W, torch.from_numpy(np.ascontiguousarray(Xs)).cuda()).cpu().numpy()
    p = to_oracle(w)
    ref = apo.predict(p, Wc, Xs.astype(np.float64))
    # the bound's magnitude sum_j |k(x*, x_j)| |W_j|, with the RBF row of each
    # test point evaluated in numpy (for the bound only; the expected values
    # are the oracle's)
    X64 = p.X
    mag = np.empty((Xs.shape[0], w.l))
    for r, x in enumerate(Xs.astype(np.float64)):
        krow = p.outputscale * np.exp(-0.5 * (((X64 - x) / w.lengthscale) ** 2).sum(1))
        mag[r] = krow @ np.abs(Wc)
    bound = 1e-12 * mag + 1e-300
    err = np.abs(mean - ref)
    print(f"[predict-fullsize] worst err {err.max():.3e}, worst err/bound "
          f"{np.max(err / bound):.3e}", flush=True)
    assert np.all(err <= bound)


def test_predict_edge_cases():
    w = gen.small(8, 500, 3, 2, 100)
    s, B, W, R = ap.from_workload(w, tile=ap.TILE_SPLIT)
    empty = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    assert s.predict(W, empty).shape == (0, 2)
    with pytest.raises(ValueError):
        s.predict(W, torch.empty((5, 4), dtype=torch.float32, device="cuda"))
    lib = ap.load()
    import ctypes
    code = lib.ap_predict(s.handle, ctypes.c_void_p(W.data_ptr()), ctypes.c_void_p(0), 5,
                          ctypes.c_void_p(0), ctypes.c_void_p(0))
    assert code == ap.ERR_INVALID_ARG
    code = lib.ap_predict(s.handle, ctypes.c_void_p(W.data_ptr()), ctypes.c_void_p(0), -1,
                          ctypes.c_void_p(0), ctypes.c_void_p(0))
    assert code == ap.ERR_INVALID_ARG
