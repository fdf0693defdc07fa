"""The stochastic MLL gradient (ap_mll_grad) against the FP64 oracle. Both
sides sum the same n^2 FP64 terms C_ij dK^_ij/dtheta in different orders, so
the bound is 1e-11 of sum_ij |C_ij| |dK^_ij/dtheta| (computed here in numpy
for the bound only), plus the exact identity that the per-64-row partials add
up to the gradient."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import apo
from paper_2310_17137_amd import gen
from tests.helpers import to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2310_17137_amd import ap  # noqa: E402


def _abs_terms(p, W, rows):
    """sum over (i in rows, all j) of |C_ij| |dK^_ij/dtheta| per component."""
    X, B, ls, s = p.X, p.B, np.asarray(p.lengthscale, dtype=np.float64), p.outputscale
    P = p.l - 1
    bc = np.empty_like(B)
    bc[:, 0] = -0.5 * W[:, 0]
    if P:
        bc[:, 1:] = B[:, 1:] / (2.0 * P)
    out = np.zeros(p.d + 2)
    for i in rows:
        c = np.abs(bc @ W[i])
        dx2 = (X - X[i]) ** 2
        r2 = (dx2 / ls ** 2).sum(1)
        r = np.sqrt(r2)
        if p.kernel == apo.RBF:
            k = s * np.exp(-0.5 * r2)
            g = k
        elif p.kernel == apo.MATERN32:
            e = s * np.exp(-np.sqrt(3.0) * r)
            k, g = (1 + np.sqrt(3.0) * r) * e, 3.0 * e
        else:
            e = s * np.exp(-np.sqrt(5.0) * r)
            k, g = (1 + np.sqrt(5.0) * r + 5.0 * r2 / 3.0) * e, 5.0 / 3.0 * (1 + np.sqrt(5.0) * r) * e
        out[: p.d] += (c * g) @ dx2 / ls ** 3
        out[p.d] += c @ k / s
        out[p.d + 1] += c[i]
    return out


CASES = [
    # (seed, n, d, l, b, kernel, noise, ell)
    (0, 900, 3, 1, 128, gen.RBF, 0.1, 0.3),        # no probes: the quadratic term alone
    (1, 777, 5, 7, 128, gen.MATERN32, 0.05, 0.6),
    (2, 1100, 8, 16, 256, gen.MATERN52, 0.02, 1.2),
    (3, 500, 16, 32, 250, gen.RBF, 0.05, 2.0),
]


@pytest.mark.parametrize("case", CASES)
def test_mll_grad_matches_oracle(case):
    seed, n, d, l, b, kern, noise, ell = case
    rng = np.random.default_rng(60 + seed)
    w = gen.small(seed, n, d, l, b, kernel=kern, noise=noise,
                  ell=ell * rng.uniform(0.7, 1.4, size=d), outputscale=1.3)
    print(f"[mll-case] seed={seed} n={n} d={d} l={l} kernel={kern}", flush=True)
    s, B, W, R = ap.from_workload(w, tile=ap.TILE_FP64)
    s.reset(B, W, R)
    s.epoch(B, W, R, 3)  # weights of a partial solve
    g, part = s.mll_grad(B, W, R, partials=True)
    p = to_oracle(w)
    Wc = W.cpu().numpy()
    ref = apo.mll_grad(p, Wc)
    bound = 1e-11 * _abs_terms(p, Wc, range(n)) + 1e-300
    print(f"[mll] gpu {g} oracle {ref} worst err/bound {np.max(np.abs(g - ref) / bound):.3e}",
          flush=True)
    assert np.all(np.abs(g - ref) <= bound)
    pc = part.cpu().numpy()
    assert np.all(pc[:, d + 2:] == 0.0)
    np.testing.assert_allclose(pc[:, : d + 2].sum(0), g, rtol=1e-12, atol=1e-12 * np.abs(g).max())


def test_mll_grad_fullsize_sampled_row_slices():
    """n = 2M, l = 32 (y and 31 Rademacher probes), W ~ N(0, 1): three 64-row
    slices of the double sum (first, middle, the ragged last) against the
    oracle's sums over the same rows and all 2M columns."""
    w = gen.c3()
    print(f"[mll-fullsize] n={w.n} l={w.l}", flush=True)
    s, B, W, R = ap.from_workload(w, tile=ap.TILE_FP64)
    rng = np.random.default_rng(4)
    Wc = rng.standard_normal((w.n, w.l))
    W.copy_(torch.from_numpy(Wc))
    g, part = s.mll_grad(B, W, R, partials=True)
    pc = part.cpu().numpy()
    p = to_oracle(w)
    nsl = pc.shape[0]
    for k in [0, nsl // 2, nsl - 1]:
        r0, r1 = 64 * k, min(64 * k + 64, w.n)
        ref = apo.mll_grad(p, Wc, rows=(r0, r1))
        bound = 1e-11 * _abs_terms(p, Wc, range(r0, r1)) + 1e-300
        got = pc[k, : w.d + 2]
        print(f"[mll-fullsize] slice {k}: worst err/bound "
              f"{np.max(np.abs(got - ref) / bound):.3e}", flush=True)
        assert np.all(np.abs(got - ref) <= bound)
    np.testing.assert_allclose(pc[:, : w.d + 2].sum(0), g, rtol=1e-12,
                               atol=1e-12 * np.abs(g).max())
