"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Every case draws its inputs from the seeded generators; the oracle and the GPU
see the same FP32 values (the oracle widened to FP64). Tolerances:
  - cached block inverses (FP64): 1e-9 relative to the largest entry, times the
    block's condition number over 1e4;
  - FP32 tiles: iterates W within 1e-5 relative (Frobenius) of the oracle's.
    The residual R is FP32, so after an update its error is bounded by FP32
    rounding of K^_{:,I} delta: ||dR|| <= 1e-5 ||R|| + 2 u32 || |K^_{:,I}| |delta| ||
    (u32 = 2^-24). Where that amplification factor || |K||delta| || / ||R|| is
    large (ill-conditioned cases) the iterates inherit it, and the bar becomes
    4 u32 times the factor. Over several epochs the bar is at most twice the
    FP32-tile floor (tests.helpers.fp32_tile_floor): the distance from the
    oracle of a perfect FP32-tile run of the same updates (kernel values and
    step correctly rounded to FP32, 32-column chunks (64-column pairs for
    l > 16) summed in FP32, emulated
    on the CPU), printed with the GPU's error for every epoch. The FP32 sums
    inside each chunk, not the kernel values, set that floor: on the 4096-point
    recipe it is 3.4e-5 after 30 epochs, against 7e-6 with the kernel values
    rounded and FP64 sums. The GPU's kernel values are within about 2 ulp (the
    unit-block column test checks that);
  - BF16 tiles: one update within 2e-2 relative; solves reach a true FP64
    relative residual below the tolerance;
  - FP64 true residual: 1e-9 relative to ||B||.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import apo
from paper_2310_17137_amd import gen
from tests.helpers import dense_khat, fp32_tile_floor, tile_trajectory, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2310_17137_amd import ap  # noqa: E402


def _gpu(w, tile=ap.TILE_FP32, **over):
    print(f"[case] {w.name} n={w.n} d={w.d} l={w.l} b={w.b} kernel={w.kernel} tile={tile} {over}",
          flush=True)
    return ap.from_workload(w, tile=tile, **over)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = [
    # (seed, n, d, l, b, kernel, noise, ell)
    (0, 1000, 3, 1, 100, apo.RBF, 0.1, 0.3),         # b not a multiple of 64, ragged last block
    (1, 777, 5, 7, 128, apo.MATERN32, 0.05, 0.6),    # ragged n, odd l
    (2, 1536, 8, 16, 512, apo.MATERN52, 0.01, 1.2),
    (3, 700, 11, 32, 256, apo.RBF, 0.02, 0.9),       # full RHS bucket, d = 11
    (4, 300, 16, 3, 300, apo.MATERN52, 0.1, 2.0),    # one block (b = n), d = 16
    (5, 2048, 2, 32, 64, apo.MATERN32, 0.001, 0.2),  # many small blocks
]


def _small(case, order=apo.CYCLIC):
    seed, n, d, l, b, kern, noise, ell = case
    rng = np.random.default_rng(100 + seed)
    ls = ell * rng.uniform(0.7, 1.4, size=d)
    return gen.small(seed, n, d, l, b, kernel=kern, noise=noise, ell=ls, outputscale=1.3,
                     order=order, dist="normal" if seed % 2 else "uniform")


@pytest.mark.parametrize("case", CASES[:5])
def test_block_inverses_match_dense(case):
    w = _small(case)
    s, B, W, R = _gpu(w)
    p = to_oracle(w)
    K = dense_khat(p)
    for j in sorted({0, s.m // 2, s.m - 1}):
        blk = p.block(j)
        ref = np.linalg.inv(K[blk, blk])
        got = s.block_inverse(j).cpu().numpy()
        kappa = np.linalg.cond(K[blk, blk])
        tol = 1e-9 * max(1.0, kappa / 1e4) * np.abs(ref).max()
        np.testing.assert_allclose(got, ref, rtol=0, atol=tol)


U32 = 2.0 ** -24


def _amplification(p, K, blk, delta, R_new):
    s = p.block(blk)
    return np.linalg.norm(np.abs(K[:, s]) @ np.abs(delta)) / max(np.linalg.norm(R_new), 1e-300)


@pytest.mark.parametrize("case", CASES)
def test_single_update_fp32(case):
    w = _small(case)
    s, B, W, R = _gpu(w)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    K = dense_khat(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    tol = 1e-5
    for blk in [s.m - 1, 0]:
        delta = apo.update(p, L, Wo, Ro, blk)
        s.update(B, W, R, blk)
        torch.cuda.synchronize()
        # the first step is an FP64 solve of the same FP32 R_I; the second one
        # sees the first update's FP32 rounding, amplified as for the iterates
        assert _rel(W.cpu().numpy(), Wo) < tol
        tol = max(1e-5, 4 * U32 * _amplification(p, K, blk, delta, Ro))
        sl = p.block(blk)
        bound = 1e-5 * np.linalg.norm(Ro) + 2 * U32 * np.linalg.norm(np.abs(K[:, sl]) @ np.abs(delta))
        assert np.linalg.norm(R.cpu().numpy() - Ro) <= bound
        assert np.all(R.cpu().numpy()[sl] == 0.0)  # the projection zeroes R_I


def _epoch_tol(p, L, K):
    Wt, Rt = np.zeros_like(p.B), p.B.copy()
    delta = apo.update(p, L, Wt, Rt, 0)
    return max(1e-5, 4 * U32 * _amplification(p, K, 0, delta, Rt))


@pytest.mark.parametrize("case", CASES)
def test_epochs_fp32_match_oracle(case):
    w = _small(case)
    s, B, W, R = _gpu(w)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    K = dense_khat(p)
    tol = _epoch_tol(p, L, K) if p.m > 1 else 1e-5
    floor = fp32_tile_floor(p, 3)
    tol = max(tol, 2 * max(floor))
    print(f"[tol] W iterates within {tol:.2e}", flush=True)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for ep in range(3):
        s.epoch(B, W, R, 1)
        apo.epoch(p, L, Wo, Ro)
        rho, cols = s.rel_residual()
        e = _rel(W.cpu().numpy(), Wo)
        print(f"[fp32] epoch {ep + 1} W err {e:.3e} floor {floor[ep]:.3e}", flush=True)
        assert e < tol, ep
        rho_o = apo.rel_residual(p, Ro)
        assert abs(rho - rho_o) <= max(tol * rho_o, 1e-7)


@pytest.mark.parametrize("case", [CASES[1], CASES[3], CASES[5]])
def test_greedy_fp32_match_oracle(case):
    w = _small(case, order=apo.GREEDY)
    s, B, W, R = _gpu(w)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for _ in range(2):
        s.epoch(B, W, R, 1)
        apo.epoch(p, L, Wo, Ro)
        torch.cuda.synchronize()
        assert _rel(W.cpu().numpy(), Wo) < 1e-5


@pytest.mark.parametrize("case", CASES)
def test_single_update_split(case):
    """Split path: FP32 tiles from plain FP32 features (kernel values within a
    few FP32 ulps) times a three-term BF16 split of tile and step: the change of
    R is bounded like the FP32 path's, with 8 u32 for the tile's ulps."""
    w = _small(case)
    s, B, W, R = _gpu(w, tile=ap.TILE_SPLIT)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    K = dense_khat(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for blk in [s.m // 2, 0]:
        delta = apo.update(p, L, Wo, Ro, blk)
        s.update(B, W, R, blk)
        torch.cuda.synchronize()
        sl = p.block(blk)
        mag = np.linalg.norm(np.abs(K[:, sl]) @ np.abs(delta))
        err = np.linalg.norm(R.cpu().numpy() - Ro)
        print(f"[split] |dR| {err:.3e} bound {1e-5 * np.linalg.norm(Ro) + 8 * U32 * mag:.3e}")
        assert err <= 1e-5 * np.linalg.norm(Ro) + 8 * U32 * mag
        assert np.all(R.cpu().numpy()[sl] == 0.0)


@pytest.mark.parametrize("case", CASES)
def test_epochs_split_match_oracle(case):
    w = _small(case)
    s, B, W, R = _gpu(w, tile=ap.TILE_SPLIT)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    K = dense_khat(p)
    tol = 2 * _epoch_tol(p, L, K) if p.m > 1 else 1e-5
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for ep in range(3):
        s.epoch(B, W, R, 1)
        apo.epoch(p, L, Wo, Ro)
        rho, _ = s.rel_residual()
        e = _rel(W.cpu().numpy(), Wo)
        print(f"[split] epoch {ep + 1} W err {e:.3e} (tol {tol:.2e})", flush=True)
        assert e < tol, ep


@pytest.mark.parametrize("case", CASES)
def test_epochs_fp64_tiles_match_oracle(case):
    """FP64 kernel tiles: only the stored residual is FP32, so the iterates stay
    within 1e-5 of the oracle's whatever the conditioning."""
    w = _small(case)
    s, B, W, R = _gpu(w, tile=ap.TILE_FP64)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for ep in range(3):
        s.epoch(B, W, R, 1)
        apo.epoch(p, L, Wo, Ro)
        rho, _ = s.rel_residual()
        e = _rel(W.cpu().numpy(), Wo)
        print(f"[fp64] epoch {ep + 1} W err {e:.3e}", flush=True)
        assert e < 1e-5, ep
        rho_o = apo.rel_residual(p, Ro)
        assert abs(rho - rho_o) <= max(1e-5 * rho_o, 1e-7)


@pytest.mark.parametrize("case,tile", [(CASES[0], ap.TILE_FP64), (CASES[1], ap.TILE_FP64),
                                       (CASES[5], ap.TILE_FP64), (CASES[3], ap.TILE_SPLIT)])
def test_random_order_matches_oracle(case, tile):
    """Random order (Section 3, "Block Selection"): the device draws each
    update's block from the seeded generator, the oracle from its own
    implementation of the same generator; the iterates agree as for cyclic
    order (a different block anywhere would move W by far more)."""
    w = _small(case, order=apo.RANDOM)
    w.seed = 31337 + case[0]
    s, B, W, R = _gpu(w, tile=tile)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    K = dense_khat(p)
    tol = 1e-5 if tile == ap.TILE_FP64 else max(2 * _epoch_tol(p, L, K), 1e-5)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for ep in range(3):
        s.epoch(B, W, R, 1)
        apo.epoch(p, L, Wo, Ro, ep)
        e = _rel(W.cpu().numpy(), Wo)
        print(f"[random] epoch {ep + 1} W err {e:.3e} (bound {tol:.1e})", flush=True)
        assert e < tol, ep


@pytest.mark.parametrize("n,d,l,b,kern,order", [
    (8500, 3, 4, 4096, apo.RBF, apo.GREEDY),     # the largest block (m = 3, last block 308)
    (900, 20, 20, 256, apo.MATERN32, apo.CYCLIC),  # the most features, matrix-core product
])
def test_limits_fp64_tiles_match_oracle(n, d, l, b, kern, order):
    """The build's size limits (b = 4096, d = 20) on FP64 tiles: two epochs
    against the oracle's iterates, as for the small cases."""
    rng = np.random.default_rng(n + d)
    w = gen.small(12, n, d, l, b, kernel=kern, noise=0.05,
                  ell=(0.3 if d == 3 else 2.0) * rng.uniform(0.8, 1.25, size=d), order=order)
    s, B, W, R = _gpu(w, tile=ap.TILE_FP64)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for ep in range(2):
        s.epoch(B, W, R, 1)
        apo.epoch(p, L, Wo, Ro, ep)
        e = _rel(W.cpu().numpy(), Wo)
        print(f"[limits] n={n} d={d} b={b} epoch {ep + 1}: W err {e:.3e}", flush=True)
        assert e < 1e-5, ep


@pytest.mark.parametrize("tile", [ap.TILE_FP32, ap.TILE_SPLIT])
@pytest.mark.parametrize("n,d,l,b,kern,order", [
    (8500, 3, 4, 4096, apo.RBF, apo.GREEDY),     # the largest block, vector-unit product
    (900, 20, 20, 256, apo.MATERN32, apo.CYCLIC),  # the most features, 32-row matrix tile
    (900, 20, 12, 256, apo.MATERN52, apo.CYCLIC),  # the most features, 16-row matrix tile
    (700, 11, 16, 128, apo.RBF, apo.GREEDY),     # 11 features padded to 12, 16-row tile
    (600, 16, 10, 100, apo.MATERN32, apo.CYCLIC),  # 16 features, 16-row tile, ragged blocks
])
def test_limits_reduced_tiles_match_oracle(n, d, l, b, kern, order, tile):
    """The size limits on FP32 and split tiles: two epochs against the
    oracle's iterates, with the bars of the small cases (FP32: twice the
    emulated FP32-tile floor or the amplification bound; split: twice the
    amplification bound)."""
    rng = np.random.default_rng(n + d)
    w = gen.small(12, n, d, l, b, kernel=kern, noise=0.05,
                  ell=(0.3 if d == 3 else 2.0) * rng.uniform(0.8, 1.25, size=d), order=order)
    s, B, W, R = _gpu(w, tile=tile)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    K = dense_khat(p)
    base = _epoch_tol(p, L, K)
    if tile == ap.TILE_FP32:
        tol = max(base, 2 * max(fp32_tile_floor(p, 2)))
    else:
        tol = 2 * base
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for ep in range(2):
        s.epoch(B, W, R, 1)
        apo.epoch(p, L, Wo, Ro, ep)
        e = _rel(W.cpu().numpy(), Wo)
        print(f"[limits] tile {tile} n={n} d={d} b={b} epoch {ep + 1}: W err {e:.3e} "
              f"bar {tol:.3e}", flush=True)
        assert e < tol, ep


@pytest.mark.parametrize("tile", [ap.TILE_FP32, ap.TILE_SPLIT, ap.TILE_FP64, ap.TILE_BF16])
def test_single_point_system_is_solved_in_one_update(tile):
    """n = 1: K^ = s + sigma^2, so one update gives W = B / (s + sigma^2) and
    R = 0 exactly (the projection zeroes the block's rows), in every tile mode."""
    w = gen.small(21, 1, 1, 3, 1, kernel=apo.MATERN52, noise=0.25, ell=0.7, outputscale=1.3)
    s, B, W, R = _gpu(w, tile=tile)
    s.reset(B, W, R)
    s.epoch(B, W, R, 1)
    torch.cuda.synchronize()
    expect = w.B.astype(np.float64) / (1.3 + 0.25)
    np.testing.assert_allclose(W.cpu().numpy(), expect, rtol=1e-14, atol=0)
    assert np.all(R.cpu().numpy() == 0.0)
    rho, _ = s.rel_residual()
    assert rho == 0.0


@pytest.mark.parametrize("tile", [ap.TILE_FP32, ap.TILE_SPLIT, ap.TILE_FP64])
@pytest.mark.parametrize("n,d,l,b", [
    (2, 1, 3, 1),      # two unit blocks
    (300, 1, 9, 100),  # one feature; l = 9 takes the FP32 16-row matrix tile
    (65, 20, 32, 64),  # the widest features with l = 32, a last block of one point
    # a last block of 24 points: its 64-column FP64-tile step reaches 40 rows
    # past n, beyond the 32 padding rows (the staged sources are clamped)
    (224, 3, 32, 100),
])
def test_degenerate_shapes_match_oracle(n, d, l, b, tile):
    w = gen.small(22, n, d, l, b, kernel=apo.RBF, noise=0.1, ell=0.6 if d == 1 else 3.0)
    s, B, W, R = _gpu(w, tile=tile)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    K = dense_khat(p)
    tol = 1e-5 if tile == ap.TILE_FP64 else max(_epoch_tol(p, L, K),
                                                 2 * max(fp32_tile_floor(p, 3)))
    if tile == ap.TILE_SPLIT:
        tol *= 2
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for ep in range(3):
        s.epoch(B, W, R, 1)
        apo.epoch(p, L, Wo, Ro)
        e = _rel(W.cpu().numpy(), Wo)
        print(f"[shape] tile {tile} n={n} d={d} l={l} b={b} epoch {ep + 1}: W err {e:.3e} "
              f"bar {tol:.3e}", flush=True)
        assert e < tol, ep
        rho, _ = s.rel_residual()
        assert abs(rho - apo.rel_residual(p, Ro)) <= max(tol * apo.rel_residual(p, Ro), 1e-7)


def test_random_order_single_block_equals_cyclic():
    """m = 1: every draw is block 0, so random order is cyclic order bit for bit."""
    case = CASES[4]  # b = n
    wr = _small(case, order=apo.RANDOM)
    wr.seed = 99
    wc = _small(case)
    sr, B, Wr, Rr = _gpu(wr, tile=ap.TILE_FP64)
    sc, _, Wc, Rc = _gpu(wc, tile=ap.TILE_FP64)
    sr.reset(B, Wr, Rr)
    sc.reset(B, Wc, Rc)
    sr.epoch(B, Wr, Rr, 3)
    sc.epoch(B, Wc, Rc, 3)
    torch.cuda.synchronize()
    assert torch.equal(Wr, Wc) and torch.equal(Rr, Rc)


@pytest.mark.parametrize("l", [32, 1])
def test_c3_generator_fp64_tiles_track_oracle(l):
    """The ill-conditioned n = 2M recipe at n = 32768 (64-cluster mixture, RBF
    lengthscale 0.1, sigma^2 = 1e-4, b = 2048, 32 right-hand sides or the target
    column alone): FP64 tiles follow the oracle's iterates over 3 epochs, and
    the maintained residual stays the true one."""
    w = gen.c3(n=32768, l=l)
    s, B, W, R = _gpu(w, tile=ap.TILE_FP64)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for ep in range(3):
        s.epoch(B, W, R, 1)
        apo.epoch(p, L, Wo, Ro)
        rho, _ = s.rel_residual()
        e = _rel(W.cpu().numpy(), Wo)
        rho_o = apo.rel_residual(p, Ro)
        print(f"[c3-32k] epoch {ep + 1} rho {rho:.6f} oracle {rho_o:.6f} W err {e:.3e}", flush=True)
        assert abs(rho - rho_o) <= 1e-4 * rho_o
        assert e < 1e-3
    Rt = torch.empty_like(R)
    cols = s.residual(B, W, R, R_out=Rt)
    drift = float((R - Rt).norm() / Rt.norm())
    print(f"[c3-32k] maintained vs true residual {drift:.3e}", flush=True)
    assert drift < 1e-4


@pytest.mark.parametrize("case", CASES)
def test_single_update_bf16(case):
    w = _small(case)
    s, B, W, R = _gpu(w, tile=ap.TILE_BF16)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    blk = s.m // 2
    s.update(B, W, R, blk)
    delta = apo.update(p, L, Wo, Ro, blk)
    torch.cuda.synchronize()
    # the first update's W is an FP64 solve of the same R_I: as tight as FP32
    assert _rel(W.cpu().numpy(), Wo) < 1e-5
    # R - K^[:, I] delta with BF16 tiles (8-bit significands for the kernel
    # values and the step): the error of the change is bounded by 2^-7 times
    # the magnitude of the products, || |K^[:, I]| |delta| ||.
    K = dense_khat(p)
    sl = p.block(blk)
    mag = np.linalg.norm(np.abs(K[:, sl]) @ np.abs(delta))
    dR = R.cpu().numpy() - p.B
    dRo = Ro - p.B
    err = np.linalg.norm(dR - dRo)
    print(f"[bf16] |d(dR)| / |dR| = {err / np.linalg.norm(dRo):.3e}, bound {2**-7 * mag / np.linalg.norm(dRo):.3e}")
    assert err <= 2.0 ** -7 * mag
    assert np.all(R.cpu().numpy()[sl] == 0.0)


@pytest.mark.parametrize("case", CASES[:4])
def test_true_residual_fp64(case):
    w = _small(case)
    s, B, W, R = _gpu(w)
    s.reset(B, W, R)
    s.epoch(B, W, R, 2)
    Rt = torch.empty_like(R)
    cols = s.residual(B, W, R, R_out=Rt)
    p = to_oracle(w)
    Wg = W.cpu().numpy()
    ref = p.B - dense_khat(p) @ Wg
    nb = np.linalg.norm(p.B)
    assert np.linalg.norm(Rt.cpu().numpy() - ref) <= 1e-6 * nb  # stored as FP32
    ref_cols = np.linalg.norm(ref, axis=0) / np.linalg.norm(p.B, axis=0)
    np.testing.assert_allclose(cols, ref_cols, rtol=1e-9)
    # the maintained FP32 residual drifts from the true one by FP32 rounding
    tol = _epoch_tol(p, apo.factor(p), dense_khat(p))
    assert np.linalg.norm(R.cpu().numpy() - ref) <= tol * nb


def test_c1_trajectory_fp32():
    """C1 (n = 4096, RBF, b = 512, one RHS): 30 epochs against the oracle. The
    target is 1e-5. A perfect FP32-tile run is already 3.4e-5 from the oracle
    (the FP32 sums inside each 32-column chunk; kernel values rounded to FP32
    with FP64 sums give 7e-6), so the bar is max(1e-5, 2 x that floor); the
    floor and the GPU's error are printed for every epoch."""
    w = gen.c1()
    s, B, W, R = _gpu(w)
    s.reset(B, W, R)
    p = to_oracle(w)
    floor = fp32_tile_floor(p, 30)
    tol = max(1e-5, 2 * max(floor))
    print(f"[c1] tolerance {tol:.3e}", flush=True)
    L = apo.factor(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    worst = 0.0
    for ep in range(30):
        s.epoch(B, W, R, 1)
        apo.epoch(p, L, Wo, Ro)
        rho, _ = s.rel_residual()
        e = _rel(W.cpu().numpy(), Wo)
        rho_o = apo.rel_residual(p, Ro)
        print(f"[c1] epoch {ep + 1} rho {rho:.8f} oracle {rho_o:.8f} W err {e:.3e} "
              f"floor {floor[ep]:.3e}", flush=True)
        worst = max(worst, e)
        assert rho == pytest.approx(rho_o, rel=1e-4)  # a norm of the FP32 residual
    assert worst < tol


def test_solve_mixed_reaches_tolerance():
    """BF16 tiles with FP64 refinement reach a true relative residual < 1e-2."""
    w = gen.small(7, 3000, 3, 8, 256, kernel=apo.RBF, noise=0.1, ell=0.05)
    w.tol, w.refine_every, w.max_epochs = 1e-2, 5, 200
    s, B, W, R = _gpu(w, tile=ap.TILE_BF16)
    st = s.solve(B, W, R)
    assert st.converged, st
    assert st.rho_true < 1e-2
    p = to_oracle(w)
    rows = np.arange(0, w.n, 37)
    true = apo.residual_rows(p, W.cpu().numpy(), rows)
    col = np.linalg.norm(true, axis=0) / np.linalg.norm(p.B[rows], axis=0)
    assert col.mean() < 3e-2  # row-sampled estimate of the same ratio


def test_solve_fp32_matches_oracle_solve():
    w = gen.small(8, 2000, 3, 4, 200, kernel=apo.MATERN52, noise=0.1, ell=0.04)
    w.tol, w.max_epochs, w.min_epochs = 1e-3, 300, 2
    s, B, W, R = _gpu(w)
    st = s.solve(B, W, R)
    p = to_oracle(w)
    res = apo.solve(p)
    assert st.converged == res.converged
    assert st.epochs == res.epochs
    tol = max(1e-5, 2 * max(fp32_tile_floor(p, st.epochs)))
    e = _rel(W.cpu().numpy(), res.W)
    print(f"[solve-fp32] {st.epochs} epochs, W err {e:.3e}, bar {tol:.3e}", flush=True)
    assert e < tol


def test_not_positive_definite_reports_block():
    w = gen.small(9, 600, 2, 1, 100)
    X = w.X.copy()
    X[333] = X[310]  # duplicate inside block 3 (rows 300..399)
    Xt = torch.from_numpy(X).cuda()
    # a short lengthscale keeps every other block far from singular
    with pytest.raises(ap.ApError) as e:
        ap.Solver(Xt, l=1, b=100, kernel=ap.RBF, lengthscale=0.005, noise=0.0)
    assert e.value.code == ap.ERR_NOT_PD
    assert "block 3" in str(e.value)
    # by-index noise: the same points are fine
    ap.Solver(Xt, l=1, b=100, kernel=ap.RBF, lengthscale=0.005, noise=1e-3)


def test_invalid_arguments_and_workspace():
    X = torch.rand(100, 3, device="cuda")
    with pytest.raises(ap.ApError) as e:
        ap.Solver(X, l=1, b=0, kernel=ap.RBF, lengthscale=0.5)
    assert e.value.code == ap.ERR_INVALID_ARG
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(ap.ApError) as e:
        ap.Solver(X, l=1, b=50, kernel=ap.RBF, lengthscale=0.5, workspace=small)
    assert e.value.code == ap.ERR_WORKSPACE
    s = ap.Solver(X, l=1, b=50, kernel=ap.RBF, lengthscale=0.5)
    B = torch.rand(100, 1, device="cuda")
    W, R = s.new_state(B)
    with pytest.raises(ap.ApError):
        s.update(B, W, R, 2)  # block index out of range (m = 2)


def test_nonfinite_rhs_is_reported():
    X = torch.rand(200, 3, device="cuda")
    s = ap.Solver(X, l=2, b=50, kernel=ap.RBF, lengthscale=0.5)
    B = torch.rand(200, 2, device="cuda")
    B[17, 1] = float("nan")
    W, R = s.new_state(B)
    s.reset(B, W, R)
    s.epoch(B, W, R, 1)
    with pytest.raises(ap.ApError) as e:
        s.rel_residual()
    assert e.value.code == ap.ERR_NONFINITE


@pytest.mark.parametrize("tile", [ap.TILE_FP32, ap.TILE_FP64])
@pytest.mark.parametrize("where", ["one_block", "every_block"])
def test_greedy_never_selects_past_the_blocks(tile, where):
    """Modified Gauss-Southwell rule on a residual with NaN rows: a block whose
    norm is NaN is never selected; when every norm is NaN the rule takes block
    0 and sets the status word. Either way every update stays on the m blocks
    and the epoch ends with AP_ERR_NONFINITE."""
    print(f"[case] greedy nonfinite tile={tile} where={where}", flush=True)
    n, b = 400, 50  # m = 8
    X = torch.rand(n, 3, device="cuda")
    s = ap.Solver(X, l=2, b=b, kernel=ap.RBF, lengthscale=0.5, noise=0.1, order=ap.GREEDY,
                  tile=tile)
    B = torch.rand(n, 2, device="cuda")
    if where == "one_block":
        B[17, 1] = float("nan")  # block 0
    else:
        B[::b, 0] = float("nan")  # first row of every block
    W, R = s.new_state(B)
    s.reset(B, W, R)
    s.epoch(B, W, R, 2)
    torch.cuda.synchronize()
    assert s.peek().status == ap.ERR_NONFINITE
    with pytest.raises(ap.ApError) as e:
        s.rel_residual()
    assert e.value.code == ap.ERR_NONFINITE
    Wh = W.cpu().numpy()
    if where == "one_block":
        # block 0 never updated; every other block's steps finite
        assert np.all(Wh[:b] == 0.0)
        assert np.all(np.isfinite(Wh[b:]))
        assert np.any(Wh[b:] != 0.0)
    else:
        # only block 0 ever updated
        assert np.all(Wh[b:] == 0.0)


@pytest.mark.parametrize("kern", [apo.RBF, apo.MATERN32, apo.MATERN52])
@pytest.mark.parametrize("tile", [ap.TILE_FP32, ap.TILE_SPLIT, ap.TILE_BF16, ap.TILE_FP64])
def test_kernel_column_through_unit_blocks(kern, tile):
    """With b = 1 every block is one point j, the step is R_j / (s + sigma^2)
    and one update subtracts that step times the kernel column k(x_:, x_j): the
    change of R reads out the GPU's kernel values one column at a time.
    FP32-grade tiles: kernel values within about 2 ulp at every magnitude (the
    exponent's argument is carried to FP64 accuracy), the step and the product
    rounded once each, R stored in FP32: the bound is u32 (4 |R| + 6 |k delta|);
    FP64 tiles meet the same bound with room. BF16 tiles (8-bit products, the
    exponent's argument from BF16 products): 2^-7 |R| + |k delta|."""
    rng = np.random.default_rng(11)
    w = gen.small(12, 1500, 5, 3, 1, kernel=kern, noise=0.05,
                  ell=rng.uniform(0.15, 0.6, size=5), outputscale=1.7)
    s, B, W, R = _gpu(w, tile=tile)
    s.reset(B, W, R)
    p = to_oracle(w)
    L = apo.factor(p)
    K = dense_khat(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    for j in [0, 777, 1499]:
        R0 = Ro.copy()
        delta = apo.update(p, L, Wo, Ro, j)
        s.update(B, W, R, j)
        torch.cuda.synchronize()
        Rg = R.cpu().numpy().astype(np.float64)
        kcol = np.abs(K[:, j:j + 1])
        if tile == ap.TILE_BF16:
            rel, mag = 2.0 ** -7, np.abs(R0) + kcol * np.abs(delta)
        else:
            rel, mag = U32, 4 * np.abs(R0) + 6 * kcol * np.abs(delta)
        err = np.abs(Rg - Ro)
        err[j] = 0.0  # the selected row is zeroed by both
        print(f"[column] kern {kern} tile {tile} j {j}: worst err/bound "
              f"{np.max(err / (rel * mag)):.3f}", flush=True)
        assert np.all(err <= rel * mag)
        R.copy_(torch.from_numpy(Ro.astype(np.float32)).cuda())  # same start for the next column


@pytest.mark.parametrize("order", [apo.CYCLIC, apo.GREEDY, apo.RANDOM])
def test_graph_replay_equals_eager_launches(order):
    """Epochs replay a captured HIP graph; with profiling on the same launches
    go out one by one. Every replay, with eager work and synchronizations in
    between, gives bitwise the same W and R as the eager epochs."""
    w = _small(CASES[1], order=order)
    sg, B, Wg, Rg = _gpu(w, tile=ap.TILE_SPLIT)
    se, _, We, Re = _gpu(w, tile=ap.TILE_SPLIT)
    se.profile(True)
    sg.reset(B, Wg, Rg)
    se.reset(B, We, Re)
    for ep in range(4):
        sg.epoch(B, Wg, Rg, 1)
        se.epoch(B, We, Re, 1)
        torch.cuda.synchronize()
        _ = (Wg.sum() + We.sum()).item()  # eager work between replays
        assert torch.equal(Wg, We), ep
        assert torch.equal(Rg, Re), ep
        assert sg.rel_residual()[0] == se.rel_residual()[0]


def test_solve_escalates_to_fp64_tiles():
    """BF16 tiles on the ill-conditioned cluster recipe (n = 16384): an FP64
    true residual finds the maintained one off by more than 5% (or not finite),
    the rest of the solve runs on FP64 tiles, and from then on the maintained
    residual stays the true one."""
    w = gen.c3(n=16384, l=8)
    w.refine_every, w.max_epochs = 2, 6
    s, B, W, R = _gpu(w, tile=ap.TILE_BF16)
    st = s.solve(B, W, R)
    print(f"[escalate] {st}", flush=True)
    assert st.tile == ap.TILE_FP64 and 1 <= st.escalated_at <= 2
    # a restart from W = 0 happens at the escalation or not at all
    assert st.restarted_at in (-1, st.escalated_at)
    assert np.isfinite(st.rho_true) and np.isfinite(st.rho_maintained)
    Rt = torch.empty_like(R)
    s.residual(B, W, R, R_out=Rt)
    drift = float((R - Rt).norm() / Rt.norm())
    print(f"[escalate] maintained vs true after the solve {drift:.3e}", flush=True)
    assert drift < 1e-4


def _same_update(sa, sb, w, B, W, R, blk):
    """One update on block blk by two handles from the same (W, R): bitwise
    equal results mean the same tile arithmetic."""
    Wa, Ra, Wb, Rb = W.clone(), R.clone(), W.clone(), R.clone()
    sa.update(B, Wa, Ra, blk)
    sb.update(B, Wb, Rb, blk)
    torch.cuda.synchronize()
    return torch.equal(Ra, Rb) and torch.equal(Wa, Wb)


def test_solve_keeps_a_tile_set_by_the_caller():
    """ap_set_tile(FP64) on a split-tile handle, then ap_solve: the handle is
    still on FP64 tiles afterwards (its next update is bitwise an FP64-tile
    handle's, not a split-tile handle's)."""
    w = _small(CASES[1])
    w.max_epochs = 3
    s, B, W, R = _gpu(w, tile=ap.TILE_SPLIT)
    s.set_tile(ap.TILE_FP64)
    st = s.solve(B, W, R)
    assert st.tile == ap.TILE_FP64 and st.escalated_at == -1
    ref64, _, _, _ = _gpu(w, tile=ap.TILE_FP64)
    ref_split, _, _, _ = _gpu(w, tile=ap.TILE_SPLIT)
    assert _same_update(s, ref64, w, B, W, R, 1)
    assert not _same_update(s, ref_split, w, B, W, R, 1)


def test_solve_error_after_escalation_restores_the_tile():
    """A NaN in B: the first epoch's norms are not finite, the solve restarts
    on FP64 tiles, fails there too and returns AP_ERR_NONFINITE. The handle
    is back on its BF16 tiles afterwards (bitwise a fresh BF16 handle's next
    update on finite data)."""
    w = _small(CASES[0])
    s, B, W, R = _gpu(w, tile=ap.TILE_BF16)
    Bbad = B.clone()
    Bbad[5, 0] = float("nan")
    with pytest.raises(ap.ApError) as e:
        s.solve(Bbad, W, R)
    assert e.value.code == ap.ERR_NONFINITE
    ref16, _, _, _ = _gpu(w, tile=ap.TILE_BF16)
    ref64, _, _, _ = _gpu(w, tile=ap.TILE_FP64)
    s.reset(B, W, R)
    s.epoch(B, W, R, 1)
    assert _same_update(s, ref16, w, B, W, R, 2)
    assert not _same_update(s, ref64, w, B, W, R, 2)


@pytest.fixture(scope="module")
def c3_65k():
    """The ill-conditioned n = 2M recipe's generator at n = 65 536 with 16
    right-hand sides (b = 2048, m = 32): the oracle's first three cyclic epochs
    and the FP32-tile floor beside them (computed once for the tests below)."""
    w = gen.c3(n=65536, l=16)
    p = to_oracle(w)
    return w, p, tile_trajectory(p, 3, "fp32", log=lambda m: print(m, flush=True))


def test_c3_generator_fp32_tiles_track_oracle(c3_65k):
    """FP32 tiles (the mixed path's update, on the matrix cores for l = 16)
    over epochs 1-3: W within twice the emulated FP32-tile floor of the
    oracle's iterates, printed per epoch."""
    w, p, traj = c3_65k
    s, B, W, R = _gpu(w, tile=ap.TILE_FP32)
    s.reset(B, W, R)
    for ep, (Wo, floor) in enumerate(traj):
        s.epoch(B, W, R, 1)
        e = _rel(W.cpu().numpy(), Wo)
        print(f"[c3-65k fp32] epoch {ep + 1} W err {e:.3e} floor {floor:.3e}", flush=True)
        assert e < max(1e-5, 2 * floor), ep


def test_c3_generator_split_tiles_vs_oracle(c3_65k):
    """Split tiles on the same system: the tile and step are FP32-grade
    (three BF16 terms each), so W stays within twice the FP32-tile floor of
    the oracle's iterates. The BF16 matrix cores keep only the bits within
    FP32 range of each 16-product group's largest term, which moves the
    maintained residual away from the FP64 true one (printed beside it)."""
    w, p, traj = c3_65k
    s, B, W, R = _gpu(w, tile=ap.TILE_SPLIT)
    s.reset(B, W, R)
    Rt = torch.empty_like(R)
    for ep, (Wo, floor) in enumerate(traj):
        s.epoch(B, W, R, 1)
        e = _rel(W.cpu().numpy(), Wo)
        rho, _ = s.rel_residual()
        rt = float(np.mean(s.residual(B, W, R, R_out=Rt)))
        print(f"[c3-65k split] epoch {ep + 1} W err {e:.3e} floor {floor:.3e} "
              f"rho {rho:.6f} true {rt:.6f}", flush=True)
        assert e < 2 * floor, ep


def test_epochs_bf16_track_emulated_floor():
    """BF16 tiles on a well-conditioned system (n = 3000, sigma^2 = 0.1, RBF
    lengthscale 0.05): five cyclic epochs against the oracle, printed beside
    the emulated BF16-tile floor (kernel values and step rounded to BF16,
    sixteen products per FP32 accumulator step), within three times it (the
    floor leaves out the BF16 squared distance's own rounding)."""
    w = gen.small(7, 3000, 3, 8, 256, kernel=apo.RBF, noise=0.1, ell=0.05)
    p = to_oracle(w)
    traj = tile_trajectory(p, 5, "bf16", log=lambda m: print(m, flush=True))
    s, B, W, R = _gpu(w, tile=ap.TILE_BF16)
    s.reset(B, W, R)
    for ep, (Wo, floor) in enumerate(traj):
        s.epoch(B, W, R, 1)
        e = _rel(W.cpu().numpy(), Wo)
        print(f"[bf16] epoch {ep + 1} W err {e:.3e} floor {floor:.3e}", flush=True)
        assert e < 3 * floor, ep

