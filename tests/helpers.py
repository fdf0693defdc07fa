"""Shared test helpers: bridge from the seeded workloads to the FP64 oracle, and
dense library-routine references (scikit-learn kernels, numpy solves) that are
independent of the oracle's own arithmetic."""
from __future__ import annotations

import numpy as np

from oracle import apo
from paper_2310_17137_amd import gen


def to_oracle(w: gen.Workload, **over) -> apo.Problem:
    kw = dict(X=w.X.astype(np.float64), B=w.B.astype(np.float64), kernel=w.kernel,
              lengthscale=w.lengthscale, outputscale=w.outputscale, noise=w.noise, b=w.b,
              order=w.order, tol=w.tol, min_epochs=w.min_epochs, max_epochs=w.max_epochs,
              seed=w.seed)
    kw.update(over)
    return apo.Problem(**kw)


def sk_kernel(kernel: int, lengthscale):
    from sklearn.gaussian_process.kernels import RBF, Matern
    ls = np.asarray(lengthscale, dtype=np.float64)
    if kernel == apo.RBF:
        return RBF(length_scale=ls)
    if kernel == apo.MATERN32:
        return Matern(length_scale=ls, nu=1.5)
    if kernel == apo.MATERN52:
        return Matern(length_scale=ls, nu=2.5)
    raise ValueError(kernel)


def dense_khat(p: apo.Problem) -> np.ndarray:
    """K^ = s k(X, X) + sigma^2 I from scikit-learn's kernel routines."""
    K = p.outputscale * sk_kernel(p.kernel, p.lengthscale)(p.X)
    return K + p.noise * np.eye(p.n)


def knorm2(E: np.ndarray, K: np.ndarray) -> float:
    """||E||_K^2 = tr(E^T K E)."""
    return float(np.sum(E * (K @ E)))


def fp32_tile_floor(p, epochs: int) -> list[float]:
    """Per-epoch relative distance (Frobenius) between the FP64 oracle's cyclic
    iterates and those of a perfect FP32-tile implementation of the same
    updates: every kernel value K^_ij rounded once to FP32, the step s delta
    rounded to FP32, the products of each 32-column chunk accumulated in FP32
    (numpy's FP32 matrix product), the chunk sums in FP64, and R stored in
    FP32 after each update; block solves and W in FP64. It is the rounding
    floor the GPU's FP32-grade tiles are judged against: their arithmetic
    differs only in the order of the FP32 sums and in kernel values within
    about 2 ulp instead of half an ulp."""
    from oracle import apo
    K32 = apo.khat_block(p, slice(0, p.n), slice(0, p.n)).astype(np.float32)
    L = apo.factor(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    W, R = np.zeros_like(p.B), p.B.astype(np.float32).astype(np.float64)
    out = []
    for _ in range(epochs):
        apo.epoch(p, L, Wo, Ro)
        for j in range(p.m):
            s = p.block(j)
            d = apo.block_solve(apo.block_factor(L, p, j), R[s])
            W[s] += d
            d32 = d.astype(np.float32)
            upd = np.zeros_like(R)
            for c0 in range(s.start, s.stop, 32):
                cs = slice(c0, min(c0 + 32, s.stop))
                upd += (K32[:, cs] @ d32[c0 - s.start:cs.stop - s.start]).astype(np.float64)
            R = (R - upd).astype(np.float32).astype(np.float64)
            R[s] = 0.0
        out.append(float(np.linalg.norm(W - Wo) / np.linalg.norm(Wo)))
    return out
