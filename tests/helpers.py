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


def fp32_rounding_floor(p, epochs: int, order_blocks=None) -> float:
    """Relative distance, after `epochs` cyclic epochs, between the FP64 oracle
    iterates and the iterates of the same updates with every kernel value
    K^_ij rounded once to FP32 and R stored in FP32 after each update (block
    solves, the product's accumulation and W kept in FP64). It is the error a
    perfect FP32-tile implementation would show, the rounding floor against
    which the GPU's FP32-grade paths are judged."""
    from oracle import apo
    K = apo.khat_block(p, slice(0, p.n), slice(0, p.n))
    K32 = K.astype(np.float32).astype(np.float64)
    L = apo.factor(p)
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    W, R = np.zeros_like(p.B), p.B.astype(np.float32).astype(np.float64)
    blocks = list(range(p.m)) if order_blocks is None else order_blocks
    for _ in range(epochs):
        apo.epoch(p, L, Wo, Ro)
        for j in blocks:
            s = p.block(j)
            d = apo.block_solve(apo.block_factor(L, p, j), R[s])
            W[s] += d
            R = (R - K32[:, s] @ d).astype(np.float32).astype(np.float64)
            R[s] = 0.0
    return float(np.linalg.norm(W - Wo) / np.linalg.norm(Wo))
