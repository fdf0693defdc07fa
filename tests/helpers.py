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


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32)


_FLOOR_LIB = None


def _floor_lib():
    """tests/tile_floor.c, compiled on first use (gcc, OpenMP) next to it."""
    global _FLOOR_LIB
    if _FLOOR_LIB is None:
        import ctypes
        import os
        import subprocess
        here = os.path.dirname(os.path.abspath(__file__))
        src = os.path.join(here, "tile_floor.c")
        lib = os.path.join(here, "_tile_floor.so")
        if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", lib + ".tmp", src],
                           check=True)
            os.replace(lib + ".tmp", lib)
        L = ctypes.CDLL(lib)
        P = ctypes.c_void_p
        L.chunk_products.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, P]
        L.chunk_products.restype = None
        _FLOOR_LIB = L
    return _FLOOR_LIB


def _chunk_products(Kt, dt, group: int, span: int = 32) -> np.ndarray:
    """Sum_q Kt[:, q] dt[q] over a block as the matrix cores form it (see
    tests/tile_floor.c): FP32 sums over runs of span columns, `group` products
    per rounding. Kt (n x len) and dt (len x l) hold the rounded operands
    (float32)."""
    Kt = np.ascontiguousarray(Kt, dtype=np.float32)
    dt = np.ascontiguousarray(dt, dtype=np.float32)
    n, ln = Kt.shape
    l = dt.shape[1]
    out = np.empty((n, l))
    _floor_lib().chunk_products(Kt.ctypes.data, dt.ctypes.data, n, ln, l, group, span,
                                out.ctypes.data)
    return out


def fp32_product_group(l: int) -> int:
    """Products the FP32 tiles add per rounding of a chunk's FP32 accumulator:
    one (vector FMAs, l <= 8), four (v_mfma_f32_16x16x4f32, 8 < l <= 16) or
    two (v_mfma_f32_32x32x2f32)."""
    if l <= 8:
        return 1
    if l <= 16:
        return 4
    return 2


def fp32_sum_span(l: int) -> int:
    """Columns the FP32 tiles sum in one FP32 accumulator before adding the sum
    into FP64: a 32-column chunk, or a pair of chunks for the
    v_mfma_f32_32x32x2f32 kernel (l > 16)."""
    return 64 if l > 16 else 32


def tile_trajectory(p, epochs: int, mode: str = "fp32", log=None):
    """Cyclic epochs of the FP64 oracle beside a perfect reduced-precision
    tile implementation of the same updates. Returns, per epoch, the oracle's
    W and the relative distance (Frobenius) of the emulated run's W from it:
    the rounding floor the GPU's tiles are measured against.

    mode "fp32": every kernel value K^_ij rounded once to FP32 and the step
    s delta rounded to FP32; each chunk (32 columns, or a 64-column pair for
    l > 16: fp32_sum_span) summed on an FP32 accumulator as the FP32 tile
    kernel for this l forms it (fp32_product_group). mode "bf16":
    the kernel values over s and the step s delta rounded to BF16, sixteen
    products per accumulator step (v_mfma_f32_32x32x16_bf16). In both the
    chunk sums add up in FP64, R is stored in FP32 after each update with the
    block's rows set to 0, and block solves and W are FP64. The kernel columns
    of each block are formed as needed, so large n fits."""
    from oracle import apo
    L = apo.factor(p)
    group = fp32_product_group(p.B.shape[1])
    span = fp32_sum_span(p.B.shape[1])
    Wo, Ro = np.zeros_like(p.B), p.B.copy()
    W, R = np.zeros_like(p.B), p.B.astype(np.float32).astype(np.float64)
    so = p.outputscale
    out = []
    for _ in range(epochs):
        apo.epoch(p, L, Wo, Ro)
        for j in range(p.m):
            s = p.block(j)
            d = apo.block_solve(apo.block_factor(L, p, j), R[s])
            W[s] += d
            K = apo.khat_block(p, slice(0, p.n), s)
            if mode == "bf16":
                upd = so * _chunk_products(bf16(K / so), bf16(so * d), 16) / so
            else:
                upd = _chunk_products(K.astype(np.float32), d.astype(np.float32), group, span)
            del K
            R = (R - upd).astype(np.float32).astype(np.float64)
            R[s] = 0.0
        out.append((Wo.copy(), float(np.linalg.norm(W - Wo) / np.linalg.norm(Wo))))
        if log:
            log(f"[floor] {mode} epoch {len(out)}: {out[-1][1]:.3e}")
    return out


def fp32_tile_floor(p, epochs: int) -> list[float]:
    """Per-epoch FP32-tile rounding floor (tile_trajectory, mode "fp32")."""
    return [f for _, f in tile_trajectory(p, epochs, "fp32")]
