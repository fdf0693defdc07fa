"""ctypes binding of the FP64 CPU oracle (``oracle/ap_oracle.c``).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module. The GPU path never does.

Arrays are numpy float64, C-contiguous, row-major: X is n x d, B / W / R are
n x l. Section and equation names refer to Wu et al., "Large-Scale Gaussian
Processes via Alternating Projection" (AISTATS 2024).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ap_oracle.c")
_LIB = os.path.join(_HERE, "libaporacle.so")

RBF, MATERN32, MATERN52 = 0, 1, 2
CYCLIC, GREEDY, RANDOM = 0, 1, 2
KERNELS = {"rbf": RBF, "matern32": MATERN32, "matern52": MATERN52}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                        "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("l", ctypes.c_int32),
                ("b", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("lengthscale", ctypes.POINTER(ctypes.c_double)),
                ("outputscale", ctypes.c_double), ("noise", ctypes.c_double),
                ("order", ctypes.c_int32), ("tol", ctypes.c_double),
                ("min_epochs", ctypes.c_int32), ("max_epochs", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64, I32, D = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        C = ctypes.POINTER(_Cfg)
        sig = {
            "apo_num_threads": (I32, []),
            "apo_kernel": (D, [C, P, P]),
            "apo_khat_block": (None, [C, P, I64, I64, I64, I64, P]),
            "apo_num_blocks": (I64, [C]),
            "apo_cholesky": (I64, [P, I64]),
            "apo_factor": (I64, [C, P, P, P]),
            "apo_factor_one": (I64, [C, P, I64, P]),
            "apo_update_block": (None, [C, P, P, P, P, I64, P]),
            "apo_block_solve": (None, [P, I64, I32, P, P]),
            "apo_apply_update": (None, [C, P, P, I64, P]),
            "apo_update": (None, [C, P, P, P, P, I64, P]),
            "apo_block_norms": (None, [C, P, P]),
            "apo_select_greedy": (I64, [C, P]),
            "apo_splitmix64": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64]),
            "apo_select_random": (I64, [C, ctypes.c_uint64]),
            "apo_rel_residual": (D, [C, P, P]),
            "apo_epoch": (None, [C, P, P, P, P, I64, P]),
            "apo_solve": (I32, [C, P, P, P, P, P, P]),
            "apo_bcd_update": (None, [C, P, P, P, P, I64]),
            "apo_residual_rows": (None, [C, P, P, P, P, I64, P]),
            "apo_residual": (None, [C, P, P, P, P]),
            "apo_predict": (None, [C, P, P, P, I64, P]),
            "apo_mll_grad_rows": (None, [C, P, P, P, I64, I64, P]),
            "apo_mll_grad": (None, [C, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class Problem:
    """A kernel system K^ W = B with K^ = k(X, X) + noise * I (Section 2)."""
    X: np.ndarray
    B: np.ndarray
    kernel: int
    lengthscale: np.ndarray
    outputscale: float = 1.0
    noise: float = 0.1
    b: int = 512
    order: int = CYCLIC
    tol: float = 1e-2
    min_epochs: int = 0
    max_epochs: int = 1000
    seed: int = 0  # random order: seed of the block draws
    _keep: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        self.X = _f64(self.X)
        self.B = _f64(self.B)
        if self.B.ndim == 1:
            self.B = self.B[:, None].copy()
        self.lengthscale = _f64(np.broadcast_to(self.lengthscale, (self.X.shape[1],)))
        if isinstance(self.kernel, str):
            self.kernel = KERNELS[self.kernel]

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]

    @property
    def l(self):
        return self.B.shape[1]

    @property
    def m(self):
        return (self.n + self.b - 1) // self.b

    def cfg(self) -> _Cfg:
        c = _Cfg(self.n, self.d, self.l, self.b, int(self.kernel),
                 self.lengthscale.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 float(self.outputscale), float(self.noise), int(self.order), float(self.tol),
                 int(self.min_epochs), int(self.max_epochs),
                 int(self.seed) & 0xFFFFFFFFFFFFFFFF)
        self._keep = [self.lengthscale]
        return c

    def block(self, j: int) -> slice:
        return slice(j * self.b, min((j + 1) * self.b, self.n))


class NotPositiveDefinite(RuntimeError):
    def __init__(self, block: int, pivot: int):
        super().__init__(f"block {block}: non-positive Cholesky pivot at {pivot}")
        self.block, self.pivot = block, pivot


def num_threads() -> int:
    return int(_load().apo_num_threads())


def kernel(p: Problem, x, y) -> float:
    x, y = _f64(x), _f64(y)
    c = p.cfg()
    return _load().apo_kernel(ctypes.byref(c), _p(x), _p(y))


def khat_block(p: Problem, rows: slice, cols: slice) -> np.ndarray:
    """K^[rows, cols] with the noise added where row index == column index."""
    i0, i1, _ = rows.indices(p.n)
    j0, j1, _ = cols.indices(p.n)
    out = np.empty((i1 - i0, j1 - j0))
    c = p.cfg()
    _load().apo_khat_block(ctypes.byref(c), _p(p.X), i0, i1, j0, j1, _p(out))
    return out


def cholesky(A: np.ndarray) -> np.ndarray:
    A = _f64(A).copy()
    piv = _load().apo_cholesky(_p(A), A.shape[0])
    if piv >= 0:
        raise NotPositiveDefinite(-1, piv)
    return A


def factor(p: Problem) -> np.ndarray:
    """Cholesky factors of every K^_{I,I}: array m x b x b (last block in the
    leading len x len corner)."""
    L = np.zeros((p.m, p.b, p.b))
    piv = ctypes.c_int64(-1)
    c = p.cfg()
    bad = _load().apo_factor(ctypes.byref(c), _p(p.X), _p(L), ctypes.byref(piv))
    if bad >= 0:
        raise NotPositiveDefinite(bad, piv.value)
    return L


def factor_one(p: Problem, j: int) -> np.ndarray:
    """Cholesky factor of the single block K^_{I_j,I_j} (len_j x len_j)."""
    s = p.block(j)
    ln = s.stop - s.start
    Lj = np.zeros((ln, ln))
    c = p.cfg()
    piv = _load().apo_factor_one(ctypes.byref(c), _p(p.X), j, _p(Lj))
    if piv >= 0:
        raise NotPositiveDefinite(j, piv)
    return Lj


def update_block(p: Problem, Lj: np.ndarray, W: np.ndarray, R: np.ndarray, blk: int) -> np.ndarray:
    """One AP update in place given block blk's own factor; returns the step."""
    s = p.block(blk)
    delta = np.empty((s.stop - s.start, p.l))
    c = p.cfg()
    _load().apo_update_block(ctypes.byref(c), _p(p.X), _p(_f64(Lj)), _p(W), _p(R), blk,
                             _p(delta))
    return delta


def block_factor(L: np.ndarray, p: Problem, j: int) -> np.ndarray:
    ln = p.block(j).stop - p.block(j).start
    return np.ascontiguousarray(L[j].reshape(-1)[: ln * ln].reshape(ln, ln))


def block_solve(Lj: np.ndarray, RI: np.ndarray) -> np.ndarray:
    Lj, RI = _f64(Lj), _f64(RI)
    if RI.ndim == 1:
        RI = RI[:, None].copy()
    out = np.empty_like(RI)
    _load().apo_block_solve(_p(Lj), Lj.shape[0], RI.shape[1], _p(RI), _p(out))
    return out


def apply_update(p: Problem, R: np.ndarray, blk: int, delta: np.ndarray) -> None:
    """R <- R - K^_{:,I} delta in place (eq. text_update_of_r)."""
    c = p.cfg()
    delta = _f64(delta)
    _load().apo_apply_update(ctypes.byref(c), _p(p.X), _p(R), blk, _p(delta))


def update(p: Problem, L: np.ndarray, W: np.ndarray, R: np.ndarray, blk: int) -> np.ndarray:
    """One AP update in place; returns the step K^_{I,I}^{-1} R_I."""
    s = p.block(blk)
    delta = np.empty((s.stop - s.start, p.l))
    c = p.cfg()
    _load().apo_update(ctypes.byref(c), _p(p.X), _p(L), _p(W), _p(R), blk, _p(delta))
    return delta


def block_norms(p: Problem, R: np.ndarray) -> np.ndarray:
    out = np.empty(p.m)
    c = p.cfg()
    _load().apo_block_norms(ctypes.byref(c), _p(_f64(R)), _p(out))
    return out


def select_greedy(p: Problem, R: np.ndarray) -> int:
    c = p.cfg()
    return int(_load().apo_select_greedy(ctypes.byref(c), _p(_f64(R))))


def rel_residual(p: Problem, R: np.ndarray, B: np.ndarray | None = None) -> float:
    B = p.B if B is None else _f64(B)
    c = p.cfg()
    return float(_load().apo_rel_residual(ctypes.byref(c), _p(_f64(R)), _p(B)))


def epoch(p: Problem, L: np.ndarray, W: np.ndarray, R: np.ndarray, t: int = 0) -> np.ndarray:
    """One epoch of m updates in place; returns the selected blocks. t is the
    number of epochs before this one (the random rule's draws continue
    across epochs)."""
    sel = np.empty(p.m, dtype=np.int64)
    c = p.cfg()
    _load().apo_epoch(ctypes.byref(c), _p(p.X), _p(L), _p(W), _p(R), int(t), _p(sel))
    return sel


def splitmix64(seed: int, k: int) -> int:
    """Output k (from 0) of SplitMix64 seeded with `seed`."""
    return int(_load().apo_splitmix64(int(seed) & 0xFFFFFFFFFFFFFFFF, int(k)))


def select_random(p: Problem, u: int) -> int:
    """The random rule's block for update u since the start of the solve."""
    c = p.cfg()
    return int(_load().apo_select_random(ctypes.byref(c), int(u)))


@dataclass
class SolveResult:
    W: np.ndarray
    R: np.ndarray
    rho: np.ndarray
    epochs: int
    converged: bool


def solve(p: Problem) -> SolveResult:
    """Algorithm 1 with the paper's stopping rule (see module docstring)."""
    W = np.zeros((p.n, p.l))
    R = np.zeros((p.n, p.l))
    rho = np.zeros(max(p.max_epochs, 1))
    ep = ctypes.c_int32(0)
    c = p.cfg()
    st = _load().apo_solve(ctypes.byref(c), _p(p.X), _p(p.B), _p(W), _p(R), _p(rho),
                           ctypes.byref(ep))
    if st == -2:
        raise NotPositiveDefinite(ep.value, -1)
    return SolveResult(W, R, rho[: ep.value].copy(), ep.value, st == 0)


def bcd_update(p: Problem, L: np.ndarray, W: np.ndarray, blk: int) -> None:
    """Algorithm 2 step in place: W_I <- K^_{I,I}^{-1}(B_I - K^_{I,not I} W_{not I})."""
    c = p.cfg()
    _load().apo_bcd_update(ctypes.byref(c), _p(p.X), _p(L), _p(p.B), _p(W), blk)


def residual_rows(p: Problem, W: np.ndarray, rows) -> np.ndarray:
    """B[rows] - K^[rows, :] W in FP64 (Lemma residual_equality)."""
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    W = _f64(W)
    out = np.empty((rows.size, p.l))
    c = p.cfg()
    _load().apo_residual_rows(ctypes.byref(c), _p(p.X), _p(p.B), _p(W), _p(rows), rows.size,
                              _p(out))
    return out


def predict(p: Problem, W: np.ndarray, Xs: np.ndarray) -> np.ndarray:
    """Posterior mean K(Xs, X) W at the test points Xs (ns x d), in FP64."""
    Xs = np.ascontiguousarray(_f64(Xs).reshape(-1, p.d))
    W = _f64(W)
    out = np.empty((Xs.shape[0], p.l))
    c = p.cfg()
    _load().apo_predict(ctypes.byref(c), _p(p.X), _p(W), _p(Xs), Xs.shape[0], _p(out))
    return out


def mll_grad(p: Problem, W: np.ndarray, rows: tuple[int, int] | None = None) -> np.ndarray:
    """Stochastic estimate of the negative log marginal likelihood's gradient
    in (lengthscales, outputscale, noise) from W = K^^{-1} B, B = [y, probes]
    (Section 2, eq. loss_grad_unbiased); rows = (i0, i1) sums only those rows
    of the double sum."""
    W = _f64(W)
    out = np.empty(p.d + 2)
    c = p.cfg()
    i0, i1 = rows if rows is not None else (0, p.n)
    _load().apo_mll_grad_rows(ctypes.byref(c), _p(p.X), _p(p.B), _p(W), int(i0), int(i1),
                              _p(out))
    return out


def residual(p: Problem, W: np.ndarray) -> np.ndarray:
    W = _f64(W)
    out = np.empty((p.n, p.l))
    c = p.cfg()
    _load().apo_residual(ctypes.byref(c), _p(p.X), _p(p.B), _p(W), _p(out))
    return out


def adam_train(p: Problem, steps: int, epochs: int, lr: float = 0.1, warm: bool = True,
               beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """The training loop in FP64 (Section 5, "MLL Optimization": Adam with step
    size 0.1 on the stochastic gradient of eq. loss_grad_unbiased): per step,
    the block factors at the current (lengthscales, outputscale, noise), exactly
    `epochs` epochs of Algorithm 1 from the previous step's W (R = B - K^ W, by
    Lemma residual_equality) or, without warm, from W = 0, the gradient, and
    one Adam step (Kingma and Ba, 2015) on the logarithms of the
    hyperparameters. Returns the hyperparameters and gradients of every step,
    each a (steps x (d + 2)) array."""
    import dataclasses
    d = p.d
    phi = np.log(np.concatenate([p.lengthscale, [p.outputscale, p.noise]]))
    m1 = np.zeros_like(phi)
    m2 = np.zeros_like(phi)
    W = np.zeros_like(p.B)
    thetas, grads = [], []
    for t in range(1, steps + 1):
        theta = np.exp(phi)
        q = dataclasses.replace(p, lengthscale=theta[:d].copy(), outputscale=float(theta[d]),
                                noise=float(theta[d + 1]))
        L = factor(q)
        if warm and t > 1:
            R = residual(q, W)
        else:
            W = np.zeros_like(p.B)
            R = q.B.copy()
        for e in range(epochs):
            epoch(q, L, W, R, e)
        g = mll_grad(q, W)
        thetas.append(theta)
        grads.append(g)
        gphi = g * theta
        m1 = beta1 * m1 + (1 - beta1) * gphi
        m2 = beta2 * m2 + (1 - beta2) * gphi ** 2
        phi = phi - lr * (m1 / (1 - beta1 ** t)) / (np.sqrt(m2 / (1 - beta2 ** t)) + eps)
    return np.array(thetas), np.array(grads)
