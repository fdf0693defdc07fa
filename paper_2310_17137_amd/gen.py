"""Seeded synthetic workloads for the alternating-projection solver.

This module draws inputs only: features X, right-hand sides B and kernel
hyperparameters. It holds none of the solver's arithmetic, and it is the one
module that both the GPU path's callers and the FP64 oracle's tests use.

The paper's own workloads are UCI regression sets that are not available here;
these draws stand in for them at the paper's scales (Section 5, Table 1):
n = 4096 (parity), 262 144, 2 000 000 (house-electric scale) and 4 000 000
(gas-sensors scale), plus a stream of serving requests. B follows the paper's
right-hand-side recipe: column 0 is a noisy label vector y, the remaining
columns are Rademacher probe vectors (Section 2 "Hyperparameter Training";
appendix "Further Experimental Details").

Every array is returned as float32 (X: n x d, B: n x l, row-major); the oracle
reads the same values widened to float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RBF, MATERN32, MATERN52 = 0, 1, 2
CYCLIC, GREEDY, RANDOM = 0, 1, 2
KERNEL_NAMES = {RBF: "rbf", MATERN32: "matern32", MATERN52: "matern52"}


@dataclass
class Workload:
    name: str
    X: np.ndarray            # n x d float32
    B: np.ndarray            # n x l float32
    kernel: int
    lengthscale: np.ndarray  # d float64
    outputscale: float
    noise: float
    b: int
    order: int = CYCLIC
    tol: float = 1e-2
    min_epochs: int = 0
    max_epochs: int = 1000
    refine_every: int = 0
    seed: int = 0            # random order: seed of the block draws
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]

    @property
    def l(self) -> int:
        return self.B.shape[1]

    @property
    def m(self) -> int:
        return (self.n + self.b - 1) // self.b


def _rademacher(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    return rng.integers(0, 2, size=(n, k), dtype=np.int8).astype(np.float64) * 2.0 - 1.0


def _rhs(rng, y: np.ndarray, l: int) -> np.ndarray:
    n = y.shape[0]
    B = np.empty((n, l), dtype=np.float64)
    B[:, 0] = y
    if l > 1:
        B[:, 1:] = _rademacher(rng, n, l - 1)
    return B.astype(np.float32)


def c1(seed: int = 0, n: int = 4096) -> Workload:
    """Plain FP64 parity case: n = 4096, d = 3, X ~ U[0,1]^3, RBF ell = 0.5,
    s = 1, sigma^2 = 0.1, y = sin(2 pi sum x) + N(0, 0.1^2), b = 512, cyclic,
    one right-hand side, tolerance 1e-2."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, size=(n, 3))
    y = np.sin(2 * np.pi * X.sum(1)) + 0.1 * rng.standard_normal(n)
    return Workload("c1", X.astype(np.float32), _rhs(rng, y, 1), RBF, np.full(3, 0.5), 1.0, 0.1,
                    b=512, tol=1e-2)


def c2(seed: int = 0, n: int = 262144, l: int = 16, b: int = 1024) -> Workload:
    """n = 262 144, d = 8, X ~ N(0, I), Matern-5/2 ARD with ell_k = exp(N(0, 0.5^2)),
    s = 1, sigma^2 = 1e-2, b = 1024, 16 right-hand sides: y = sin(2 pi sum x / d)
    + N(0, 0.1^2) and 15 Rademacher probes; cyclic order."""
    rng = np.random.default_rng(seed)
    d = 8
    X = rng.standard_normal((n, d))
    ell = np.exp(0.5 * rng.standard_normal(d))
    y = np.sin(2 * np.pi * X.sum(1) / d) + 0.1 * rng.standard_normal(n)
    return Workload("c2" if l == 16 else f"c2_l{l}", X.astype(np.float32), _rhs(rng, y, l),
                    MATERN52, ell, 1.0, 1e-2, b=b, tol=1e-2)


def c3(seed: int = 0, n: int = 2_000_000, l: int = 32, b: int = 2048,
       noise: float = 1e-4) -> Workload:
    """Ill-conditioned case at house-electric scale: n = 2 000 000, d = 3, a
    64-component Gaussian mixture (centres U[0,1]^3, equal weights, sd 0.02,
    redrawn until inside [0,1]^3), RBF ell = 0.1, s = 1, sigma^2 = 1e-4, b = 2048,
    32 right-hand sides (y = sin(2 pi sum x) + N(0, 0.01^2) and 31 Rademacher),
    cyclic order, FP64 refinement every 5 epochs, tolerance 1e-2. `noise`
    replaces sigma^2 for the better-conditioned variant of the same inputs."""
    rng = np.random.default_rng(seed)
    d = 3
    centres = rng.uniform(0.0, 1.0, size=(64, d))
    comp = rng.integers(0, 64, size=n)
    X = centres[comp] + 0.02 * rng.standard_normal((n, d))
    bad = np.nonzero(((X < 0.0) | (X > 1.0)).any(1))[0]
    while bad.size:
        X[bad] = centres[comp[bad]] + 0.02 * rng.standard_normal((bad.size, d))
        bad = bad[((X[bad] < 0.0) | (X[bad] > 1.0)).any(1)]
    y = np.sin(2 * np.pi * X.sum(1)) + 0.01 * rng.standard_normal(n)
    name = "c3" + ("" if noise == 1e-4 else f"_noise{noise:g}") + ("" if l == 32 else f"_l{l}")
    return Workload(name, X.astype(np.float32), _rhs(rng, y, l), RBF, np.full(d, 0.1), 1.0, noise,
                    b=b, tol=1e-2, refine_every=5)


def c3_heldout(seed: int = 0, n_test: int = 100_000):
    """Held-out points of the c3(seed) mixture: the same 64 centres (that
    generator's first draw), new points and target noise from a stream of
    their own; returns (X_test as float32, y_test as float64) with
    y = sin(2 pi sum x) + N(0, 0.01^2), as for the training targets."""
    d = 3
    centres = np.random.default_rng(seed).uniform(0.0, 1.0, size=(64, d))
    rng = np.random.default_rng([seed, 7])
    comp = rng.integers(0, 64, size=n_test)
    X = centres[comp] + 0.02 * rng.standard_normal((n_test, d))
    bad = np.nonzero(((X < 0.0) | (X > 1.0)).any(1))[0]
    while bad.size:
        X[bad] = centres[comp[bad]] + 0.02 * rng.standard_normal((bad.size, d))
        bad = bad[((X[bad] < 0.0) | (X[bad] > 1.0)).any(1)]
    y = np.sin(2 * np.pi * X.sum(1)) + 0.01 * rng.standard_normal(n_test)
    return X.astype(np.float32), y


def c4(seed: int = 0, n: int = 4_000_000, l: int = 8, b: int = 2048) -> Workload:
    """Gas-sensors scale: n = 4 000 000, d = 11, 95% draws U[-1,1]^11 plus 5%
    exact copies of uniformly chosen draws, shuffled; Matern-3/2 ARD with
    ell_k = exp(N(0, 0.5^2)), s = 1, sigma^2 = 1e-3, b = 2048, 8 right-hand sides
    (y = sin(2 pi sum x / d) + N(0, 0.1^2) and 7 Rademacher), greedy order,
    exactly 20 epochs."""
    rng = np.random.default_rng(seed)
    d = 11
    n_dup = n // 20
    base = rng.uniform(-1.0, 1.0, size=(n - n_dup, d))
    dup = base[rng.integers(0, n - n_dup, size=n_dup)]
    X = np.concatenate([base, dup])[rng.permutation(n)]
    ell = np.exp(0.5 * rng.standard_normal(d))
    y = np.sin(2 * np.pi * X.sum(1) / d) + 0.1 * rng.standard_normal(n)
    return Workload("c4", X.astype(np.float32), _rhs(rng, y, l), MATERN32, ell, 1.0, 1e-3, b=b,
                    order=GREEDY, tol=0.0, min_epochs=20, max_epochs=20)


@dataclass
class Request:
    """One serving request: its arrival time and the seeded recipe of its
    problem; ``make()`` draws the arrays on demand."""
    rid: int
    arrival: float           # seconds after the stream starts
    n: int
    d: int
    kernel: int
    ell: float
    noise: float
    l: int
    b: int
    seed: int

    def make(self) -> Workload:
        sub = np.random.default_rng([self.seed, self.rid])
        X = sub.uniform(0.0, 1.0, size=(self.n, self.d))
        y = np.sin(2 * np.pi * X.sum(1) / math.sqrt(self.d)) + 0.1 * sub.standard_normal(self.n)
        return Workload(f"req{self.rid}", X.astype(np.float32), _rhs(sub, y, self.l), self.kernel,
                        np.full(self.d, self.ell), 1.0, self.noise, b=self.b, tol=1e-2)

    def footprint_points(self) -> int:
        return self.n


def serving_requests(seed: int = 0, count: int = 512, rate: float = 1.0,
                     n_min: int = 8192, n_max: int = 524288, b: int = 1024) -> list[Request]:
    """A seeded stream of solve requests with Poisson arrivals (rate per second):
    n log-uniform in [n_min, n_max], d in {3, 8, 16}, kernel in {RBF, Matern-3/2,
    Matern-5/2}, isotropic ell = sqrt(d) exp U[ln 0.1, ln 1], sigma^2 log-uniform
    in [1e-4, 1e-1], s = 1, 1..32 right-hand sides (y = sin(2 pi sum x / sqrt d)
    + N(0, 0.1^2) plus Rademacher probes), X ~ U[0,1]^d, b = 1024, cyclic."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(math.floor(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        d = int(rng.choice([3, 8, 16]))
        kern = int(rng.integers(0, 3))
        ell = math.sqrt(d) * math.exp(rng.uniform(math.log(0.1), math.log(1.0)))
        noise = math.exp(rng.uniform(math.log(1e-4), math.log(1e-1)))
        l = int(rng.integers(1, 33))
        out.append(Request(rid, t, n, d, kern, ell, noise, l, b, seed))
    return out


def small(seed: int, n: int, d: int, l: int, b: int, kernel: int = RBF, noise: float = 0.1,
          ell: float | np.ndarray = 0.5, outputscale: float = 1.0, order: int = CYCLIC,
          dist: str = "uniform") -> Workload:
    """Small seeded problem for parity and edge-case tests."""
    rng = np.random.default_rng(seed)
    if dist == "normal":
        X = rng.standard_normal((n, d))
    else:
        X = rng.uniform(0.0, 1.0, size=(n, d))
    y = np.sin(2 * np.pi * X.sum(1) / max(d, 1)) + 0.1 * rng.standard_normal(n)
    ls = np.broadcast_to(np.asarray(ell, dtype=np.float64), (d,)).copy()
    return Workload(f"small{seed}", X.astype(np.float32), _rhs(rng, y, l), kernel, ls,
                    outputscale, noise, b=b, order=order)
