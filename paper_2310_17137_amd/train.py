"""Hyperparameter training of a GP by Adam on the stochastic gradient of the
negative log marginal likelihood (Section 2, eq. loss_grad_unbiased; Section 5,
"MLL Optimization"), with every linear solve done by alternating projection.

Each iteration:
  1. factors the diagonal blocks at the current hyperparameters theta = (the d
     lengthscales, the outputscale s, the noise sigma^2) (ap_factor_blocks, in
     one workspace reused by every iteration);
  2. solves K^_theta W = B, B = [y, z_1 .. z_P], by Algorithm 1 from the
     previous iteration's W (ap_solve_from: R = B - K^_theta W as the FP64 true
     residual; the warm start the paper's discussion suggests), the first
     iteration from W = 0;
  3. takes the gradient estimate for every component of theta (ap_mll_grad);
  4. makes one Adam step (Kingma and Ba, ICLR 2015) on log theta, with the
     paper's step size 0.1 by default.
The probes z stay the same in every iteration (the columns of B the caller
passes), and the prior mean is 0. A step's solve either runs to the stopping
rule (tol, min/max epochs, FP64 true residuals every refine_every epochs) or,
with `epochs` set, exactly that many epochs.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import ap


@dataclass
class StepRecord:
    step: int
    theta: np.ndarray        # hyperparameters the step's solve used
    grad: np.ndarray         # gradient of the negative MLL with respect to theta
    epochs: int
    rho: float               # stopping ratio at the end of the solve
    converged: bool
    t_factor: float
    t_solve: float
    t_grad: float


class Trainer:
    def __init__(self, X, B, *, kernel: int, lengthscale, outputscale: float, noise: float,
                 b: int, order: int = ap.CYCLIC, tile: int = ap.TILE_FP64, lr: float = 0.1,
                 epochs: int | None = None, tol: float = 1e-2, max_epochs: int = 1000,
                 refine_every: int = 5, warm: bool = True, betas=(0.9, 0.999),
                 eps: float = 1e-8, seed: int = 0):
        import torch
        self.torch = torch
        self.X, self.B = X, B
        self.n, self.d = int(X.shape[0]), int(X.shape[1])
        self.l = int(B.shape[1])
        self.kernel, self.b, self.order, self.tile = int(kernel), int(b), int(order), int(tile)
        ell = np.broadcast_to(np.asarray(lengthscale, dtype=np.float64), (self.d,))
        theta = np.concatenate([ell, [float(outputscale), float(noise)]])
        if not np.all(theta > 0):
            raise ValueError("lengthscales, outputscale and noise must be positive")
        self.phi = np.log(theta)             # Adam runs on log theta
        self.lr, self.beta1, self.beta2, self.eps = float(lr), betas[0], betas[1], float(eps)
        self.m1 = np.zeros_like(self.phi)
        self.m2 = np.zeros_like(self.phi)
        self.t = 0
        self.warm = bool(warm)
        if epochs is not None:
            # exactly `epochs` epochs: no tolerance stop, no true-residual holds
            self.solve_kw = dict(tol=0.0, min_epochs=int(epochs), max_epochs=int(epochs),
                                 refine_every=0)
        else:
            self.solve_kw = dict(tol=float(tol), min_epochs=0, max_epochs=int(max_epochs),
                                 refine_every=int(refine_every))
        self.seed = int(seed)
        need = ap.workspace_bytes(n=self.n, d=self.d, l=self.l, b=self.b, kernel=self.kernel,
                                  lengthscale=1.0, tile=self.tile)
        if need == 0:
            raise ValueError("these sizes are outside the library's limits")
        self.ws = torch.empty(need + 256, dtype=torch.uint8, device=X.device)
        self.W = torch.zeros((self.n, self.l), dtype=torch.float64, device=X.device)
        self.R = torch.empty((self.n, self.l), dtype=torch.float32, device=X.device)
        self.solver = None
        self.history: list[StepRecord] = []

    @property
    def theta(self) -> np.ndarray:
        return np.exp(self.phi)

    def step(self) -> StepRecord:
        theta = self.theta
        d = self.d
        t0 = time.perf_counter()
        self.solver = None  # the previous handle; its work is ordered before the next
        self.solver = ap.Solver(self.X, l=self.l, b=self.b, kernel=self.kernel,
                                lengthscale=theta[:d], outputscale=theta[d], noise=theta[d + 1],
                                order=self.order, tile=self.tile, seed=self.seed,
                                workspace=self.ws, **self.solve_kw)
        t1 = time.perf_counter()
        warm = self.warm and self.t > 0
        st = self.solver.solve(self.B, self.W, self.R, warm=warm)
        t2 = time.perf_counter()
        grad = self.solver.mll_grad(self.B, self.W, self.R)
        t3 = time.perf_counter()
        # Adam on phi = log theta: d loss / d phi = theta * d loss / d theta
        self.t += 1
        g = grad * theta
        self.m1 = self.beta1 * self.m1 + (1.0 - self.beta1) * g
        self.m2 = self.beta2 * self.m2 + (1.0 - self.beta2) * g * g
        mhat = self.m1 / (1.0 - self.beta1 ** self.t)
        vhat = self.m2 / (1.0 - self.beta2 ** self.t)
        self.phi = self.phi - self.lr * mhat / (np.sqrt(vhat) + self.eps)
        rec = StepRecord(self.t, theta, np.asarray(grad, dtype=np.float64), st.epochs,
                         st.rho_true if math.isfinite(st.rho_true) else st.rho_maintained,
                         st.converged, t1 - t0, t2 - t1, t3 - t2)
        self.history.append(rec)
        return rec
