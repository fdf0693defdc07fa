"""Continuous-batching request loop for GP solves on one GPU.

Requests (features X, right-hand sides B, kernel hyperparameters) arrive over
time. The server admits a request as soon as it has arrived, a slot is free and
its HBM footprint (the solver's workspace from ap_workspace_bytes, which holds
the cached FP64 block inverses, plus X, B, W and R) fits the budget. Each
admitted request owns a HIP stream and stays resident; the loop keeps every
active request's next epochs queued on its own stream, so the work of requests
of different n, d, l and hyperparameters overlaps on the device, and it admits
newcomers as slots and memory free up. Each epoch is the library's captured
graph of Algorithm 1 block updates. A request finishes when the FP64 true
residual (Lemma residual_equality) confirms the mean column ratio is below its
tolerance, or at max_epochs. The FP64 true residual also runs every
refine_every epochs; when it and the maintained residual disagree by more than
5% the request continues on FP64 tiles.

A request's arithmetic depends only on its own inputs and the loop's fixed
check schedule, never on what else is active, so its result is bitwise the same
alone and in a mix.
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import ap, gen


def footprint_bytes(n: int, d: int, l: int, b: int, kernel: int, tile: int) -> int:
    ws = ap.workspace_bytes(n=n, d=d, l=l, b=b, kernel=kernel, lengthscale=1.0, tile=tile)
    return ws + 256 + n * d * 4 + n * l * (4 + 8 + 4)


@dataclass
class Done:
    rid: int
    n: int
    d: int
    l: int
    kernel: int
    arrival: float
    admitted: float
    finished: float
    epochs: int
    rho_true: float
    converged: bool
    tile: int
    footprint: int
    W: object = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Active:
    def __init__(self, req, w, solver, X, B, W, R, stream, admitted, fp, tile):
        self.req, self.w, self.solver = req, w, solver
        self.X, self.B, self.W, self.R = X, B, W, R
        self.stream, self.admitted, self.fp = stream, admitted, fp
        self.epochs = 0
        self.event = None
        self.tile = tile
        self.refines = 0


class Server:
    def __init__(self, budget_bytes: float = 200e9, max_active: int = 16,
                 tile: int = ap.TILE_SPLIT, refine_every: int = 5, epochs_per_step: int = 1,
                 max_epochs: int = 1000, tol: float = 1e-2, keep_w: bool = False,
                 device: str = "cuda"):
        import torch
        self.torch = torch
        self.budget = float(budget_bytes)
        self.max_active = int(max_active)
        self.tile = int(tile)
        self.refine_every = int(refine_every)
        self.k = int(epochs_per_step)
        self.max_epochs = int(max_epochs)
        self.tol = float(tol)
        self.keep_w = keep_w
        self.device = torch.device(device)
        self.peak_bytes = 0
        self.peak_active = 0

    # -- request lifecycle ------------------------------------------------------
    def _admit(self, req, now: float) -> _Active:
        torch = self.torch
        w = req.make()
        stream = torch.cuda.Stream(device=self.device)  # default priority
        with torch.cuda.stream(stream):
            X = torch.from_numpy(w.X).to(self.device, non_blocking=False)
            B = torch.from_numpy(w.B).to(self.device, non_blocking=False)
            s = ap.Solver(X, l=w.l, b=w.b, kernel=w.kernel, lengthscale=w.lengthscale,
                          outputscale=w.outputscale, noise=w.noise, order=w.order,
                          tile=self.tile, refine_every=self.refine_every, tol=self.tol,
                          max_epochs=self.max_epochs, stream=stream)
            W, R = s.new_state(B)
            s.reset(B, W, R, stream=stream)
        fp = footprint_bytes(w.n, w.d, w.l, w.b, w.kernel, self.tile)
        a = _Active(req, w, s, X, B, W, R, stream, now, fp, self.tile)
        self._enqueue(a)
        return a

    def _enqueue(self, a: _Active):
        torch = self.torch
        a.solver.epoch(a.B, a.W, a.R, self.k, stream=a.stream)
        a.event = torch.cuda.Event()
        a.event.record(a.stream)

    def _true_rho(self, a: _Active) -> float:
        cols = a.solver.residual(a.B, a.W, a.R, stream=a.stream)  # refines R in place
        a.refines += 1
        return float(np.mean(cols))

    def _advance(self, a: _Active) -> tuple[bool, float, bool]:
        """The step queued for `a` has completed: check and decide. Returns
        (finished, rho_true, converged)."""
        a.epochs += self.k
        try:
            rho, _ = a.solver.rel_residual(stream=a.stream)
        except ap.ApError:
            rho = math.nan
        if not math.isfinite(rho) and a.tile != ap.TILE_FP64:
            # reduced-precision tiles overflowed: restart this request on FP64 tiles
            a.solver.set_tile(ap.TILE_FP64)
            a.tile = ap.TILE_FP64
            a.solver.reset(a.B, a.W, a.R, stream=a.stream)
            return False, math.nan, False
        scheduled = self.refine_every > 0 and a.epochs % self.refine_every == 0
        if scheduled or rho < self.tol or a.epochs >= self.max_epochs:
            rho_t = self._true_rho(a)
            if a.tile != ap.TILE_FP64 and abs(rho_t - rho) > 0.05 * rho_t:
                a.solver.set_tile(ap.TILE_FP64)
                a.tile = ap.TILE_FP64
            if rho_t < self.tol:
                return True, rho_t, True
            if a.epochs >= self.max_epochs:
                return True, rho_t, False
        return False, math.nan, False

    # -- the loop ---------------------------------------------------------------
    def run(self, requests, time_scale: float = 1.0, log=None) -> list[Done]:
        """Serve `requests` (gen.Request, arrival in seconds; divided by
        time_scale) in real time. Returns one record per request."""
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        active: list[_Active] = []
        done: list[Done] = []
        used = 0
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            while (pending and pending[0].arrival / time_scale <= now
                   and len(active) < self.max_active):
                req = pending[0]
                fp = footprint_bytes(req.n, req.d, req.l, req.b, req.kernel, self.tile)
                if used + fp > self.budget:
                    if not active:
                        raise RuntimeError(f"request {req.rid} alone exceeds the HBM budget")
                    break
                pending.popleft()
                a = self._admit(req, time.perf_counter() - t0)
                active.append(a)
                used += fp
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_active = max(self.peak_active, len(active))
            progressed = False
            for a in list(active):
                if not a.event.query():
                    continue
                progressed = True
                fin, rho_t, conv = self._advance(a)
                if fin:
                    t = time.perf_counter() - t0
                    rec = Done(a.req.rid, a.w.n, a.w.d, a.w.l, a.w.kernel, a.req.arrival / time_scale,
                               a.admitted, t, a.epochs, rho_t, conv, a.tile, a.fp,
                               a.W.cpu().numpy() if self.keep_w else None)
                    done.append(rec)
                    if log:
                        log(f"[serve] req {rec.rid} n={rec.n} d={rec.d} l={rec.l} done: "
                            f"{rec.epochs} epochs, rho_true {rec.rho_true:.3e}, latency "
                            f"{rec.latency:.3f} s, tile {rec.tile}")
                    active.remove(a)
                    used -= a.fp
                    del a
                else:
                    self._enqueue(a)
            if not progressed:
                if active:
                    # poll: whichever request's step completes first advances next
                    time.sleep(50e-6)
                elif pending:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival / time_scale - now)))
        torch.cuda.synchronize()
        return done


def summarize(done: list[Done], wall: float) -> dict:
    lat = np.array([d.latency for d in done])
    n2 = sum(d.n * d.n * d.epochs for d in done)
    return {
        "requests": len(done),
        "converged": int(sum(d.converged for d in done)),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "throughput_req_per_s": len(done) / wall,
        "kernel_entries_per_s": n2 / wall,
        "epochs_total": int(sum(d.epochs for d in done)),
        "escalated_to_fp64": int(sum(d.tile == ap.TILE_FP64 for d in done)),
        "wall_s": wall,
    }


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--count", type=int, default=512)
    p.add_argument("--rate", type=float, default=1.0, help="arrivals per second")
    p.add_argument("--n-min", type=int, default=8192)
    p.add_argument("--n-max", type=int, default=524288)
    p.add_argument("--max-epochs", type=int, default=1000)
    p.add_argument("--max-active", type=int, default=16)
    p.add_argument("--budget-gb", type=float, default=200.0)
    p.add_argument("--tile", default="split", choices=["split", "fp32", "fp64", "bf16"])
    p.add_argument("--refine-every", type=int, default=5)
    p.add_argument("--seed", type=int, default=0)
    a = p.parse_args(argv)
    tile = {"split": ap.TILE_SPLIT, "fp32": ap.TILE_FP32, "fp64": ap.TILE_FP64,
            "bf16": ap.TILE_BF16}[a.tile]
    reqs = gen.serving_requests(seed=a.seed, count=a.count, rate=a.rate, n_min=a.n_min,
                                n_max=a.n_max)
    srv = Server(budget_bytes=a.budget_gb * 1e9, max_active=a.max_active, tile=tile,
                 refine_every=a.refine_every, max_epochs=a.max_epochs)
    t = time.perf_counter()
    done = srv.run(reqs, log=lambda m: print(m, file=sys.stderr, flush=True))
    out = summarize(done, time.perf_counter() - t)
    out.update({"rate": a.rate, "peak_active": srv.peak_active, "peak_gb": srv.peak_bytes / 1e9})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
