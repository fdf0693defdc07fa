"""Continuous-batching request loop for GP solves on one GPU.

Requests (features X, right-hand sides B, kernel hyperparameters) arrive over
time. The server admits a request as soon as it has arrived, a slot is free and
its HBM footprint (the solver's workspace from ap_workspace_bytes, which holds
the cached FP64 block inverses, plus X, B, W and R) fits the budget; admission
uploads the request and builds its block factors on a stream of its own. Every
admitted request stays resident, and all of them advance together in batch
steps (ap_batch_step): each step is one grouped launch of the block solves of
every active request, one grouped launch of their fused K-tile updates and one
that advances their epoch state on the device, so requests of different n, d,
l and hyperparameters share every launch and the device never waits for the
host between steps. A request's epoch-end check runs on the device and holds
the request when the host has to act: every refine_every epochs and when the
maintained ratio is below the tolerance, the host replaces R by the FP64 true
residual (Lemma residual_equality) and tests it (the interval doubles, up to
16 refine_every, while the two ratios agree to 1e-5); the request finishes when that
ratio is below the tolerance or at max_epochs, moves to FP64 tiles when the
true and maintained ratios differ by more than 5%, and restarts on FP64 tiles
if its norms were not finite.

A request's arithmetic depends only on its own inputs and these decisions,
never on what else is active or on when the host acted, so its result is
bitwise the same alone and in a mix.
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
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Active:
    def __init__(self, req, w, solver, X, B, W, R, admitted, fp, tile):
        self.req, self.w, self.solver = req, w, solver
        self.X, self.B, self.W, self.R = X, B, W, R
        self.admitted, self.fp, self.tile = admitted, fp, tile
        self.hold = ap.RUN          # state being handled
        self.refine_event = None    # FP64 true residual in flight
        self.interval = 0           # epochs between true-residual holds (0: none)
        # release (or reset) in flight: until it has run, the device still
        # shows the old held state, which must not be acted on again
        self.resume_event = None

    def state(self):
        return (self.B, self.W, self.R)


class Server:
    def __init__(self, budget_bytes: float = 200e9, max_active: int = 16,
                 tile: int = ap.TILE_SPLIT, refine_every: int = 5, steps_per_call: int = 4,
                 max_epochs: int = 1000, tol: float = 1e-2, keep_w: bool = False,
                 order: int | None = None, device: str = "cuda"):
        import torch
        self.torch = torch
        self.budget = float(budget_bytes)
        self.max_active = int(max_active)
        if not 1 <= self.max_active <= 32:
            raise ValueError("max_active must be in 1..32 (one batch step serves at most 32)")
        self.tile = int(tile)
        self.refine_every = int(refine_every)
        self.steps = int(steps_per_call)
        self.max_epochs = int(max_epochs)
        self.tol = float(tol)
        self.keep_w = keep_w
        self.order = order  # block selection for every request (None: the request's own)
        self.device = torch.device(device)
        self.peak_bytes = 0
        self.peak_active = 0
        self.batch_steps = 0

    # -- request lifecycle ------------------------------------------------------
    def _admit(self, req, now: float, adm, main) -> _Active:
        torch = self.torch
        w = req.make()
        with torch.cuda.stream(adm):
            X = torch.from_numpy(w.X).to(self.device, non_blocking=False)
            B = torch.from_numpy(w.B).to(self.device, non_blocking=False)
            s = ap.Solver(X, l=w.l, b=w.b, kernel=w.kernel, lengthscale=w.lengthscale,
                          outputscale=w.outputscale, noise=w.noise,
                          order=w.order if self.order is None else self.order,
                          seed=req.rid,  # random order's draws
                          tile=self.tile, refine_every=self.refine_every, tol=self.tol,
                          max_epochs=self.max_epochs, stream=adm)  # factors, syncs `adm`
            W, R = s.new_state(B)
        adm.synchronize()
        s.reset(B, W, R, stream=main)
        fp = footprint_bytes(w.n, w.d, w.l, w.b, w.kernel, self.tile)
        a = _Active(req, w, s, X, B, W, R, now, fp, self.tile)
        a.interval = self.refine_every
        return a

    def _on_hold(self, a: _Active, pr, main):
        """`a` was seen held (state pr.state): start the host's action."""
        torch = self.torch
        a.hold = pr.state
        if pr.state == ap.HOLD_NONFINITE:
            return  # handled in _decide without a true residual
        a.solver.residual(a.B, a.W, a.R, want_col_rel=False, stream=main)  # R <- B - K^ W
        a.refine_event = torch.cuda.Event()
        a.refine_event.record(main)

    def _decide(self, a: _Active, main):
        """The host's action on held `a` is complete. Returns (finished,
        converged, rho_true, epochs). The problem is held and everything queued
        before this point has completed, so the snapshot is exact."""
        pr = a.solver.peek()
        if a.hold == ap.HOLD_NONFINITE:
            if a.tile == ap.TILE_FP64:
                return True, False, math.nan, pr.epoch
            # reduced-precision tiles overflowed: restart (W = 0, R = B) on FP64 tiles
            a.solver.set_tile(ap.TILE_FP64)
            a.tile = ap.TILE_FP64
            a.solver.reset(a.B, a.W, a.R, stream=main)
            self._resumed(a, main)
            return False, False, math.nan, pr.epoch
        rho_t = pr.rho_true
        a.refine_event = None
        if not math.isfinite(rho_t):
            return True, False, rho_t, pr.epoch
        if rho_t < self.tol:
            return True, True, rho_t, pr.epoch
        if a.hold == ap.HOLD_MAX:
            return True, False, rho_t, pr.epoch
        drift = abs(rho_t - pr.rho) / rho_t
        if a.tile != ap.TILE_FP64 and drift > 0.05:
            a.solver.set_tile(ap.TILE_FP64)
            a.tile = ap.TILE_FP64
        if a.interval > 0:
            # the true residual costs about as much as a few epochs: while the
            # maintained residual shows no drift, check less often
            if a.hold == ap.HOLD_REFINE:
                a.interval = (min(2 * a.interval, 16 * self.refine_every) if drift < 1e-5
                              else self.refine_every)
            nxt = pr.epoch + a.interval
        else:
            nxt = 0
        a.solver.release(next_refine=nxt, stream=main)
        self._resumed(a, main)
        return False, False, rho_t, pr.epoch

    def _resumed(self, a: _Active, main):
        a.hold = ap.RUN
        a.resume_event = self.torch.cuda.Event()
        a.resume_event.record(main)

    # -- the loop ---------------------------------------------------------------
    def run(self, requests, time_scale: float = 1.0, log=None) -> list[Done]:
        """Serve `requests` (gen.Request, arrival in seconds; divided by
        time_scale) in real time. Returns one record per request."""
        torch = self.torch
        main = torch.cuda.Stream(device=self.device)   # batch steps (default priority)
        adm = torch.cuda.Stream(device=self.device)    # admission: upload and factor
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        active: list[_Active] = []
        done: list[Done] = []
        inflight: collections.deque = collections.deque()
        retiring: list = []   # (buffers, event): freed once the batch stream passed them
        used = 0
        t0 = time.perf_counter()
        next_report = 20.0
        while pending or active:
            now = time.perf_counter() - t0
            if log and now >= next_report:
                next_report += 20.0
                log(f"[serve] t={now:.0f} s: {len(done)} done, {len(active)} active, "
                    f"{len(pending)} pending, {self.batch_steps} batch steps")
            # admission
            while (pending and pending[0].arrival / time_scale <= now
                   and len(active) < self.max_active):
                req = pending[0]
                fp = footprint_bytes(req.n, req.d, req.l, req.b, req.kernel, self.tile)
                if used + fp > self.budget:
                    if not active:
                        raise RuntimeError(f"request {req.rid} alone exceeds the HBM budget")
                    break
                pending.popleft()
                if log:
                    log(f"[serve] admit req {req.rid} n={req.n} d={req.d} l={req.l} "
                        f"kernel={req.kernel} noise={req.noise:.3g}")
                t_adm = time.perf_counter() - t0
                try:
                    a = self._admit(req, t_adm, adm, main)
                except ap.ApError as e:
                    # a request the library rejects (e.g. a block that is not
                    # positive definite) fails alone; the others go on
                    done.append(Done(req.rid, req.n, req.d, req.l, req.kernel,
                                     req.arrival / time_scale, t_adm, time.perf_counter() - t0,
                                     0, math.nan, False, self.tile, fp, None, str(e)))
                    if log:
                        log(f"[serve] req {req.rid} rejected: {e}")
                    continue
                active.append(a)
                used += fp
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_active = max(self.peak_active, len(active))
            # keep two batch calls queued ahead of the host
            if active and len(inflight) < 2:
                ap.batch_step([a.solver for a in active], [a.state() for a in active],
                              self.steps, stream=main)
                self.batch_steps += self.steps
                ev = torch.cuda.Event()
                ev.record(main)
                inflight.append(ev)
            progressed = False
            if inflight and inflight[0].query():
                inflight.popleft()
                progressed = True
                for a in active:
                    if a.resume_event is not None:
                        if not a.resume_event.query():
                            continue
                        a.resume_event = None
                    if a.hold == ap.RUN:
                        pr = a.solver.peek()
                        if pr.state != ap.RUN:
                            self._on_hold(a, pr, main)
            for a in list(active):
                if a.hold == ap.RUN:
                    continue
                if a.refine_event is not None and not a.refine_event.query():
                    continue
                progressed = True
                fin, conv, rho_t, epochs = self._decide(a, main)
                if not fin:
                    continue
                t = time.perf_counter() - t0
                W = a.W.cpu().numpy() if self.keep_w else None
                rec = Done(a.req.rid, a.w.n, a.w.d, a.w.l, a.w.kernel, a.req.arrival / time_scale,
                           a.admitted, t, epochs, rho_t, conv, a.tile, a.fp, W)
                done.append(rec)
                if log:
                    log(f"[serve] req {rec.rid} n={rec.n} d={rec.d} l={rec.l} done: "
                        f"{rec.epochs} epochs, rho_true {rec.rho_true:.3e}, latency "
                        f"{rec.latency:.3f} s, tile {rec.tile}")
                active.remove(a)
                used -= a.fp
                ev = torch.cuda.Event()
                ev.record(main)
                retiring.append((a, ev))
            retiring = [(a, ev) for a, ev in retiring if not ev.query()]
            if not progressed:
                if active:
                    time.sleep(50e-6)
                elif pending:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival / time_scale - now)))
        torch.cuda.synchronize()
        return done


def summarize(done: list[Done], wall: float) -> dict:
    """Latency percentiles over the requests that were served (rejected ones
    are counted in "failed"); throughput over the wall time of the run."""
    lat = np.array([d.latency for d in done if not d.error] or [math.nan])
    n2 = sum(d.n * d.n * d.epochs for d in done)
    return {
        "requests": len(done),
        "converged": int(sum(d.converged for d in done)),
        "failed": int(sum(bool(d.error) for d in done)),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "throughput_req_per_s": sum(not d.error for d in done) / wall,
        "kernel_entries_per_s": n2 / wall,
        "epochs_total": int(sum(d.epochs for d in done)),
        "escalated_to_fp64": int(sum(d.tile == ap.TILE_FP64 for d in done)),
        "wall_s": wall,
    }


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--count", type=int, default=512)
    p.add_argument("--rate", type=float, default=1.0, help="arrivals per second")
    p.add_argument("--sweep", default="",
                   help="comma-separated multiples of the measured capacity (e.g. 0.5,1,2): "
                        "first serve every request at t = 0 to measure capacity (requests/s), "
                        "then replay the Poisson stream at each multiple ('sat': capacity only)")
    p.add_argument("--n-min", type=int, default=8192)
    p.add_argument("--n-max", type=int, default=524288)
    p.add_argument("--max-epochs", type=int, default=1000)
    p.add_argument("--max-active", type=int, default=16)
    p.add_argument("--budget-gb", type=float, default=200.0)
    p.add_argument("--tile", default="split", choices=["split", "fp32", "fp64", "bf16"])
    p.add_argument("--refine-every", type=int, default=5)
    p.add_argument("--order", default="request", choices=["request", "cyclic", "greedy", "random"],
                   help="block selection (request: each request's own)")
    p.add_argument("--steps-per-call", type=int, default=4,
                   help="batch steps enqueued per ap_batch_step call")
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--quiet", action="store_true", help="no per-request log lines")
    p.add_argument("--records", default="", help="write every request's record (JSON lines) here")
    a = p.parse_args(argv)
    tile = {"split": ap.TILE_SPLIT, "fp32": ap.TILE_FP32, "fp64": ap.TILE_FP64,
            "bf16": ap.TILE_BF16}[a.tile]
    log = None if a.quiet else (lambda m: print(m, file=sys.stderr, flush=True))
    ap.load()

    def serve_once(reqs, label, rate):
        srv = Server(budget_bytes=a.budget_gb * 1e9, max_active=a.max_active, tile=tile,
                     refine_every=a.refine_every, max_epochs=a.max_epochs,
                     steps_per_call=a.steps_per_call,
                     order={"request": None, "cyclic": gen.CYCLIC, "greedy": gen.GREEDY,
                            "random": gen.RANDOM}[a.order])
        t = time.perf_counter()
        done = srv.run(reqs, log=log)
        out = summarize(done, time.perf_counter() - t)
        if a.records:
            with open(a.records, "a") as fh:
                for d in done:
                    rec = {k: v for k, v in d.__dict__.items() if k != "W"}
                    rec.update({"run": label, "latency": d.latency})
                    fh.write(json.dumps(rec) + "\n")
        out.update({"run": label, "rate": rate, "peak_active": srv.peak_active,
                    "peak_gb": srv.peak_bytes / 1e9, "count": a.count, "n_min": a.n_min,
                    "n_max": a.n_max, "max_epochs": a.max_epochs, "tile": a.tile,
                    "order": a.order,
                    "batch_steps": srv.batch_steps})
        print(json.dumps(out), flush=True)
        return out

    if not a.sweep:
        reqs = gen.serving_requests(seed=a.seed, count=a.count, rate=a.rate, n_min=a.n_min,
                                    n_max=a.n_max)
        serve_once(reqs, "poisson", a.rate)
        return
    # capacity: the whole stream queued at t = 0 (slots and HBM still limit admission)
    unit = gen.serving_requests(seed=a.seed, count=a.count, rate=1.0, n_min=a.n_min,
                                n_max=a.n_max)
    import dataclasses
    sat = serve_once([dataclasses.replace(r, arrival=0.0) for r in unit], "saturation", None)
    cap = sat["throughput_req_per_s"]
    for mult in (float(x) for x in a.sweep.split(",") if x != "sat"):
        rate = mult * cap
        # the same requests; arrival times of a rate-1 Poisson stream divided by the rate
        reqs = [dataclasses.replace(r, arrival=r.arrival / rate) for r in unit]
        serve_once(reqs, f"poisson {mult:g}x capacity", rate)
    if ap.last_error():
        print(f"[serve] library note: {ap.last_error()}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
