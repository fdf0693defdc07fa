"""The continuous-batching request loop on the GPU: results alone and in a mix
are bitwise equal, admission respects the HBM budget, a request arriving while
others run is admitted and can finish first, and served results solve their
systems (checked with the FP64 oracle on sampled rows)."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import apo
from paper_2310_17137_amd import gen
from tests.helpers import to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2310_17137_amd import ap, serve  # noqa: E402


def _requests(count=5, seed=3):
    reqs = gen.serving_requests(seed=seed, count=count, rate=50.0, n_min=2048, n_max=8192,
                                b=512)
    print("[serve-case] " + " ".join(f"(n={r.n} d={r.d} l={r.l} k={r.kernel})" for r in reqs),
          flush=True)
    return reqs


def test_results_alone_equal_results_in_mix():
    reqs = _requests()
    alone = {}
    for r in reqs:
        srv = serve.Server(max_active=1, max_epochs=12, refine_every=4, keep_w=True)
        (d,) = srv.run([dataclasses.replace(r, arrival=0.0)])
        alone[r.rid] = d
    srv = serve.Server(max_active=5, max_epochs=12, refine_every=4, keep_w=True)
    mixed = srv.run([dataclasses.replace(r, arrival=0.002 * i) for i, r in enumerate(reqs)])
    assert srv.peak_active >= 2  # their work overlapped
    for d in mixed:
        a = alone[d.rid]
        assert d.epochs == a.epochs and d.tile == a.tile
        assert np.array_equal(d.W, a.W), d.rid


def test_admission_respects_budget_and_slots():
    reqs = _requests(count=6, seed=4)
    fps = [serve.footprint_bytes(r.n, r.d, r.l, r.b, r.kernel, ap.TILE_SPLIT) for r in reqs]
    budget = sorted(fps)[-1] + sorted(fps)[-2] + 1
    srv = serve.Server(budget_bytes=budget, max_active=4, max_epochs=6, refine_every=3)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert srv.peak_bytes <= budget
    assert srv.peak_active <= 4


def test_late_short_request_finishes_before_long_one():
    long_req = gen.Request(0, 0.0, 60000, 3, gen.RBF, 0.3, 1e-2, 8, 1024, seed=9)
    short_req = gen.Request(1, 0.05, 2048, 3, gen.RBF, 0.1, 1e-1, 2, 512, seed=9)
    srv = serve.Server(max_active=4, max_epochs=40, refine_every=10)
    done = {d.rid: d for d in srv.run([long_req, short_req])}
    assert done[1].admitted < done[0].finished  # admitted while the long one ran
    assert done[1].finished < done[0].finished


def test_served_results_solve_their_systems():
    reqs = [gen.Request(0, 0.0, 4096, 3, gen.RBF, 0.05, 0.1, 4, 512, seed=5),
            gen.Request(1, 0.0, 3000, 8, gen.MATERN52, 0.3, 0.1, 3, 512, seed=5)]
    srv = serve.Server(max_active=2, max_epochs=300, refine_every=5, keep_w=True)
    for d in srv.run(reqs):
        w = reqs[d.rid].make()
        p = to_oracle(w)
        rows = np.arange(0, w.n, 17)
        true = apo.residual_rows(p, d.W, rows)
        ratio = np.mean(np.linalg.norm(true, axis=0) / np.linalg.norm(p.B[rows], axis=0))
        print(f"[served] req {d.rid}: converged {d.converged} in {d.epochs} epochs, "
              f"rho_true {d.rho_true:.3e}, sampled oracle ratio {ratio:.3e}", flush=True)
        assert d.converged and d.rho_true < 1e-2
        assert ratio < 2e-2
