"""The seeded input generators (host only): the held-out points of the n = 2M
recipe come from the same mixture as its training points."""
from __future__ import annotations

import numpy as np

from paper_2310_17137_amd import gen


def test_c3_heldout_points_share_the_training_mixture():
    w = gen.c3(n=20000, l=1)
    Xt, yt = gen.c3_heldout(n_test=500)
    X = w.X.astype(np.float64)
    # nearest training point of every held-out point: the clusters have sd 0.02
    d2 = ((Xt[:, None, :].astype(np.float64) - X[None, :, :]) ** 2).sum(-1)
    assert np.sqrt(d2.min(1)).max() < 0.1
    assert np.all((Xt >= 0.0) & (Xt <= 1.0))
    # the targets follow the training recipe: sin(2 pi sum x) + N(0, 0.01^2)
    resid = yt - np.sin(2 * np.pi * Xt.astype(np.float64).sum(1))
    assert abs(resid.std() - 0.01) < 0.002
    # a different stream from the training draws
    assert not np.any(np.all(Xt[:1] == w.X, axis=1))
