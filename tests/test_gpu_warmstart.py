"""The learned warm start judged by the plain solver: a U-Net trained on the
GPU with the library's own BF16 MFMA kernels, on steady porous-channel flows
that the solver itself generated, must bring held-out geometries to the
residual criterion (||u^n - u^(n-2)|| / (2 ||u^n||) < 1e-6) in fewer steps
and less wall-clock time, inference included, than the same solver started
from rest.  A reduced instance of the 64x64x128 study: 32x32x64 channels,
48 training samples, held-out seeds never seen in training."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DIMS = (32, 32, 64)
TRAIN = list(range(48))
TEST = list(range(900000, 900008))


@pytest.fixture(scope="module")
def trained():
    import torch
    from paper_1007_1388_amd import warmstart as ws
    t0 = time.perf_counter()
    data = ws.generate(TRAIN, concurrent=8, dims=DIMS, log=lambda m: None)
    t_gen = time.perf_counter() - t0
    steps = sorted(d["steps"] for d in data)
    tr = ws.Trainer(batch=4, dims=DIMS)
    tr.prepare(data)
    info = tr.train(data, epochs=40, lr=1e-3, log=lambda m: None)
    for d in data:
        d.clear()
    torch.cuda.synchronize()
    print("warm start: %d samples generated in %.1f s (steps to steady %s), trained in %.1f s, loss %.3e -> %.3e"
          % (len(TRAIN), t_gen, steps, info["seconds"], info["loss"][0],
             info["loss"][-1]))
    return tr, info


def test_training_reduces_the_loss(trained):
    _, info = trained
    assert np.isfinite(info["loss"]).all()
    assert info["loss"][-1] < 0.25 * info["loss"][0], info["loss"]


def test_warm_start_reaches_the_residual_faster_than_rest(trained):
    from paper_1007_1388_amd import warmstart as ws
    tr, _ = trained
    # first calls pay one-time costs (library set-up, the inference network)
    solid, gx, _ = ws.sample(TEST[0], DIMS)
    ws.solve(gx, solid, dims=DIMS, max_steps=200)
    ws.solve(gx, solid, trainer=tr, dims=DIMS, max_steps=200)
    rows = []
    for s in TEST:
        solid, gx, frac = ws.sample(s, DIMS)
        n0, t0, r0 = ws.solve(gx, solid, dims=DIMS)
        n1, t1, r1 = ws.solve(gx, solid, trainer=tr, dims=DIMS)
        assert r0 < ws.TOL and r1 < ws.TOL, (s, r0, r1)
        rows.append((n0, t0, n1, t1))
        print("seed %d (solid %.2f, g_x %.2e): from rest %d steps %.3f s, warm start %d steps %.3f s"
              % (s, frac, gx, n0, t0, n1, t1))
    n0, t0, n1, t1 = (np.array(c) for c in zip(*rows))
    print("median: from rest %d steps %.3f s, warm start %d steps %.3f s; warm faster on %d of %d"
          % (np.median(n0), np.median(t0), np.median(n1), np.median(t1), int((t1 < t0).sum()), len(rows)))
    assert np.median(n1) < np.median(n0)
    assert np.median(t1) < np.median(t0)
    assert (t1 < t0).sum() >= len(rows) * 3 // 4
