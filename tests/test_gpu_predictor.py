"""The runtime predictor trained on measured runs of the indexed k-means
(per-iteration GPU times from KM_FLAG_TIMING) and tried on held-out
workloads: its per-iteration times, and the adjustment by the asymmetric
GP once the first iterations of a task have been measured.  There are no
published predictions to compare against; the bounds here are this
library's own (per-iteration error within 35%, and the adjustment not
making the forecast of the remaining iterations worse)."""

import sys

import numpy as np
import pytest

from synth import geo_hotspots_2d, init_centroids

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(ekm, torch, n, k, seed):
    x = geo_hotspots_2d(n, seed=seed)
    c0 = init_centroids(x, k, seed + 1)
    ctx = ekm.kmeans_init(torch.from_numpy(x).cuda(), k, flags=ekm.KM_FLAG_TIMING)
    feat = ekm.kmeans_context_features(ctx)
    c = torch.from_numpy(c0).cuda()
    it, _ = ekm.kmeans_run(ctx, c, 100, stop_when_stable=True)
    per = [1e3 * sum(s.values()) for s in ekm.kmeans_step_times(ctx, cap=it)]  # us per iteration
    ctx.close()
    return [feat[0], feat[1], feat[4]], per  # ln n, ln k, ln(points per leaf)


def test_predictor_on_measured_runs():
    import torch
    import paper_2412_02244_amd as ekm
    ekm.load_library()
    train, test = [], []
    for i, (n, k) in enumerate([(n, k) for n in (200_000, 400_000, 700_000, 1_000_000) for k in (100, 300, 1000)]):
        (test if i % 4 == 3 else train).append(_run(ekm, torch, n, k, 3000 + 10 * i))
    _say(f"predictor: {len(train)} training runs, {len(test)} held out")
    p = ekm.Predictor(100, 3, order=2, sigma=4.0, noise=0.05)
    for f, per in train:
        p.add_run(f, per)
    p.fit()
    errs, before, after = [], [], []
    for f, per in test:
        v, yhat, tot = p.predict(f)
        m = len(per)
        e = [abs(yhat[j] - per[j]) / per[j] for j in range(1, m)]  # the first iteration is the odd one
        errs += e
        _say(f"  held out n=e^{f[0]:.2f} k=e^{f[1]:.2f}: iterations {m} (predicted {v}), total {sum(per):.1f} us "
             f"(predicted {tot:.1f}), per-iteration error {np.mean(e):.3f}")
        if m > 8 and v > 5:
            # remaining time after 5 measured iterations: the regressor's forecast
            # against the adjusted one (both up to the predicted iteration number)
            p.begin(f)
            for j in range(1, 6):
                rem, _ = p.observe(j, per[j - 1])
            actual_rem = sum(per[5:])
            before.append(abs(sum(yhat[5:v]) - actual_rem))
            after.append(abs(rem - actual_rem))
    mape = float(np.mean(errs))
    _say(f"predictor: per-iteration error {mape:.3f}; remaining-time error before/after adjustment "
         f"{np.mean(before) if before else 0:.1f} / {np.mean(after) if after else 0:.1f} us")
    assert np.isfinite(mape) and mape < 0.35
    if before:
        assert np.mean(after) <= 1.1 * np.mean(before) + 1e-3
