"""GPU parity of many clouds in one context (kmeans_init_batched /
kmeans_run_batched) against the oracle run on each cloud alone.

* 64 uneven 3D clouds (the batched generator with smaller sizes): every
  cloud's assignment (cloud-local ids) and centroids at every iteration of
  30, bit for bit, and kmeans_run_batched with tuned leaf size and list
  length ends where the stepped context does.
* The full batched workload (4096 clouds, sizes log-uniform in [1e3, 1e5],
  k_i = n_i / 100, 30 iterations): kmeans_run_batched's result equals a
  context run for 29 steps plus one step; that last step's assignment of
  200,000 sampled points equals the oracle's argmin against the centroids it
  started from, its centroids equal the oracle's update of every cloud, and
  14 whole clouds (the smallest, the largest and 12 evenly spaced) follow
  the oracle's 30-iteration trajectory exactly.
* Rejected inputs: a cloud with k_b > n_b, several clouds on the brute path.
"""

import sys

import numpy as np
import pytest

import oracle
from synth import batched_clouds

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ekm():
    import torch
    import paper_2412_02244_amd as m
    m.load_library()
    assert torch.cuda.is_available()
    return m


def _cloud(x, c, po, co, b):
    return x[po[b]:po[b + 1]], c[co[b]:co[b + 1]]


def test_batched_64_clouds_every_iteration(ekm):
    import torch
    dev = torch.device("cuda:0")
    x, po, c0, co = batched_clouds(n_clouds=64, seed=1103, n_range=(1_000, 20_000), init_seed=2103)
    B = len(po) - 1
    _say(f"batched 64: {x.shape[0]} points, {c0.shape[0]} centroids")
    refs = [oracle.lloyd(*_cloud(x, c0, po, co, b), max_iter=30) for b in range(B)]
    xt = torch.from_numpy(x).to(dev)
    ctx = ekm.kmeans_init_batched(xt, po, co)
    c = torch.from_numpy(c0).to(dev)
    a = torch.empty(x.shape[0], dtype=torch.int32, device=dev)
    for t in range(30):
        c, st = ekm.kmeans_step(ctx, c, torch.empty_like(c), assign_out=a, stats=True)
        ah, ch = a.cpu().numpy(), c.cpu().numpy()
        changed = 0
        for b in range(B):
            ra, rc = refs[b]["a_hist"][t], refs[b]["c_hist"][t]
            bad = np.flatnonzero(ah[po[b]:po[b + 1]] != ra)
            assert bad.size == 0, f"cloud {b} step {t + 1}: {bad.size} assignments differ, first at {bad[:5]}"
            np.testing.assert_array_equal(ch[co[b]:co[b + 1]], rc, err_msg=f"cloud {b} step {t + 1}")
            changed += ra.size if t == 0 else int((ra != refs[b]["a_hist"][t - 1]).sum())
        assert st["n_changed"] == changed, (t, st["n_changed"], changed)
    ctx.close()
    cr = torch.from_numpy(c0).to(dev)
    ar = torch.empty_like(a)
    f, G = ekm.kmeans_run_batched(xt, po, cr, co, 30, assign_out=ar)
    _say(f"batched 64: tuned leaf size {f}, leaves per list {G}")
    assert f in (16, 32, 64) and G in (4, 6, 8)
    np.testing.assert_array_equal(ar.cpu().numpy(), ah)
    np.testing.assert_array_equal(cr.cpu().numpy(), ch)


def test_batched_full_workload_sampled(ekm):
    import torch
    dev = torch.device("cuda:0")
    _say("batched 4096: generating")
    x, po, c0, co = batched_clouds()
    B = len(po) - 1
    sizes = po[1:] - po[:-1]
    _say(f"batched 4096: {x.shape[0]} points, {c0.shape[0]} centroids")
    xt = torch.from_numpy(x).to(dev)
    c_run = torch.from_numpy(c0).to(dev)
    a_run = torch.empty(x.shape[0], dtype=torch.int32, device=dev)
    f, G = ekm.kmeans_run_batched(xt, po, c_run, co, 30, assign_out=a_run)
    _say(f"batched 4096: kmeans_run_batched done, leaf size {f}, leaves per list {G}")

    ctx = ekm.kmeans_init_batched(xt, po, co, leaf_size=f, cand_tile=G)
    c29 = torch.from_numpy(c0).to(dev)
    it, _ = ekm.kmeans_run(ctx, c29, 29)
    assert it == 29
    a30 = torch.empty_like(a_run)
    c30 = ekm.kmeans_step(ctx, c29, torch.empty_like(c29), assign_out=a30)
    ctx.close()
    a30, c30, c29 = a30.cpu().numpy(), c30.cpu().numpy(), c29.cpu().numpy()
    np.testing.assert_array_equal(a_run.cpu().numpy(), a30)
    np.testing.assert_array_equal(c_run.cpu().numpy(), c30)
    _say("batched 4096: run and stepped context agree")

    # sampled points: the oracle's argmin against their cloud's centroids
    rng = np.random.default_rng(77)
    idx = np.sort(rng.choice(x.shape[0], 200_000, replace=False))
    cl = np.searchsorted(po, idx, side="right") - 1
    for b in np.unique(cl):
        sel = idx[cl == b]
        want, _ = oracle.assign(x[sel], c29[co[b]:co[b + 1]])
        np.testing.assert_array_equal(a30[sel], want, err_msg=f"cloud {b}: sampled points")
    _say("batched 4096: sampled assignments equal the oracle's")

    # every cloud's update from the last assignment
    for b in range(B):
        xb, cb = _cloud(x, c29, po, co, b)
        want, _ = oracle.update(xb, a30[po[b]:po[b + 1]], cb)
        np.testing.assert_array_equal(c30[co[b]:co[b + 1]], want, err_msg=f"cloud {b}: update")
    _say("batched 4096: every cloud's update equals the oracle's")

    # whole trajectories of a few clouds
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))} | {int(i * B // 12) for i in range(12)})
    for b in pick:
        ref = oracle.lloyd(*_cloud(x, c0, po, co, b), max_iter=30, history=False)
        np.testing.assert_array_equal(a30[po[b]:po[b + 1]], ref["a"], err_msg=f"cloud {b}")
        np.testing.assert_array_equal(c30[co[b]:co[b + 1]], ref["c"], err_msg=f"cloud {b}")
    _say(f"batched 4096: clouds {pick} equal the oracle's 30-iteration runs")


def test_batched_rejects(ekm):
    import torch
    dev = torch.device("cuda:0")
    x = torch.rand(300, 3, device=dev)
    with pytest.raises(ekm.EKMError):
        ekm.kmeans_init_batched(x, [0, 100, 300], [0, 101, 110])
    with pytest.raises(ekm.EKMError):
        ekm.kmeans_init_batched(x, [0, 100, 300], [0, 10, 20], algo=ekm.KM_BRUTE)
    with pytest.raises(ValueError):
        ekm.kmeans_init_batched(x, [0, 100, 300], [0, 10])
