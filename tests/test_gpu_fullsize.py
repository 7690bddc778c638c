"""GPU parity at the benchmark sizes, and on inputs built to stress the
exactness argument.

* 1e6 x 2D geo hotspots, k = 1000 (the benchmark workload): every point's
  assignment and every centroid, bit for bit, at every iteration of the run
  until it is stable or 100 iterations, against the FP64 oracle's own
  trajectory; kmeans_run stops at the same iteration.
* 1e7 x 3D ellipsoid surfaces, k = 1e4 and 1e5: every iteration the
  committed digests cover (tests/golden/surfaces3d_1e7_oracle.json, written
  by tests/golden/make_surfaces3d_oracle.py from the oracle alone), compared
  as SHA-256 of the whole assignment and the whole centroid array.
* The distortion pair at its full batch shape, all 256 clouds.
* Near ties the FP32 pass cannot order (the FP64 recheck decides), data far
  from the origin (the FP32 rounding of the centroids dominates the error
  bound), tiny candidate capacities (every fallback path), non-finite input
  and inputs too wide for exact sums.
"""

import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
from synth import geo_hotspots_2d, init_centroids, make_config, sha256_of

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN_3D = os.path.join(HERE, "golden", "surfaces3d_1e7_oracle.json")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def ekm():
    import torch
    import paper_2412_02244_amd as m
    m.load_library()
    assert torch.cuda.is_available()
    return m


def _steps(ekm, x, c0, iters, algo=1, flags=0, leaf_size=0):
    import torch
    dev = torch.device("cuda:0")
    ctx = ekm.kmeans_init(torch.from_numpy(x).to(dev), c0.shape[0], algo=algo, flags=flags, leaf_size=leaf_size)
    c = torch.from_numpy(c0).to(dev)
    a = torch.empty(x.shape[0], dtype=torch.int32, device=dev)
    for _ in range(iters):
        c, st = ekm.kmeans_step(ctx, c, torch.empty_like(c), assign_out=a, stats=True)
        yield a.cpu().numpy(), c.cpu().numpy(), st
    ctx.close()


def _compare(ekm, x, c0, ref, name, algo=1, flags=0):
    stats = []
    for t, (a, c, st) in enumerate(_steps(ekm, x, c0, ref["iters"], algo, flags)):
        bad = np.flatnonzero(a != ref["a_hist"][t])
        assert bad.size == 0, f"{name}: iteration {t + 1}: {bad.size} assignments differ, first at {bad[:5]}"
        np.testing.assert_array_equal(c, ref["c_hist"][t], err_msg=f"{name}: centroids at iteration {t + 1}")
        prev = ref["a_hist"][t - 1] if t else None
        assert st["n_changed"] == (x.shape[0] if prev is None else int((ref["a_hist"][t] != prev).sum()))
        stats.append(st)
    return stats


def test_geo2d_1e6_every_point_every_iteration(ekm):
    import torch
    x, c0, cfg = make_config(1)
    _say("[fullsize] geo2d 1e6 k=1000: oracle trajectory (until stable, at most 100 iterations)")
    ref = oracle.lloyd(x, c0, max_iter=100, stop_when_stable=True)
    _say(f"[fullsize] oracle: {ref['iters']} iterations; GPU step by step")
    stats = _compare(ekm, x, c0, ref, "geo2d 1e6")
    # the pruning machinery is really in use at this size
    assert sum(s["inter_leaf_points"] for s in stats[1:]) > 0
    assert sum(s["single_cand_points"] for s in stats) > 0
    assert sum(s["region_points"] for s in stats) > 0  # regions assigned whole
    _say("[fullsize] geo2d 1e6: kmeans_run until stable")
    dev = torch.device("cuda:0")
    ctx = ekm.kmeans_init(torch.from_numpy(x).to(dev), c0.shape[0])
    c = torch.from_numpy(c0).to(dev)
    a = torch.empty(x.shape[0], dtype=torch.int32, device=dev)
    iters, _ = ekm.kmeans_run(ctx, c, 100, stop_when_stable=True, assign_out=a)
    ctx.close()
    assert iters == ref["iters"]
    np.testing.assert_array_equal(c.cpu().numpy(), ref["c"])
    np.testing.assert_array_equal(a.cpu().numpy(), ref["a"])


@pytest.fixture(scope="module")
def surfaces():
    if not os.path.exists(GOLDEN_3D):
        pytest.skip("oracle digests for the 1e7 3D workload are not committed")
    golden = json.load(open(GOLDEN_3D))
    x, _, _ = make_config(2)
    assert sha256_of(x) == golden["data_sha256"], "the 1e7 3D generator no longer gives the committed data"
    return x, golden


@pytest.mark.parametrize("k", [10_000, 100_000])
def test_surfaces3d_1e7_oracle_digests(ekm, surfaces, k):
    x, golden = surfaces
    runs = [r for r in golden["runs"] if r["k"] == k]
    if not runs:
        pytest.skip(f"no oracle digests for k={k}")
    run = runs[0]
    c0 = init_centroids(x, k, 2002)
    assert _digest(c0) == run["c0_sha256"]
    _say(f"[fullsize] surfaces3d 1e7 k={k}: {len(run['steps'])} iterations against the oracle digests")
    for t, (a, c, st) in enumerate(_steps(ekm, x, c0, len(run["steps"]))):
        ref = run["steps"][t]
        if _digest(a.astype(np.int32)) != ref["assign_sha256"]:
            raise AssertionError(f"k={k} iteration {t + 1}: assignment digest differs "
                                 f"(first 16: {a[:16].tolist()} vs {ref['assign_head']}; "
                                 f"changed {st['n_changed']} vs {ref['n_changed']})")
        assert _digest(c.astype(np.float64)) == ref["centroids_sha256"], \
            f"k={k} iteration {t + 1}: centroid digest differs (c0 {c[0].tolist()} vs {ref['centroid0']})"
        assert st["n_changed"] == ref["n_changed"]


def test_distortion_full_batch_all_clouds(ekm):
    """256 clouds x 16,384 3D points, k = 512: every cloud's assignment
    bit-exact, loss within 1e-12 relative, gradients at the FP32 output
    tolerance (1e-6)."""
    import torch
    from synth import distortion_batch
    xb, cb = distortion_batch()
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(xb).to(dev)
    ct = torch.from_numpy(cb).to(dev)
    _say(f"[fullsize] distortion B={xb.shape[0]} n={xb.shape[1]} k={cb.shape[1]}: all clouds")
    a_gpu, loss = ekm.distortion_fwd(xt, ct)
    g = torch.linspace(0.5, 1.5, xb.shape[0], dtype=torch.float64, device=dev)
    gx, gc = ekm.distortion_bwd(xt, ct, a_gpu, g)
    a_gpu, loss, gx, gc = a_gpu.cpu().numpy(), loss.cpu().numpy(), gx.cpu().numpy(), gc.cpu().numpy()
    a_ref, l_ref = oracle.distortion_fwd(xb, cb)
    bad = np.flatnonzero((a_gpu != a_ref).any(1))
    assert bad.size == 0, f"assignments differ in clouds {bad[:8]}"
    np.testing.assert_allclose(loss, l_ref, rtol=1e-12)
    gx_ref, gc_ref = oracle.distortion_bwd(xb, cb, a_ref, g.cpu().numpy())
    np.testing.assert_allclose(gx, gx_ref, rtol=1e-6, atol=1e-6 * np.abs(gx_ref).max())
    np.testing.assert_allclose(gc, gc_ref, rtol=1e-6, atol=1e-6 * np.abs(gc_ref).max())


def test_fp32_blind_near_ties_are_rechecked(ekm):
    """Centroid pairs closer than FP32 can resolve: their fl32 copies are
    equal, so the FP32 pass sees exact ties that the lower index would win,
    while the FP64 distances make the other centroid strictly nearer for
    half of the points.  Only the FP64 recheck gets these right."""
    rng = np.random.default_rng(61)
    base = rng.uniform(0.25, 0.75, (40, 2)).astype(np.float32).astype(np.float64)  # FP32-exact
    # 3e-9 is below half an FP32 ulp on [0.25, 1), so base + 3e-9 rounds back to base
    k = 2 * base.shape[0]
    c0 = np.empty((k, 2))
    c0[0::2] = base + np.array([3e-9, 0.0])  # lower index: slightly to the right in FP64 ...
    c0[1::2] = base                           # ... the same point in FP32
    assert (c0[0::2].astype(np.float32) == c0[1::2].astype(np.float32)).all()
    x = (np.repeat(base, 50, 0) + rng.normal(0, 0.01, (50 * base.shape[0], 2))).astype(np.float32)
    ref = oracle.lloyd(x, c0, max_iter=2)
    a_ref = ref["a_hist"][0]
    assert (a_ref % 2 == 1).any() and (a_ref % 2 == 0).any(), "both members of the pairs win somewhere"
    for algo in (ekm.KM_INDEXED, ekm.KM_BRUTE):
        stats = _compare(ekm, x, c0, ref, f"fp32-blind ties algo={algo}", algo=algo)
        assert stats[0]["rechecked"] > 0
    # tiny lists: leaves scan all k (split over a workgroup's waves) and the
    # recheck runs there too
    stats = _compare(ekm, x, c0, ref, "fp32-blind ties, small lists", flags=ekm.KM_FLAG_SMALL_LISTS)
    assert stats[0]["rechecked"] > 0 and sum(s["fallback_points"] for s in stats) > 0


def test_large_offset_data(ekm):
    """Points around (1000, -2000): the FP32 rounding of the centroids is
    large next to the cluster spread, so the error bound is wide and many
    points are rechecked in FP64."""
    x = geo_hotspots_2d(40_000, n_hot=30, seed=63).astype(np.float64)
    x = (x * 0.05 + np.array([1000.0, -2000.0])).astype(np.float32)
    c0 = init_centroids(x, 200, 64)
    ref = oracle.lloyd(x, c0, max_iter=6)
    stats = _compare(ekm, x, c0, ref, "offset")
    assert sum(s["rechecked"] for s in stats) > 0


def test_small_lists_force_every_fallback(ekm):
    """KM_FLAG_SMALL_LISTS shrinks the candidate capacities: groups overflow,
    leaves are deferred to the per-leaf pass, and some leaves scan all k;
    the trajectory stays equal to the oracle's."""
    x = geo_hotspots_2d(60_000, seed=65)
    c0 = init_centroids(x, 500, 66)
    ref = oracle.lloyd(x, c0, max_iter=4)
    stats = _compare(ekm, x, c0, ref, "small lists", flags=ekm.KM_FLAG_SMALL_LISTS)
    for f in ("group_overflows", "deferred_leaves", "fallback_points"):
        assert sum(s[f] for s in stats) > 0, f


def test_nonfinite_points_rejected(ekm):
    import torch
    dev = torch.device("cuda:0")
    for bad in (np.nan, np.inf, -np.inf):
        x = np.random.default_rng(67).uniform(0, 1, (5000, 3)).astype(np.float32)
        x[1234, 1] = bad
        with pytest.raises(ekm.EKMError) as e:
            ekm.kmeans_init(torch.from_numpy(x).to(dev), 10)
        assert e.value.status == ekm.KM_ERR_INVALID and "NaN" in str(e.value)


def test_too_wide_for_exact_sums_rejected(ekm):
    import torch
    dev = torch.device("cuda:0")
    x = np.random.default_rng(68).uniform(0, 1, (4096, 2)).astype(np.float32)
    x[0, 0] = 1e30
    x[1, 1] = 1e-30
    with pytest.raises(ekm.EKMError) as e:
        ekm.kmeans_init(torch.from_numpy(x).to(dev), 8)
    assert e.value.status == ekm.KM_ERR_NOT_EXACT


def test_stream_mismatch_rejected(ekm):
    """A context's work goes to the stream it was created on; stepping it
    while another stream is current is refused by the binding."""
    import torch
    x = torch.rand(5000, 2, device="cuda")
    ctx = ekm.kmeans_init(x, 10)
    c = x[:10].double().clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with pytest.raises(ValueError):
            ekm.kmeans_step(ctx, c)
        with pytest.raises(ValueError):
            ekm.kmeans_run(ctx, c, 2)
    ekm.kmeans_step(ctx, c)  # back on the creation stream
    torch.cuda.synchronize()
    ctx.close()
