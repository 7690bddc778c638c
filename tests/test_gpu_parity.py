"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Assignments must be bit-identical every iteration (lowest index on ties);
centroids must be bit-identical as well (exact sums, one rounding, IEEE
division), which is stricter than the 1e-12 relative bound the method
allows.  Sizes span many leaves and blocks with ragged tails; the full-size
2D case is checked step by step on sampled points plus the full update.
"""

import sys

import numpy as np
import pytest

import oracle
from synth import ellipsoid_surfaces_3d, gaussian_mixture_2d, geo_hotspots_2d, init_centroids, make_config

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


def _run_steps(ekm, x, c0, iters, algo, leaf_size=0, stats=False):
    """Step the GPU from c0; return per-step (assign, centroids, stats)."""
    import torch
    dev = torch.device("cuda:0")
    ctx = ekm.kmeans_init(torch.from_numpy(x).to(dev), c0.shape[0], algo=algo, leaf_size=leaf_size,
                          flags=ekm.KM_FLAG_SSE)
    c = torch.from_numpy(c0).to(dev)
    a = torch.empty(x.shape[0], dtype=torch.int32, device=dev)
    out = []
    for _ in range(iters):
        c, st = ekm.kmeans_step(ctx, c, torch.empty_like(c), assign_out=a, stats=True)
        out.append((a.cpu().numpy().copy(), c.cpu().numpy().copy(), st))
    ctx.close()
    return out


def _check_trajectory(ekm, x, c0, iters, algo, leaf_size=0, name=""):
    _say(f"[parity] {name} n={x.shape[0]} k={c0.shape[0]} d={x.shape[1]} algo={algo} f={leaf_size} iters={iters}")
    ref = oracle.lloyd(x, c0, max_iter=iters, stop_when_stable=False)
    got = _run_steps(ekm, x, c0, iters, algo, leaf_size)
    for t in range(iters):
        a, c, st = got[t]
        bad = np.flatnonzero(a != ref["a_hist"][t])
        assert bad.size == 0, f"{name}: iteration {t + 1}: {bad.size} assignments differ, first at {bad[:5]}"
        np.testing.assert_array_equal(c, ref["c_hist"][t], err_msg=f"{name}: centroids at iteration {t + 1}")
        assert st["sse"] == pytest.approx(ref["sse"][t], rel=1e-12)
        prev = ref["a_hist"][t - 1] if t else None
        want_changed = x.shape[0] if t == 0 else int((ref["a_hist"][t] != prev).sum())
        assert st["n_changed"] == want_changed
    return got


def test_plain_fp64_brute_gaussian2d(ekm):
    x, c0, cfg = make_config(0)
    _check_trajectory(ekm, x, c0, cfg["iters"], ekm.KM_BRUTE, name="gauss2d fp64")


@pytest.mark.parametrize("algo", ["indexed", "brute"])
def test_geo2d_fp32_trajectory(ekm, algo):
    x = geo_hotspots_2d(30_011, seed=1001)
    c0 = init_centroids(x, 150, 2001)
    a = ekm.KM_INDEXED if algo == "indexed" else ekm.KM_BRUTE
    got = _check_trajectory(ekm, x, c0, 12, a, name=f"geo2d {algo}")
    if algo == "indexed":
        st = got[-1][2]
        assert st["dist_evals"] < 0.2 * st["brute_evals"]  # the index prunes most pairs
        assert st["single_cand_points"] > 0


def test_ellipsoids3d_indexed_trajectory(ekm):
    x = ellipsoid_surfaces_3d(40_000, n_ell=12, seed=1002)
    c0 = init_centroids(x, 400, 2002)
    _check_trajectory(ekm, x, c0, 6, ekm.KM_INDEXED, name="ellipsoids3d")


@pytest.mark.parametrize("f", [8, 16, 32, 64])
def test_leaf_sizes(ekm, f):
    x = geo_hotspots_2d(9_999, seed=7)
    c0 = init_centroids(x, 77, 8)
    _check_trajectory(ekm, x, c0, 4, ekm.KM_INDEXED, leaf_size=f, name=f"leaf f={f}")


def test_large_k_radix_tree_path(ekm):
    # k above the single-workgroup tree limit: centroids sorted by the device radix sort
    x = ellipsoid_surfaces_3d(120_000, n_ell=30, seed=5)
    c0 = init_centroids(x, 9000, 6)
    _check_trajectory(ekm, x, c0, 3, ekm.KM_INDEXED, name="k=9000")


@pytest.mark.parametrize("case", ["n1k1", "ragged", "k_eq_n", "identical", "dup_centroids", "far_centroid",
                                  "tiny_values", "negative"])
def test_edge_cases(ekm, case):
    rng = np.random.default_rng(11)
    if case == "n1k1":
        x = np.array([[0.25, 0.5]], np.float32)
        c0 = x.astype(np.float64)
    elif case == "ragged":
        x = rng.uniform(0, 1, (65, 3)).astype(np.float32)
        c0 = init_centroids(x, 3, 1)
    elif case == "k_eq_n":
        x = rng.uniform(0, 1, (130, 2)).astype(np.float32)
        c0 = init_centroids(x, 130, 2)
    elif case == "identical":
        x = np.full((300, 2), 0.375, np.float32)
        c0 = np.array([[0.375, 0.375], [0.5, 0.5], [0.375, 0.375]])
    elif case == "dup_centroids":
        x = rng.uniform(0, 1, (500, 2)).astype(np.float32)
        c0 = init_centroids(x, 10, 3)
        c0[7] = c0[2]
    elif case == "far_centroid":
        x = rng.uniform(0, 1, (500, 3)).astype(np.float32)
        c0 = init_centroids(x, 6, 4)
        c0[4] = [40.0, -30.0, 25.0]
    elif case == "tiny_values":
        x = (rng.uniform(0, 1, (700, 2)) * 1e-6).astype(np.float32)
        c0 = init_centroids(x, 9, 5)
    else:
        x = rng.uniform(-3, -1, (700, 2)).astype(np.float32)
        c0 = init_centroids(x, 9, 6)
    for algo in (ekm.KM_INDEXED, ekm.KM_BRUTE):
        _check_trajectory(ekm, x, c0, 3, algo, name=f"edge {case}")


def test_ties_on_bisector_go_to_lowest_index(ekm):
    # points exactly on the bisector of two centroids (exact in FP32 and FP64)
    ys = np.linspace(0, 1, 257, dtype=np.float32)
    x = np.stack([np.full_like(ys, 0.5), ys], 1)
    x = np.concatenate([x, np.array([[0.25, 0.5], [0.75, 0.5]], np.float32)])
    c0 = np.array([[0.75, 0.5], [0.25, 0.5]])
    for algo in (ekm.KM_INDEXED, ekm.KM_BRUTE):
        got = _check_trajectory(ekm, x, c0, 1, algo, name="bisector")
        assert (got[0][0][:257] == 0).all()


@pytest.fixture(scope="module")
def surfaces_1e7():
    x, _, _ = make_config(2)
    return x


@pytest.mark.parametrize("k", [10_000, 100_000])
def test_full_size_surfaces3d_sampled(ekm, surfaces_1e7, k):
    """1e7 x 3D ellipsoid surfaces, k = 1e4 (LDS tree build) and 1e5 (global
    radix tree build): two steps; sampled assignments against the oracle's
    brute force, every centroid against the oracle's exact update of the
    GPU's own assignment."""
    import torch
    x = surfaces_1e7
    c0 = init_centroids(x, k, 2002)  # the seed make_config(2) uses
    dev = torch.device("cuda:0")
    _say(f"[parity] surfaces3d n={x.shape[0]} k={k}: context")
    ctx = ekm.kmeans_init(torch.from_numpy(x).to(dev), k, algo=ekm.KM_INDEXED)
    rng = np.random.default_rng(k)
    sample = np.concatenate([rng.choice(x.shape[0], 5000, replace=False), np.arange(64), [x.shape[0] - 1]])
    c = torch.from_numpy(c0).to(dev)
    a = torch.empty(x.shape[0], dtype=torch.int32, device=dev)
    for t in range(2):
        _say(f"[parity] surfaces3d k={k} step {t + 1}")
        c_prev = c.cpu().numpy()
        c = ekm.kmeans_step(ctx, c, assign_out=a)
        a_gpu = a.cpu().numpy()
        a_ref, _ = oracle.assign(x[sample], c_prev)
        assert (a_gpu[sample] == a_ref).all(), f"step {t + 1}: sampled assignments differ from the oracle"
        c_ref, _ = oracle.update(x, a_gpu, c_prev)
        np.testing.assert_array_equal(c.cpu().numpy(), c_ref)
    ctx.close()


def test_full_size_geo2d_stepwise(ekm):
    """1e6 x 2D, k=1000 (the benchmark workload): each step's sampled
    assignments against the oracle's brute force, the whole update against
    the oracle's exact means, and indexed == brute on every point."""
    import torch
    x, c0, cfg = make_config(1)
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(x).to(dev)
    _say("[parity] full-size geo2d: contexts")
    ci = ekm.kmeans_init(xt, 1000, algo=ekm.KM_INDEXED)
    cb = ekm.kmeans_init(xt, 1000, algo=ekm.KM_BRUTE)
    rng = np.random.default_rng(0)
    sample = np.concatenate([rng.choice(x.shape[0], 4000, replace=False), np.arange(64), [x.shape[0] - 1]])
    c = torch.from_numpy(c0).to(dev)
    ai = torch.empty(x.shape[0], dtype=torch.int32, device=dev)
    ab = torch.empty_like(ai)
    for t in range(4):
        _say(f"[parity] full-size geo2d step {t + 1}")
        c_prev = c.cpu().numpy()
        cn_i = ekm.kmeans_step(ci, c, assign_out=ai)
        cn_b = ekm.kmeans_step(cb, c, assign_out=ab)
        a_i, a_b = ai.cpu().numpy(), ab.cpu().numpy()
        assert (a_i == a_b).all(), f"step {t + 1}: indexed and brute disagree on {(a_i != a_b).sum()} points"
        a_ref, _ = oracle.assign(x[sample], c_prev)
        assert (a_i[sample] == a_ref).all(), f"step {t + 1}: sampled assignments differ from the oracle"
        c_ref, _ = oracle.update(x, a_i, c_prev)
        np.testing.assert_array_equal(cn_i.cpu().numpy(), c_ref)
        np.testing.assert_array_equal(cn_b.cpu().numpy(), c_ref)
        c = cn_i
    ci.close()
    cb.close()


def test_run_until_stable_matches_oracle(ekm):
    import torch
    x = gaussian_mixture_2d(20_000, seed=21, dtype=np.float32)
    c0 = init_centroids(x, 30, 22)
    ref = oracle.lloyd(x, c0, max_iter=100, stop_when_stable=True)
    dev = torch.device("cuda:0")
    for algo in (ekm.KM_INDEXED, ekm.KM_BRUTE):
        _say(f"[parity] run until stable algo={algo}")
        ctx = ekm.kmeans_init(torch.from_numpy(x).to(dev), 30, algo=algo)
        c = torch.from_numpy(c0).to(dev)
        a = torch.empty(x.shape[0], dtype=torch.int32, device=dev)
        iters, stats = ekm.kmeans_run(ctx, c, 100, stop_when_stable=True, assign_out=a, per_iter=True)
        ctx.close()
        assert iters == ref["iters"]
        np.testing.assert_array_equal(c.cpu().numpy(), ref["c"])
        np.testing.assert_array_equal(a.cpu().numpy(), ref["a"])
        assert stats[-1]["n_changed"] == 0


def test_resume_is_bit_identical(ekm):
    import torch
    x = geo_hotspots_2d(20_000, seed=31)
    c0 = init_centroids(x, 60, 32)
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(x).to(dev)
    ctx = ekm.kmeans_init(xt, 60)
    c = torch.from_numpy(c0).to(dev)
    ekm.kmeans_run(ctx, c, 8)
    c_mid = c.clone()
    ekm.kmeans_run(ctx, c, 7)
    ctx.close()
    ctx2 = ekm.kmeans_init(xt, 60)
    ekm.kmeans_run(ctx2, c_mid, 7)
    ctx2.close()
    assert torch.equal(c, c_mid)


def test_deterministic_stats(ekm):
    x = geo_hotspots_2d(50_000, seed=41)
    c0 = init_centroids(x, 200, 42)
    r1 = _run_steps(ekm, x, c0, 3, ekm.KM_INDEXED)
    r2 = _run_steps(ekm, x, c0, 3, ekm.KM_INDEXED)
    for (a1, c1, s1), (a2, c2, s2) in zip(r1, r2):
        assert (a1 == a2).all() and (c1 == c2).all()
        assert s1 == s2


@pytest.mark.parametrize("k", [40, 1500])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_distortion_fwd_bwd(ekm, dtype, k):
    """k = 40: the centroid-gradient sums of a cloud sit in LDS, and the
    20,000 points of a cloud span two LDS workgroups; k = 1500 (3D): they do
    not fit, and the kernel with global atomics runs."""
    import torch
    from synth import distortion_batch
    xb, cb = distortion_batch(n_clouds=4, n=20_000 if k == 40 else 5000, k=k, seed=51)
    if dtype == "f64":
        xb, cb = xb.astype(np.float64), cb.astype(np.float64)
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(xb).to(dev).requires_grad_(True)
    ct = torch.from_numpy(cb).to(dev).requires_grad_(True)
    _say(f"[parity] distortion {dtype}")
    loss = ekm.Distortion.apply(xt, ct)
    g = torch.tensor([1.0, -0.5, 2.0, 0.25], dtype=torch.float64, device=dev)
    (loss * g).sum().backward()
    a_ref, l_ref = oracle.distortion_fwd(xb, cb)
    a_gpu, _ = ekm.distortion_fwd(xt.detach(), ct.detach())
    assert (a_gpu.cpu().numpy() == a_ref).all()
    np.testing.assert_allclose(loss.detach().cpu().numpy(), l_ref, rtol=1e-12)
    gx_ref, gc_ref = oracle.distortion_bwd(xb, cb, a_ref, g.cpu().numpy())
    tol = 1e-6 if dtype == "f32" else 1e-12
    np.testing.assert_allclose(xt.grad.cpu().numpy(), gx_ref, rtol=tol, atol=tol * np.abs(gx_ref).max())
    np.testing.assert_allclose(ct.grad.cpu().numpy(), gc_ref, rtol=tol, atol=tol * np.abs(gc_ref).max())


def test_distortion_full_batch_sampled_clouds(ekm):
    """The distortion pair at its full batch shape (256 clouds x 16,384 3D
    points, k = 512, one launch each way): four clouds, including the first
    and the last, checked against the oracle (assignments bit-exact, loss
    1e-12 relative, gradients at the FP32 output tolerance)."""
    import torch
    from synth import distortion_batch
    xb, cb = distortion_batch()
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(xb).to(dev)
    ct = torch.from_numpy(cb).to(dev)
    _say(f"[parity] distortion full batch B={xb.shape[0]} n={xb.shape[1]} k={cb.shape[1]}")
    a_gpu, loss = ekm.distortion_fwd(xt, ct)
    g = torch.linspace(0.5, 1.5, xb.shape[0], dtype=torch.float64, device=dev)
    gx, gc = ekm.distortion_bwd(xt, ct, a_gpu, g)
    a_gpu, loss, gx, gc = a_gpu.cpu().numpy(), loss.cpu().numpy(), gx.cpu().numpy(), gc.cpu().numpy()
    pick = np.array([0, 77, 190, xb.shape[0] - 1])
    a_ref, l_ref = oracle.distortion_fwd(xb[pick], cb[pick])
    assert (a_gpu[pick] == a_ref).all()
    np.testing.assert_allclose(loss[pick], l_ref, rtol=1e-12)
    gx_ref, gc_ref = oracle.distortion_bwd(xb[pick], cb[pick], a_ref, g.cpu().numpy()[pick])
    np.testing.assert_allclose(gx[pick], gx_ref, rtol=1e-6, atol=1e-6 * np.abs(gx_ref).max())
    np.testing.assert_allclose(gc[pick], gc_ref, rtol=1e-6, atol=1e-6 * np.abs(gc_ref).max())
