"""The library's own kernel sources, built for the CPU (tests/cpuemu: every
lane a fiber, wave operations and barriers as checked rendezvous, device
memory as host memory under AddressSanitizer), run small k-means
trajectories that are compared with the FP64 oracle.

This needs no GPU.  It catches out-of-bounds accesses, wave operations or
barriers that only part of a wave (or workgroup) reaches, and LDS hand-offs
between lanes without a wave barrier (the emulated lanes run ahead of one
another between rendezvous, so a missing one reads stale data).
"""

import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from synth import ellipsoid_surfaces_3d, gaussian_mixture_2d, geo_hotspots_2d, init_centroids

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "cpuemu"))
import build_emu  # noqa: E402

KM_F64, KM_F32 = 0, 1
KM_BRUTE, KM_INDEXED = 0, 1
KM_FLAG_SSE = 1
STATS = np.dtype([("n_changed", "<i8"), ("dist_evals", "<i8"), ("brute_evals", "<i8"),
                  ("single_cand_points", "<i8"), ("rechecked", "<i8"), ("cand_total", "<i8"),
                  ("leaves", "<i8"), ("sse", "<f8"), ("inter_leaf_points", "<i8"), ("inter_points", "<i8"),
                  ("fallback_points", "<i8"), ("deferred_leaves", "<i8"), ("group_overflows", "<i8"),
                  ("groups_skipped", "<i8"), ("region_points", "<i8")])

CTX_INFO = np.dtype([("device_bytes", "<i8"), ("model_bytes", "<i8"), ("model_bytes_actual_counts", "<i8"),
                     ("leaves", "<i8"), ("groups", "<i8"), ("allocations", "<i8"), ("leaf_size", "<i4"),
                     ("leaves_per_group", "<i4")])


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    return build_emu.build(str(tmp_path_factory.mktemp("cpuemu")))


def _run(driver, tmp_path, mode, x, c0, iters, algo, leaf_size=0, flags=0):
    n, d = x.shape
    k = c0.shape[0]
    pdt = KM_F32 if x.dtype == np.float32 else KM_F64
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        np.array([n, d, k, iters, algo, leaf_size, flags, pdt], np.int64).tofile(f)
        np.ascontiguousarray(x).tofile(f)
        np.ascontiguousarray(c0, np.float64).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([driver, mode, str(inp), str(out)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, f"emulated run failed ({r.returncode}):\n{r.stderr[-4000:]}"
    raw = open(out, "rb").read()
    if mode == "info":
        return np.frombuffer(raw, CTX_INFO)[0]
    if mode == "run":
        it = int(np.frombuffer(raw[:4], np.int32)[0])
        a = np.frombuffer(raw[4:4 + 4 * n], np.int32)
        c = np.frombuffer(raw[4 + 4 * n:], np.float64).reshape(k, d)
        return it, a, c
    step = 4 * n + 8 * k * d + STATS.itemsize
    res = []
    for t in range(iters):
        b = raw[t * step:(t + 1) * step]
        a = np.frombuffer(b[:4 * n], np.int32)
        c = np.frombuffer(b[4 * n:4 * n + 8 * k * d], np.float64).reshape(k, d)
        st = np.frombuffer(b[4 * n + 8 * k * d:], STATS)[0]
        res.append((a, c, st))
    return res


def _check(driver, tmp_path, x, c0, iters, algo, leaf_size=0):
    ref = oracle.lloyd(x, c0, max_iter=iters)
    got = _run(driver, tmp_path, "kmeans", x, c0, iters, algo, leaf_size, KM_FLAG_SSE)
    for t, (a, c, st) in enumerate(got):
        bad = np.flatnonzero(a != ref["a_hist"][t])
        assert bad.size == 0, f"iteration {t + 1}: {bad.size} assignments differ, first at {bad[:5]}"
        np.testing.assert_array_equal(c, ref["c_hist"][t], err_msg=f"centroids at iteration {t + 1}")
        assert st["sse"] == pytest.approx(ref["sse"][t], rel=1e-12)
        prev = ref["a_hist"][t - 1] if t else None
        want = x.shape[0] if prev is None else int((ref["a_hist"][t] != prev).sum())
        assert st["n_changed"] == want
    return got


@pytest.mark.parametrize("leaf_size", [0, 16])
def test_emulated_indexed_2d(driver, tmp_path, leaf_size):
    x = geo_hotspots_2d(3000, n_hot=12, seed=71)
    c0 = init_centroids(x, 40, 72)
    _check(driver, tmp_path, x, c0, 3, KM_INDEXED, leaf_size)


def test_emulated_indexed_3d(driver, tmp_path):
    x = ellipsoid_surfaces_3d(2500, 4, seed=73)
    c0 = init_centroids(x, 30, 74)
    _check(driver, tmp_path, x, c0, 3, KM_INDEXED)


def test_emulated_large_k_tree_keeps_its_order(driver, tmp_path):
    """k above the one-workgroup tree limit: the centroid tree is built in
    global memory, sorted on the first step and every eighth after it, and
    between sorts rebuilt over the order it had (and the inter bound comes
    from the tree search seeded by the last step's bound plus drift).  Ten
    steps equal the oracle's."""
    x = ellipsoid_surfaces_3d(14000, 6, seed=75)
    c0 = init_centroids(x, 4500, 76)
    _check(driver, tmp_path, x, c0, 10, KM_INDEXED)


def test_emulated_large_k_small_frontier(driver, tmp_path):
    """The same path with tiny capacities: the wave search for the nearest
    other centroid overflows its frontier and every lane searches alone."""
    x = geo_hotspots_2d(4400, n_hot=15, seed=77).astype(np.float32)
    c0 = init_centroids(x, 4150, 78)
    ref = oracle.lloyd(x, c0, max_iter=2)
    got = _run(driver, tmp_path, "kmeans", x, c0, 2, KM_INDEXED, 0, KM_FLAG_SSE | KM_FLAG_SMALL_LISTS)
    for t, (a, c, st) in enumerate(got):
        np.testing.assert_array_equal(a, ref["a_hist"][t])
        np.testing.assert_array_equal(c, ref["c_hist"][t])


def test_emulated_brute_fp32_and_fp64(driver, tmp_path):
    x = geo_hotspots_2d(1500, n_hot=6, seed=75)
    c0 = init_centroids(x, 20, 76)
    _check(driver, tmp_path, x, c0, 2, KM_BRUTE)
    xd = gaussian_mixture_2d(1200, seed=77)
    _check(driver, tmp_path, xd, init_centroids(xd, 15, 78), 2, KM_BRUTE)


def test_emulated_run_until_stable(driver, tmp_path):
    x = gaussian_mixture_2d(2000, seed=79).astype(np.float32)
    c0 = init_centroids(x, 12, 80)
    ref = oracle.lloyd(x, c0, max_iter=60, stop_when_stable=True)
    it, a, c = _run(driver, tmp_path, "run", x, c0, 60, KM_INDEXED, flags=1 << 16)
    assert it == ref["iters"]
    np.testing.assert_array_equal(a, ref["a"])
    np.testing.assert_array_equal(c, ref["c"])


KM_FLAG_SMALL_LISTS = 4


def test_emulated_fallback_paths(driver, tmp_path):
    """Tiny candidate capacities: group overflow, deferred leaves and the
    scan of all k centroids all run, and the trajectory is unchanged.  The
    statistics are folded by several workgroups that hand their totals to
    the last one: the change counts and the objective still match."""
    x = geo_hotspots_2d(4000, n_hot=10, seed=81)
    c0 = init_centroids(x, 90, 82)
    ref = oracle.lloyd(x, c0, max_iter=3)
    got = _run(driver, tmp_path, "kmeans", x, c0, 3, KM_INDEXED, 0, KM_FLAG_SSE | KM_FLAG_SMALL_LISTS)
    for t, (a, c, st) in enumerate(got):
        np.testing.assert_array_equal(a, ref["a_hist"][t])
        np.testing.assert_array_equal(c, ref["c_hist"][t])
        assert st["sse"] == pytest.approx(ref["sse"][t], rel=1e-12)
        want = x.shape[0] if t == 0 else int((ref["a_hist"][t] != ref["a_hist"][t - 1]).sum())
        assert st["n_changed"] == want
    tot = {f: sum(int(st[f]) for _, _, st in got) for f in ("group_overflows", "deferred_leaves", "fallback_points")}
    assert all(v > 0 for v in tot.values()), tot


def test_emulated_fallback_scan_with_fp32_blind_ties(driver, tmp_path):
    """Centroid pairs that FP32 cannot tell apart (their fl32 copies are
    equal; FP64 makes the higher index nearer for some points), with tiny
    list capacities: leaves scan all k centroids, and the FP64 recheck of
    that scan gives the oracle's lowest-index FP64 argmin."""
    rng = np.random.default_rng(83)
    base = rng.uniform(0.25, 0.75, (24, 2)).astype(np.float32).astype(np.float64)
    c0 = np.empty((48, 2))
    c0[0::2] = base + np.array([3e-9, 0.0])  # below half an FP32 ulp: the same fl32 point
    c0[1::2] = base
    x = (np.repeat(base, 40, 0) + rng.normal(0, 0.01, (40 * base.shape[0], 2))).astype(np.float32)
    ref = oracle.lloyd(x, c0, max_iter=2)
    assert (ref["a_hist"][0] % 2 == 1).any() and (ref["a_hist"][0] % 2 == 0).any()
    got = _run(driver, tmp_path, "kmeans", x, c0, 2, KM_INDEXED, 0, KM_FLAG_SSE | KM_FLAG_SMALL_LISTS)
    for t, (a, c, st) in enumerate(got):
        np.testing.assert_array_equal(a, ref["a_hist"][t])
        np.testing.assert_array_equal(c, ref["c_hist"][t])
    assert got[0][2]["rechecked"] > 0 and got[0][2]["fallback_points"] > 0, got[0][2]


def test_emulated_long_candidate_lists(driver, tmp_path):
    """2,000 uniform points and, far away, a tight blob of 150 points holding
    all 150 centroids: from every uniform leaf the blob's centroids are
    almost equidistant, so each leaf keeps them all as candidates (lists of
    about 150, several 64-entry chunks per scan and recheck), one leaf per
    group.  Four steps equal the oracle's."""
    rng = np.random.default_rng(85)
    blob = np.array([6.0, 6.0]) + rng.normal(0, 0.01, (150, 2))
    x = np.concatenate([rng.uniform(0, 1, (2000, 2)), blob]).astype(np.float32)
    c0 = x[2000:].astype(np.float64)
    ref = oracle.lloyd(x, c0, max_iter=4)
    got = _run(driver, tmp_path, "kmeans", x, c0, 4, KM_INDEXED, 0, KM_FLAG_SSE | (1 << 20))
    for t, (a, c, st) in enumerate(got):
        np.testing.assert_array_equal(a, ref["a_hist"][t], err_msg=f"step {t + 1}")
        np.testing.assert_array_equal(c, ref["c_hist"][t], err_msg=f"step {t + 1}")
        assert st["sse"] == pytest.approx(ref["sse"][t], rel=1e-12)
    assert got[0][2]["cand_total"] > 100 * got[0][2]["leaves"] // 2, got[0][2]


def test_emulated_uniform_long_lists(driver, tmp_path):
    """4,000 uniform points and 1,500 uniform centroids drawn apart from
    them: at the first step the leaves span wide boxes against a dense
    centroid set, with lists of 30 to 130 candidates that differ from leaf
    to leaf (unlike the blob case above, where every leaf keeps the same
    ones).  Three steps equal the oracle's."""
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, (4000, 2)).astype(np.float32)
    c0 = rng.uniform(0, 1, (1500, 2))
    ref = oracle.lloyd(x, c0, max_iter=3)
    got = _run(driver, tmp_path, "kmeans", x, c0, 3, KM_INDEXED, 0, KM_FLAG_SSE | (1 << 20))
    for t, (a, c, st) in enumerate(got):
        np.testing.assert_array_equal(a, ref["a_hist"][t], err_msg=f"step {t + 1}")
        np.testing.assert_array_equal(c, ref["c_hist"][t], err_msg=f"step {t + 1}")
        assert st["sse"] == pytest.approx(ref["sse"][t], rel=1e-12)
    st = got[0][2]
    assert st["cand_total"] > 40 * st["leaves"], st  # long lists


def test_emulated_long_trajectory_inter_bounds(driver, tmp_path):
    """Ten steps: the exact sums are carried from step to step and moved
    point by point or leaf by leaf, the inter bounds keep leaves and points,
    and regions with a single candidate are assigned whole; every step still
    equals the oracle."""
    x = gaussian_mixture_2d(5000, seed=83).astype(np.float32)
    c0 = init_centroids(x, 25, 84)
    got = _check(driver, tmp_path, x, c0, 10, KM_INDEXED)
    kept_leaf = sum(int(st["inter_leaf_points"]) for _, _, st in got[1:])
    kept_pt = sum(int(st["inter_points"]) for _, _, st in got[1:])
    region = sum(int(st["region_points"]) for _, _, st in got)
    assert kept_leaf > 0 and kept_pt > 0 and region > 0, (kept_leaf, kept_pt, region)
    assert got[0][2]["inter_leaf_points"] == 0  # nothing is kept before the first assignment


def _clouds(sizes, ks, seed):
    """Concatenated clouds of the given sizes (a mix of 2-D workloads) with
    their own initial centroids, and the offsets of both."""
    xs, cs = [], []
    for b, (n, k) in enumerate(zip(sizes, ks)):
        gen = (geo_hotspots_2d, gaussian_mixture_2d)[b % 2]
        x = gen(n, seed=seed + 2 * b).astype(np.float32)
        xs.append(x)
        cs.append(init_centroids(x, k, seed + 2 * b + 1))
    po = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    co = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
    return xs, cs, po, co


def _run_batched(driver, tmp_path, mode, xs, cs, po, co, iters, leaf_size=0, cand_tile=0, flags=0):
    x = np.concatenate(xs)
    c0 = np.concatenate(cs)
    n, d = x.shape
    k = c0.shape[0]
    B = len(xs)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        np.array([n, d, k, iters, KM_INDEXED, leaf_size, flags | cand_tile << 20, KM_F32], np.int64).tofile(f)
        np.array([B], np.int64).tofile(f)
        po.tofile(f)
        co.tofile(f)
        x.tofile(f)
        np.ascontiguousarray(c0, np.float64).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([driver, mode, str(inp), str(out)], capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, f"emulated run failed ({r.returncode}):\n{r.stderr[-4000:]}"
    raw = open(out, "rb").read()
    if mode == "infob":
        return np.frombuffer(raw, CTX_INFO)[0]
    if mode == "runb":
        fG = np.frombuffer(raw[:8], np.int32)
        return (int(fG[0]), int(fG[1])), np.frombuffer(raw[8:8 + 4 * n], np.int32), \
            np.frombuffer(raw[8 + 4 * n:], np.float64).reshape(k, d)
    step = 4 * n + 8 * k * d + STATS.itemsize
    res = []
    for t in range(iters):
        b = raw[t * step:(t + 1) * step]
        res.append((np.frombuffer(b[:4 * n], np.int32), np.frombuffer(b[4 * n:4 * n + 8 * k * d],
                                                                      np.float64).reshape(k, d)))
    return res


def test_emulated_batched_clouds(driver, tmp_path):
    """Clouds of different sizes and centroid counts (one with k_b = n_b, one
    with a single centroid) in one context: every cloud's step equals the
    oracle run on that cloud alone, with cloud-local centroid ids."""
    sizes, ks = [900, 40, 1300, 7, 600], [14, 40, 25, 1, 9]
    xs, cs, po, co = _clouds(sizes, ks, 90)
    got = _run_batched(driver, tmp_path, "batched", xs, cs, po, co, 4, flags=KM_FLAG_SSE)
    for b in range(len(xs)):
        ref = oracle.lloyd(xs[b], cs[b], max_iter=4)
        for t, (a, c) in enumerate(got):
            np.testing.assert_array_equal(a[po[b]:po[b + 1]], ref["a_hist"][t], err_msg=f"cloud {b} step {t + 1}")
            np.testing.assert_array_equal(c[co[b]:co[b + 1]], ref["c_hist"][t], err_msg=f"cloud {b} step {t + 1}")


def test_emulated_run_batched_autotune(driver, tmp_path):
    """kmeans_run_batched with leaf size and list length left to the tuner
    (it times its candidates on the clouds, then runs them all): the result
    is the oracle's whatever it picked, and the pick is one of the candidates."""
    sizes, ks = [700, 500, 800], [10, 6, 12]
    xs, cs, po, co = _clouds(sizes, ks, 95)
    (f, G), a, c = _run_batched(driver, tmp_path, "runb", xs, cs, po, co, 3)
    assert f in (16, 32, 64) and G in (4, 6, 8), (f, G)
    for b in range(len(xs)):
        ref = oracle.lloyd(xs[b], cs[b], max_iter=3)
        np.testing.assert_array_equal(a[po[b]:po[b + 1]], ref["a"], err_msg=f"cloud {b}")
        np.testing.assert_array_equal(c[co[b]:co[b + 1]], ref["c"], err_msg=f"cloud {b}")
    (f2, G2), a2, c2 = _run_batched(driver, tmp_path, "runb", xs, cs, po, co, 3, leaf_size=32, cand_tile=4)
    assert (f2, G2) == (32, 4)
    np.testing.assert_array_equal(a2, a)
    np.testing.assert_array_equal(c2, c)


KM_FLAG_SMALL_LISTS, KM_FLAG_CELL_LEAVES = 4, 8


@pytest.mark.parametrize("case", ["brute32", "brute32_20k", "brute64", "packed", "packed_f16", "cells",
                                  "cells_20k", "small_lists", "tiny", "large_k", "batched"])
def test_emulated_workspace_model_is_exact_with_actual_counts(driver, tmp_path, case):
    """The workspace model evaluated with the context's actual leaf and group
    counts equals the device bytes the context holds, on every path: each
    buffer is allocated where the model puts it (no buffer of one part
    takes the arena space of another)."""
    if case == "batched":
        xs, cs, po, co = _clouds([900, 40, 1300, 7, 600], [14, 40, 25, 1, 9], 97)
        info = _run_batched(driver, tmp_path, "infob", xs, cs, po, co, 0)
    else:
        n, k = {"tiny": (300, 5), "large_k": (20000, 5000), "brute32_20k": (20000, 100),
                "cells_20k": (20000, 100)}.get(case, (6000, 60))
        x = geo_hotspots_2d(n, n_hot=12, seed=99).astype(np.float64 if case == "brute64" else np.float32)
        c0 = init_centroids(x, k, 98)
        algo = KM_BRUTE if case.startswith("brute") else KM_INDEXED
        leaf = 16 if case == "packed_f16" else 0
        flags = {"cells": KM_FLAG_CELL_LEAVES, "cells_20k": KM_FLAG_CELL_LEAVES,
                 "small_lists": KM_FLAG_SMALL_LISTS}.get(case, 0)
        info = _run(driver, tmp_path, "info", x, c0, 0, algo, leaf, flags)
    assert info["model_bytes_actual_counts"] == info["device_bytes"], info
