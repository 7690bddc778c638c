#!/usr/bin/env python3
"""Benchmark of the exact k-means hot path on one MI355X.

Workload: 1e6 2D geo-like points (Zipf-weighted Gaussian hotspots plus a
uniform background, the shape of the paper's GPS trajectory data sets),
k = 1000, centroids initialised from a seeded permutation.  One step = one
Lloyd iteration (centroid tree, leaf candidates, assignment with FP64
recheck, exact centroid update).  The timed region is K consecutive
iterations 1..K of that run (kmeans_run on a fresh context), inputs already
on the GPU.

Prints ONE JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "point-assignments/s per Lloyd iter, 1e6×2D k=1e3; indexed vs brute GPU"
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(phase: str, n: int, k: int, d: int, L: int) -> float:
    """Bytes each phase must move per launch (per-unit figure x units)."""
    if phase == "assign":
        return n * (4 * d + 8)            # read point, read + write its assignment
    if phase == "tree":
        return k * (8 * d + 16 + 16)      # FP64 centroid in, fl32 copy and tree-ordered copy out
    return k * (8 * d * 2 + 16 * d + 4)   # FP64 in/out, exact sums and counts


def time_steps(ekm, torch, ctx, c0t, steps: int) -> float:
    """GPU milliseconds for `steps` iterations from c0t (kmeans_run; events on
    the current stream, which is the stream the library launches on)."""
    c = c0t.clone()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ekm.kmeans_run(ctx, c, steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "assign_geo2d_1e6_k1000_traffic.json")


def assign_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2412_02244_amd", "csrc", "assign.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic():
    """HBM bytes per assignment step from the committed counter summary, or
    None if the assignment kernels changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("assign_hip_sha256") != assign_source_hash():
        return None
    return t.get("bytes_per_step")


def cpu_baseline(x, c0, target_s: float):
    import oracle
    t = time.perf_counter()
    oracle.lloyd(x, c0, max_iter=1, history=False)
    t1 = time.perf_counter() - t
    iters = int(max(1, min(100, target_s / max(t1, 1e-6))))
    t = time.perf_counter()
    oracle.lloyd(x, c0, max_iter=iters, history=False)
    dt = time.perf_counter() - t
    return dict(value=x.shape[0] * iters / dt, unit="point-assignments/s", cores=oracle.num_threads(),
                kind="oracle",
                sample=f"Lloyd iterations 1..{iters} of the same 1e6x2D k=1000 run (FP64 brute force, "
                       f"{dt:.1f} s on the host)")


def summarize_counters(fetch_csv: str, write_csv: str) -> dict:
    """HBM bytes per assignment step from two rocprofv3 --pmc runs of
    `bench.py --quick --copy-calib` (FETCH_SIZE, then WRITE_SIZE, in KiB per
    dispatch).  Each counter is scaled by what it reads for the 256 MiB
    device copy in the same run (expected: 256 MiB fetched, 256 MiB
    written)."""
    import csv
    import statistics

    copy_bytes = float(256 << 20)

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        by = {}
        for r in rows:
            by.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return by

    out = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        by = per_kernel(path, name)
        copies = [max(v) for k, v in by.items() if "copyBuffer" in k or "copy" in k.lower() and "ekm" not in k]
        calib = max(copies) / copy_bytes if copies else 1.0
        waves = [v for k, v in by.items() if "k_assign_waves" in k]
        heavy = [v for k, v in by.items() if "k_assign_heavy" in k]
        w = statistics.median(waves[0]) if waves else 0.0
        h = statistics.median(heavy[0]) if heavy else 0.0
        out[name] = dict(assign_waves_bytes=w / calib, assign_heavy_bytes=h / calib, copy_scale=calib)
    total = sum(v["assign_waves_bytes"] + v["assign_heavy_bytes"] for v in out.values())
    res = dict(workload="geo2d hotspots n=1e6 d=2 k=1000", counters=out, bytes_per_step=total,
               assign_hip_sha256=assign_source_hash())
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(res, f, indent=1)
    return res


def main() -> int:
    if len(sys.argv) == 4 and sys.argv[1] == "--summarize-counters":
        print(json.dumps(summarize_counters(sys.argv[2], sys.argv[3]), indent=1))
        return 0
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="indexed timing only (for profiler runs)")
    ap.add_argument("--workload", choices=["geo2d", "surfaces3d"], default="geo2d",
                    help="geo2d: 1e6 x 2D, k=1000 (the metric); surfaces3d: 1e7 x 3D ellipsoid surfaces")
    ap.add_argument("--k", type=int, default=0, help="surfaces3d: number of centroids (default 10000)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): this build has no multi-GPU path; "
              "the sharding design is described in DESIGN.md", file=sys.stderr)
        return 2

    import torch

    import paper_2412_02244_amd as ekm
    from synth import make_config

    ekm.load_library()
    dev = torch.device("cuda:0")
    if args.workload == "geo2d":
        x, c0, cfg = make_config(1)
    else:
        x, c0, cfg = make_config(2, k=args.k or 10_000)
    n, d = x.shape
    k = c0.shape[0]
    K, W = args.steps, args.warmup
    log(f"workload n={n} d={d} k={k}; warmup {W}, timed {K} iterations")
    xt = torch.from_numpy(x).to(dev)
    c0t = torch.from_numpy(c0).to(dev)

    # warm-up: context creation and W iterations, then a fresh context for timing
    w = ekm.kmeans_init(xt, k, algo=ekm.KM_INDEXED)
    if W:
        time_steps(ekm, torch, w, c0t, W)
    w.close()
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx = ekm.kmeans_init(xt, k, algo=ekm.KM_INDEXED)
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t) * 1e3
    log(f"index build (Morton sort + leaves) {init_ms:.2f} ms wall")

    ms = time_steps(ekm, torch, ctx, c0t, K)
    ctx.close()
    ms_per_step = ms / K
    value = n / (ms_per_step * 1e-3)
    log(f"indexed: {ms_per_step * 1e3:.1f} us/iteration -> {value:.3e} point-assignments/s")

    # per-iteration counters (same iterations, separate untimed pass)
    sctx = ekm.kmeans_init(xt, k, algo=ekm.KM_INDEXED)
    c = c0t.clone()
    per_iter = []
    for _ in range(K):
        c, st = ekm.kmeans_step(sctx, c, stats=True)
        per_iter.append(st)
    L = per_iter[0]["leaves"]
    sctx.close()
    evals = sum(s["dist_evals"] for s in per_iter)
    brute_evals = sum(s["brute_evals"] for s in per_iter)
    single = sum(s["single_cand_points"] for s in per_iter)
    rechecked = sum(s["rechecked"] for s in per_iter)
    cand_total = sum(s["cand_total"] for s in per_iter) / K

    # per-phase GPU time with HIP events (same iterations, KM_FLAG_TIMING)
    tctx = ekm.kmeans_init(xt, k, algo=ekm.KM_INDEXED, flags=ekm.KM_FLAG_TIMING)
    time_steps(ekm, torch, tctx, c0t, K)
    phase_ms, nsteps = ekm.kmeans_phase_times(tctx)
    tctx.close()
    phase_us = {p: 1e3 * v / max(1, nsteps) for p, v in phase_ms.items()}
    log("phase us/iteration: " + ", ".join(f"{p} {v:.1f}" for p, v in phase_us.items()))

    dominant = max(phase_us, key=phase_us.get)
    bytes_dom = algorithmic_bytes(dominant, n, k, d, L)
    achieved = bytes_dom / (phase_us[dominant] * 1e-6) / 1e9
    kern = {"assign": "k_assign_waves + k_assign_heavy", "tree": "k_tree_small", "update": "k_finalize"}[dominant]
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 5),
                    traffic=measured_traffic() if dominant == "assign" and args.workload == "geo2d" else None,
                    kernel=kern,
                    kernel_us=round(phase_us[dominant], 2), algorithmic_bytes=bytes_dom)
    if args.copy_calib:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    out = {}
    if not args.quick:
        # brute-force GPU Lloyd (FP32 + FP64 recheck) on the same iterations
        b = ekm.kmeans_init(xt, k, algo=ekm.KM_BRUTE)
        time_steps(ekm, torch, b, c0t, 2)
        b.close()
        b = ekm.kmeans_init(xt, k, algo=ekm.KM_BRUTE)
        kb = min(K, 10)
        bms = time_steps(ekm, torch, b, c0t, kb) / kb
        b.close()
        out["brute_gpu"] = dict(value=n / (bms * 1e-3), ms_per_step=round(bms, 4), steps=kb,
                                speedup_indexed=round(bms / ms_per_step, 2))
        log(f"brute GPU: {bms * 1e3:.1f} us/iteration; indexed speedup {bms / ms_per_step:.1f}x")
    cpu = None
    if not args.no_cpu_baseline and not args.quick and args.workload == "geo2d":
        log("CPU oracle baseline ...")
        cpu = cpu_baseline(x, c0, args.cpu_seconds)
        log(f"oracle: {cpu['value']:.3e} point-assignments/s on {cpu['cores']} threads")

    line = {
        "metric": METRIC if args.workload == "geo2d" else
        f"point-assignments/s per Lloyd iter, 1e7x3D ellipsoid surfaces k={k}; indexed vs brute GPU",
        "value": value,
        "unit": "point-assignments/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"geo2d hotspots, n=1e6, d=2, k=1000" if args.workload == "geo2d" else
                                f"ellipsoid surfaces, n=1e7, d=3, k={k}") +
                               f", indexed FP32 + FP64 recheck, Lloyd iterations 1..{K}",
                   "n": n, "d": d, "k": k, "global_batch": n, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phase_us": {p: round(v, 2) for p, v in phase_us.items()},
        "index_build_ms": round(init_ms, 2),
        "pruned_fraction": round(1.0 - evals / brute_evals, 6),
        "single_candidate_point_fraction": round(single / (n * K), 4),
        "rechecked_points_per_iter": rechecked / K,
        "leaves": L,
        "candidates_total_per_iter": cand_total,
        **out,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
