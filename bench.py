#!/usr/bin/env python3
"""Benchmark of the exact k-means hot path on one MI355X.

Headline workload: 1e6 2D geo-like points (Zipf-weighted Gaussian hotspots
plus a uniform background, the shape of the paper's GPS trajectory data
sets), k = 1000, centroids initialised from a seeded permutation.  One step
= one Lloyd iteration (centroid tree with inter bounds, leaf candidates,
assignment with FP64 recheck, exact centroid update).  The timed region is
one kmeans_run call on a fresh context, iterations 1..T (T = --steps, 100 by
default, stopping early only if the assignment becomes stable), inputs
already in HBM; `ms_per_step` is its GPU time divided by T.  A second,
identical run with per-phase HIP events gives the per-iteration series, its
median over iterations 2..T and iteration 1 on its own.

Further legs (skipped with --quick): brute-force GPU Lloyd on the same
iterations, a plain device copy (the measured HBM ceiling), the 1e7 3D
ellipsoid-surface workload at k = 1e4 and 1e5, the distortion loss forward
and backward at 256 clouds x 16,384 points, and the FP64 CPU oracle on a
bounded sample.

Prints ONE JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "point-assignments/s per Lloyd iter, 1e6×2D k=1e3; indexed vs brute GPU"
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(phase: str, n: int, k: int, d: int) -> float:
    """Bytes each phase must move per launch: per-unit figure x units."""
    if phase in ("assign", "deferred"):
        return n * (4 * d + 8)            # read point, read + write its assignment
    if phase == "tree":
        return k * (8 * d * 2 + 16 + 16 + 8)  # FP64 centroid and previous centroid in; fl32, tree copy, bounds out
    return k * (8 * d * 2 + 16 * d + 4)   # FP64 in/out, exact sums and counts


KERNEL_OF_PHASE = {"tree": "k_tree_small", "assign": "k_assign_waves", "deferred": "k_assign_heavy",
                   "update": "k_finalize"}


def gpu_ms(torch, fn) -> float:
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    r = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), r


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "assign_geo2d_1e6_k1000_traffic.json")


def assign_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2412_02244_amd", "csrc", "assign.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic():
    """HBM bytes per k_assign_waves launch from the committed counter summary,
    or None if the assignment kernels changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("assign_hip_sha256") != assign_source_hash():
        return None
    return t.get("assign_waves_bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(x, c0, target_s: float):
    """The oracle as it stands, on a bounded sample of the same run: as many
    iterations from the start as fit in about target_s seconds, on every
    host thread; and one iteration of a 100k-point subset on one thread."""
    import oracle
    t = time.perf_counter()
    oracle.lloyd(x, c0, max_iter=1, history=False)
    t1 = time.perf_counter() - t
    iters = int(max(1, min(100, target_s / max(t1, 1e-6))))
    t = time.perf_counter()
    oracle.lloyd(x, c0, max_iter=iters, history=False)
    dt = time.perf_counter() - t
    one = None
    code = ("import sys,time; sys.path.insert(0,%r); import numpy as np, oracle; "
            "x=np.load(sys.argv[1]); c=np.load(sys.argv[2]); oracle.lloyd(x[:1000], c, 1, history=False); "
            "t=time.perf_counter(); oracle.lloyd(x, c, 1, history=False); print(time.perf_counter()-t)") % ROOT
    try:
        import numpy as np
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            xs, cs = os.path.join(td, "x.npy"), os.path.join(td, "c.npy")
            np.save(xs, x[:100_000])
            np.save(cs, c0)
            r = subprocess.run([sys.executable, "-c", code, xs, cs], capture_output=True, text=True, timeout=300,
                               env=dict(os.environ, OMP_NUM_THREADS="1"))
            if r.returncode == 0:
                one = 100_000 / float(r.stdout.strip().splitlines()[-1])
    except Exception as e:  # the single-core figure is context only
        log(f"one-core oracle timing failed: {e}")
    return dict(value=x.shape[0] * iters / dt, unit="point-assignments/s", cores=oracle.num_threads(),
                kind="oracle", cpu_model=cpu_model(), one_core_value=one,
                sample=f"Lloyd iterations 1..{iters} of the same 1e6x2D k=1000 run (FP64 brute force, "
                       f"{dt:.1f} s on the host); one_core_value: iteration 1 on the first 100k points, "
                       f"OMP_NUM_THREADS=1")


def copy_ceiling(torch, dev) -> dict:
    """A plain device-to-device copy of 512 MiB: the HBM bandwidth this
    box reaches in practice (bytes read + written / time)."""
    src = torch.empty(128 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(5):
        ms, _ = gpu_ms(torch, lambda: dst.copy_(src))
        best = ms if best is None else min(best, ms)
    nbytes = 2 * src.numel() * 4
    return dict(gbs=round(nbytes / (best * 1e-3) / 1e9, 1), bytes=nbytes, ms=round(best, 4))


def run_indexed(ekm, torch, xt, c0t, k, steps, stop, flags=0):
    ctx = ekm.kmeans_init(xt, k, algo=ekm.KM_INDEXED, flags=flags)
    c = c0t.clone()
    ms, (it, _) = gpu_ms(torch, lambda: ekm.kmeans_run(ctx, c, steps, stop_when_stable=stop))
    return ctx, ms, it


def series(ekm, torch, xt, c0t, k, steps, stop):
    """Per-iteration GPU times (sum of the phases) from a KM_FLAG_TIMING run."""
    ctx, _, it = run_indexed(ekm, torch, xt, c0t, k, steps, stop, flags=ekm.KM_FLAG_TIMING)
    per = ekm.kmeans_step_times(ctx, cap=it)
    ctx.close()
    return per


def leg_surfaces(ekm, torch, dev, quick_iters=None) -> dict:
    from synth import init_centroids, make_config
    x, _, _ = make_config(2)
    xt = torch.from_numpy(x).to(dev)
    n = x.shape[0]
    out = {}
    for k, iters in ((10_000, 50), (100_000, 50)):
        if quick_iters:
            iters = quick_iters
        c0t = torch.from_numpy(init_centroids(x, k, 2002)).to(dev)
        ctx, ms, it = run_indexed(ekm, torch, xt, c0t, k, iters, False)
        ctx.close()
        b = ekm.kmeans_init(xt, k, algo=ekm.KM_BRUTE)
        c = c0t.clone()
        kb = 2
        bms, _ = gpu_ms(torch, lambda: ekm.kmeans_run(b, c, kb))
        b.close()
        per = ms / it
        out[f"k={k}"] = dict(iterations=it, ms_per_iter=round(per, 4), value=n / (per * 1e-3),
                             brute_ms_per_iter=round(bms / kb, 3), speedup_vs_brute=round(bms / kb / per, 2))
        log(f"surfaces3d 1e7 k={k}: {per:.3f} ms/iteration ({it} iterations), brute {bms / kb:.2f} ms, "
            f"{bms / kb / per:.1f}x")
    return dict(workload="ellipsoid surfaces, n=1e7, d=3, indexed FP32 + FP64 recheck, Lloyd iterations 1..T",
                **out)


def leg_distortion(ekm, torch, dev) -> dict:
    from synth import distortion_batch
    xb, cb = distortion_batch()
    xt = torch.from_numpy(xb).to(dev)
    ct = torch.from_numpy(cb).to(dev)
    g = torch.ones(xb.shape[0], dtype=torch.float64, device=dev)

    def step():
        a, loss = ekm.distortion_fwd(xt, ct)
        return ekm.distortion_bwd(xt, ct, a, g)

    step()
    reps = 5
    ms, _ = gpu_ms(torch, lambda: [step() for _ in range(reps)])
    per = ms / reps
    pts = xb.shape[0] * xb.shape[1]
    log(f"distortion fwd+bwd B={xb.shape[0]} n={xb.shape[1]} k={cb.shape[1]}: {per:.3f} ms")
    return dict(workload="distortion loss forward + backward, 256 clouds x 16384 3D points, k=512, FP32 with "
                         "FP64 accumulation", ms_per_fwd_bwd=round(per, 4), points_per_s=pts / (per * 1e-3))


def leg_batched(ekm, torch, dev) -> dict:
    from synth import batched_clouds
    t0 = time.time()
    x, po, c0, co = batched_clouds()
    log(f"batched: {len(po) - 1} clouds, {x.shape[0]} points, {c0.shape[0]} centroids "
        f"(generated in {time.time() - t0:.0f} s)")
    xt = torch.from_numpy(x).to(dev)
    c0t = torch.from_numpy(c0).to(dev)
    iters = 30
    c = c0t.clone()
    tune_ms, (f, G) = gpu_ms(torch, lambda: ekm.kmeans_run_batched(xt, po, c, co, 1))
    c = c0t.clone()
    total_ms, _ = gpu_ms(torch, lambda: ekm.kmeans_run_batched(xt, po, c, co, iters))
    init_ms, ctx = gpu_ms(torch, lambda: ekm.kmeans_init_batched(xt, po, co, leaf_size=f, cand_tile=G))
    c = c0t.clone()
    run_ms, (it, _) = gpu_ms(torch, lambda: ekm.kmeans_run(ctx, c, iters))
    ctx.close()
    n = x.shape[0]
    per = run_ms / it
    log(f"batched: leaf size {f}, leaves per list {G}; {per:.3f} ms/iteration, index build {init_ms:.1f} ms, "
        f"kmeans_run_batched {total_ms:.1f} ms for {iters} iterations")
    return dict(workload="4096 3D ellipsoid-surface clouds, sizes log-uniform in [1e3,1e5], k_i=n_i/100, "
                         "indexed FP32 + FP64 recheck, 30 iterations, one context",
                clouds=len(po) - 1, points=n, centroids=int(c0.shape[0]), iterations=it, leaf_size=f,
                leaves_per_list=G, ms_per_iter=round(per, 4), value=n / (per * 1e-3),
                index_build_ms=round(init_ms, 2), run_batched_ms=round(total_ms, 2),
                run_batched_value=n * iters / (total_ms * 1e-3), first_call_with_tuning_ms=round(tune_ms, 2))


def summarize_counters(fetch_csv: str, write_csv: str) -> dict:
    """HBM bytes per k_assign_waves launch from two rocprofv3 --pmc runs of
    `bench.py --quick --copy-calib` (FETCH_SIZE, then WRITE_SIZE, in KiB per
    dispatch).  Each counter is scaled by what it reads for the 512 MiB
    device copy of the same run (expected: 512 MiB fetched, 512 MiB
    written)."""
    import csv

    copy_bytes = float(512 << 20)

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        by = {}
        for r in rows:
            by.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return by

    out = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        by = per_kernel(path, name)
        copies = [max(v) for kname, v in by.items() if "copy" in kname.lower() and "ekm" not in kname]
        calib = max(copies) / copy_bytes if copies else 1.0
        per = {}
        for kname, v in by.items():
            for short in KERNEL_OF_PHASE.values():
                if short in kname:
                    per[short] = statistics.median(v) / calib
        out[name] = dict(per_launch_bytes=per, copy_scale=calib)
    waves = sum(out[c]["per_launch_bytes"].get("k_assign_waves", 0.0) for c in out)
    res = dict(workload="geo2d hotspots n=1e6 d=2 k=1000", counters=out, assign_waves_bytes_per_launch=waves,
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
    ap.add_argument("--steps", type=int, default=100, help="Lloyd iterations timed (until stable, at most this)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline timing only (for profiler runs)")
    ap.add_argument("--only", choices=("surfaces", "distortion", "batched"),
                    help="run one further leg alone and print its JSON (for profiler runs)")
    ap.add_argument("--leg-iters", type=int, default=None,
                    help="iterations of the surfaces leg with --only (default: its full count)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run the plain device copy (calibrates HBM byte counters) in --quick mode")
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
    if args.only:
        leg = {"surfaces": lambda: leg_surfaces(ekm, torch, dev, quick_iters=args.leg_iters),
               "distortion": lambda: leg_distortion(ekm, torch, dev),
               "batched": lambda: leg_batched(ekm, torch, dev)}[args.only]()
        print(json.dumps(leg))
        return 0
    x, c0, cfg = make_config(1)
    n, d = x.shape
    k = c0.shape[0]
    K, W = args.steps, args.warmup
    log(f"workload n={n} d={d} k={k}; warmup {W}, timed: iterations 1..{K} until stable")
    xt = torch.from_numpy(x).to(dev)
    c0t = torch.from_numpy(c0).to(dev)

    # warm-up: a context and W iterations (kernels loaded, clocks up), then a fresh context
    if W:
        w, _, _ = run_indexed(ekm, torch, xt, c0t, k, W, False)
        w.close()
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx = ekm.kmeans_init(xt, k, algo=ekm.KM_INDEXED)
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t) * 1e3
    ctx.close()
    log(f"index build (Morton sort + leaves) {init_ms:.2f} ms wall")

    ctx, ms, T = run_indexed(ekm, torch, xt, c0t, k, K, True)
    ctx.close()
    ms_per_step = ms / T
    value = n / (ms_per_step * 1e-3)
    log(f"indexed: {T} iterations, {ms_per_step * 1e3:.1f} us/iteration -> {value:.3e} point-assignments/s")

    # per-iteration series (same run, HIP events at the phase boundaries)
    per = series(ekm, torch, xt, c0t, k, K, True)
    tot_us = [1e3 * sum(p.values()) for p in per]
    med_2T = statistics.median(tot_us[1:]) if len(tot_us) > 1 else tot_us[0]
    phase_mean_us = {p: 1e3 * statistics.mean(s[p] for s in per) for p in ekm.PHASES}
    phase_med_us = {p: 1e3 * statistics.median(s[p] for s in per[1:] or per) for p in ekm.PHASES}
    log(f"per-iteration: iteration 1 {tot_us[0]:.1f} us, median of 2..{len(tot_us)} {med_2T:.1f} us")
    log("phase mean us/iteration: " + ", ".join(f"{p} {v:.1f}" for p, v in phase_mean_us.items()))

    # per-iteration counters (same iterations, separate pass)
    sctx = ekm.kmeans_init(xt, k, algo=ekm.KM_INDEXED)
    c = c0t.clone()
    _, stats = ekm.kmeans_run(sctx, c, K, stop_when_stable=True, per_iter=True)
    sctx.close()
    Ts = len(stats)
    evals = sum(s["dist_evals"] for s in stats)
    brute_evals = sum(s["brute_evals"] for s in stats)

    dominant = max(phase_mean_us, key=phase_mean_us.get)
    bytes_dom = algorithmic_bytes(dominant, n, k, d)
    achieved = bytes_dom / (phase_mean_us[dominant] * 1e-6) / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 5),
                    traffic=measured_traffic() if dominant == "assign" else None,
                    kernel=KERNEL_OF_PHASE[dominant], kernel_us=round(phase_mean_us[dominant], 2),
                    algorithmic_bytes=bytes_dom,
                    pruned_fraction=round(1.0 - evals / brute_evals, 6))

    out = {}
    if args.copy_calib or not args.quick:
        out["copy_ceiling"] = copy_ceiling(torch, dev)
        log(f"device copy: {out['copy_ceiling']['gbs']} GB/s")
    if not args.quick:
        b = ekm.kmeans_init(xt, k, algo=ekm.KM_BRUTE)
        ekm.kmeans_run(b, c0t.clone(), 2)
        b.close()
        b = ekm.kmeans_init(xt, k, algo=ekm.KM_BRUTE)
        kb = min(K, 10)
        c = c0t.clone()
        bms, _ = gpu_ms(torch, lambda: ekm.kmeans_run(b, c, kb))
        b.close()
        bms /= kb
        out["brute_gpu"] = dict(value=n / (bms * 1e-3), ms_per_step=round(bms, 4), steps=kb,
                                speedup_indexed=round(bms / ms_per_step, 2),
                                speedup_indexed_median_2_T=round(bms / (med_2T * 1e-3), 2))
        log(f"brute GPU: {bms * 1e3:.1f} us/iteration; indexed speedup {bms / ms_per_step:.1f}x "
            f"(median of 2..T: {bms / (med_2T * 1e-3):.1f}x)")
        out["surfaces3d_1e7"] = leg_surfaces(ekm, torch, dev)
        out["distortion_256x16384"] = leg_distortion(ekm, torch, dev)
        out["batched3d_4096"] = leg_batched(ekm, torch, dev)
    cpu = None
    if not args.no_cpu_baseline and not args.quick:
        log("CPU oracle baseline ...")
        cpu = cpu_baseline(x, c0, args.cpu_seconds)
        log(f"oracle: {cpu['value']:.3e} point-assignments/s on {cpu['cores']} threads ({cpu['cpu_model']})")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "point-assignments/s",
        "n_gpus": 1,
        "steps": T,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"geo2d hotspots, n=1e6, d=2, k=1000, indexed FP32 + FP64 recheck, Lloyd "
                               f"iterations 1..{T} (until stable or {K})",
                   "n": n, "d": d, "k": k, "global_batch": n, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "iter1_us": round(tot_us[0], 2),
        "median_iter_us_2_T": round(med_2T, 2),
        "value_median_2_T": n / (med_2T * 1e-6),
        "iter_series_us": [round(v, 1) for v in tot_us],
        "phase_mean_us": {p: round(v, 2) for p, v in phase_mean_us.items()},
        "phase_median_us_2_T": {p: round(v, 2) for p, v in phase_med_us.items()},
        "index_build_ms": round(init_ms, 2),
        "pruned_fraction": round(1.0 - evals / brute_evals, 6),
        "per_iter_counts": {f: [s[f] for s in stats] for f in
                            ("n_changed", "inter_leaf_points", "inter_points", "single_cand_points",
                             "dist_evals", "rechecked", "deferred_leaves", "groups_skipped")},
        "leaves": stats[0]["leaves"],
        "iterations_counted": Ts,
        **out,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
