#!/usr/bin/env python3
"""Write tests/golden/surfaces3d_1e7_oracle.json: digests of the FP64
oracle's Lloyd trajectory on the 1e7-point 3D ellipsoid-surface workload.

The oracle needs minutes per iteration at this size (brute force over k = 1e4
and 1e5 centroids), too long for a test run, so its trajectory is computed
once here and stored as SHA-256 digests of every iteration's assignment
(int32, caller order) and centroids (float64, row-major), plus the per
iteration count of changed assignments and a few plain values for
diagnostics.  Only ``oracle`` and the seeded generators are called.

Usage:  python tests/golden/make_surfaces3d_oracle.py [--iters-small 3] [--iters-large 2]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from synth import init_centroids, make_config, sha256_of  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "surfaces3d_1e7_oracle.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def run(x: np.ndarray, k: int, iters: int) -> dict:
    c0 = init_centroids(x, k, 2002)
    t0 = time.time()
    ref = oracle.lloyd(x, c0, max_iter=iters, stop_when_stable=False)
    steps = []
    for t in range(ref["iters"]):
        a, c = ref["a_hist"][t], ref["c_hist"][t]
        prev = ref["a_hist"][t - 1] if t else None
        steps.append(dict(
            iteration=t + 1,
            assign_sha256=digest(a.astype(np.int32)),
            centroids_sha256=digest(c.astype(np.float64)),
            n_changed=int(x.shape[0] if prev is None else (a != prev).sum()),
            sse=float(ref["sse"][t]),
            assign_head=[int(v) for v in a[:16]],
            centroid0=[float(v) for v in c[0]],
        ))
    return dict(k=k, c0_sha256=digest(c0), iters=ref["iters"], seconds=round(time.time() - t0, 1),
                oracle_threads=oracle.num_threads(), steps=steps)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters-small", type=int, default=3)
    ap.add_argument("--iters-large", type=int, default=2)
    args = ap.parse_args()
    x, _, cfg = make_config(2)
    out = dict(workload="ellipsoid surfaces n=1e7 d=3 (data seed 1002, init seed 2002)",
               n=int(x.shape[0]), data_sha256=sha256_of(x), runs=[])
    for k, iters in ((10_000, args.iters_small), (100_000, args.iters_large)):
        print(f"k={k}: {iters} oracle iterations ...", flush=True)
        out["runs"].append(run(x, k, iters))
        print(f"k={k}: done in {out['runs'][-1]['seconds']} s", flush=True)
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1)
    print(f"wrote {OUT}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
