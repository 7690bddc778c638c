"""Seeded generators for the five k-means workloads (see package docstring).

Seeds: ``data_seed = 1000 + i`` and ``init_seed = 2000 + i`` for workload
index ``i`` (0..4).  Initial centroids are always the first ``k`` points of a
seeded permutation, upcast to float64 (the paper leaves initialisation to the
caller: Algorithm 1 only says centroids are initialised from k and D).
"""

from __future__ import annotations

import hashlib
import math

import numpy as np

# Workload table.  Sizes are the full ones; ``make_config`` can shrink n (and
# k with it) for tests that must finish in seconds.
CONFIGS = [
    dict(name="gauss2d_plain_fp64", d=2, n=10_000, k=100, iters=20, stop_when_stable=False,
         dtype="f64", algo="brute"),
    dict(name="geo2d_indexed", d=2, n=1_000_000, k=1000, iters=100, stop_when_stable=True,
         dtype="f32", algo="indexed"),
    dict(name="ellipsoids3d_indexed", d=3, n=10_000_000, k=(10_000, 100_000), iters=50,
         stop_when_stable=False, dtype="f32", algo="indexed"),
    dict(name="batched3d", d=3, clouds=4096, n_range=(1_000, 100_000), k_div=100, iters=30,
         dtype="f32", algo="indexed"),
    dict(name="distortion3d", d=3, clouds=256, n=16_384, k=512, dtype="f32"),
]


def sha256_of(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def init_centroids(x: np.ndarray, k: int, seed: int) -> np.ndarray:
    """First ``k`` rows of a seeded permutation of ``x``, as float64."""
    perm = np.random.default_rng(seed).permutation(x.shape[0])
    return np.ascontiguousarray(x[perm[:k]], dtype=np.float64)


def gaussian_mixture_2d(n: int, n_comp: int = 20, seed: int = 1000,
                        sigma_range=(0.005, 0.03), dtype=np.float64) -> np.ndarray:
    """Equal-weight mixture of isotropic 2D Gaussians, means U[0,1]^2."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(0.0, 1.0, (n_comp, 2))
    sig = rng.uniform(sigma_range[0], sigma_range[1], n_comp)
    comp = rng.integers(n_comp, size=n)
    x = means[comp] + sig[comp, None] * rng.standard_normal((n, 2))
    return np.ascontiguousarray(x.astype(dtype))


def geo_hotspots_2d(n: int, n_hot: int = 200, zipf_s: float = 1.1, hot_frac: float = 0.9,
                    sigma_range=(1e-3, 1e-2), seed: int = 1001, dtype=np.float32) -> np.ndarray:
    """City-like 2D point set: Zipf-weighted Gaussian hotspots plus uniform background.

    Hotspot r (rank 1..n_hot, ranks randomly assigned to hotspots) has weight
    proportional to r^-zipf_s; ``hot_frac`` of the points come from hotspots,
    the rest are uniform on [0,1]^2.  Counts are multinomial, order shuffled.
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(0.0, 1.0, (n_hot, 2))
    sig = rng.uniform(sigma_range[0], sigma_range[1], n_hot)
    w = np.arange(1, n_hot + 1, dtype=np.float64) ** (-zipf_s)
    w = w[rng.permutation(n_hot)]
    w /= w.sum()
    p = np.concatenate([hot_frac * w, [1.0 - hot_frac]])
    counts = rng.multinomial(n, p)
    lab = np.repeat(np.arange(n_hot), counts[:n_hot])
    hot = means[lab] + sig[lab, None] * rng.standard_normal((lab.size, 2))
    bg = rng.uniform(0.0, 1.0, (int(counts[-1]), 2))
    x = np.concatenate([hot, bg])[rng.permutation(n)]
    return np.ascontiguousarray(x.astype(dtype))


def _random_rotation(rng) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _ellipsoid_area(a: float, b: float, c: float) -> float:
    # Knud Thomsen's approximation (p = 1.6075, <= 1.1% error): only used to
    # split the point budget between ellipsoids.
    p = 1.6075
    return 4.0 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3.0) ** (1.0 / p)


def _ellipsoid_surface(rng, axes: np.ndarray, m: int) -> np.ndarray:
    """Area-uniform samples on the axis-aligned ellipsoid with semi-axes ``axes``.

    A direction v uniform on the unit sphere maps to diag(axes) v; the map's
    area element is proportional to ||(bc v_x, ac v_y, ab v_z)||, so accepting
    with probability (that norm / its maximum) makes the accepted points
    area-uniform.
    """
    a, b, c = axes
    scale = np.array([b * c, a * c, a * b])
    gmax = scale.max()
    out, got = [], 0
    while got < m:
        draw = max(64, int((m - got) * 2.5))
        v = rng.standard_normal((draw, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        g = np.linalg.norm(v * scale, axis=1)
        keep = rng.uniform(0.0, gmax, draw) < g
        v = v[keep]
        out.append(v * axes)
        got += v.shape[0]
    return np.concatenate(out)[:m]


def ellipsoid_surfaces_3d(n: int, n_ell: int = 50, seed: int = 1002, noise: float = 0.002,
                          axes_range=(0.02, 0.2), dtype=np.float32, rng=None) -> np.ndarray:
    """Noisy surface samples of ``n_ell`` randomly rotated ellipsoids in [0,1]^3."""
    rng = np.random.default_rng(seed) if rng is None else rng
    centers = rng.uniform(0.0, 1.0, (n_ell, 3))
    axes = rng.uniform(axes_range[0], axes_range[1], (n_ell, 3))
    rots = [_random_rotation(rng) for _ in range(n_ell)]
    areas = np.array([_ellipsoid_area(*ax) for ax in axes])
    counts = rng.multinomial(n, areas / areas.sum())
    parts = []
    for e in range(n_ell):
        if counts[e] == 0:
            continue
        s = _ellipsoid_surface(rng, axes[e], int(counts[e]))
        parts.append(s @ rots[e].T + centers[e])
    x = np.concatenate(parts)
    x += noise * rng.standard_normal(x.shape)
    x = x[rng.permutation(n)]
    return np.ascontiguousarray(x.astype(dtype))


def batched_clouds(n_clouds: int = 4096, seed: int = 1003, n_range=(1_000, 100_000),
                   ell_range=(1, 5), k_div: int = 100, init_seed: int = 2003):
    """Many independent 3D clouds, sizes log-uniform in ``n_range``.

    Returns ``(points f32 [N,3], pt_offs int64 [B+1], c0 f64 [K,3], c_offs int64 [B+1])``
    with ``k_i = max(1, n_i // k_div)`` and per-cloud initial centroids taken
    as the first k_i points of a seeded permutation of that cloud.
    """
    rng = np.random.default_rng(seed)
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    sizes = np.rint(np.exp(rng.uniform(lo, hi, n_clouds))).astype(np.int64)
    n_ells = rng.integers(ell_range[0], ell_range[1] + 1, n_clouds)
    cloud_seeds = rng.integers(0, 2**63 - 1, n_clouds)
    init_rng = np.random.default_rng(init_seed)
    pts, cs = [], []
    k_sizes = np.maximum(1, sizes // k_div)
    for i in range(n_clouds):
        x = ellipsoid_surfaces_3d(int(sizes[i]), int(n_ells[i]), seed=int(cloud_seeds[i]))
        perm = init_rng.permutation(x.shape[0])
        pts.append(x)
        cs.append(x[perm[:k_sizes[i]]].astype(np.float64))
    pt_offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    c_offs = np.concatenate([[0], np.cumsum(k_sizes)]).astype(np.int64)
    return (np.ascontiguousarray(np.concatenate(pts)), pt_offs,
            np.ascontiguousarray(np.concatenate(cs)), c_offs)


def distortion_batch(n_clouds: int = 256, n: int = 16_384, k: int = 512, seed: int = 1004,
                     init_seed: int = 2004, jitter: float = 0.01):
    """Equal-sized 3D clouds and per-cloud centroids for the distortion loss.

    Centroids are the first k points of a seeded permutation of each cloud plus
    N(0, jitter^2) noise (so that no centroid sits exactly on a data point).
    Returns float32 ``x [B,n,3]`` and ``c [B,k,3]``.
    """
    rng = np.random.default_rng(seed)
    init_rng = np.random.default_rng(init_seed)
    n_ells = rng.integers(1, 6, n_clouds)
    cloud_seeds = rng.integers(0, 2**63 - 1, n_clouds)
    xs, cs = [], []
    for i in range(n_clouds):
        x = ellipsoid_surfaces_3d(n, int(n_ells[i]), seed=int(cloud_seeds[i]), dtype=np.float64)
        perm = init_rng.permutation(n)
        c = x[perm[:k]] + jitter * init_rng.standard_normal((k, 3))
        xs.append(x)
        cs.append(c)
    return (np.ascontiguousarray(np.stack(xs).astype(np.float32)),
            np.ascontiguousarray(np.stack(cs).astype(np.float32)))


def make_config(i: int, n: int | None = None, k: int | None = None):
    """Points and initial centroids for single-cloud workload ``i`` (0, 1 or 2).

    ``n``/``k`` override the full sizes for quick tests; the generators and
    seeds are unchanged.  Returns ``(x, c0, meta)``.
    """
    cfg = dict(CONFIGS[i])
    data_seed, init_seed = 1000 + i, 2000 + i
    if i == 0:
        n = n or cfg["n"]
        k = k or cfg["k"]
        x = gaussian_mixture_2d(n, seed=data_seed)
    elif i == 1:
        n = n or cfg["n"]
        k = k or cfg["k"]
        x = geo_hotspots_2d(n, seed=data_seed)
    elif i == 2:
        n = n or cfg["n"]
        k = k or cfg["k"][0]
        x = ellipsoid_surfaces_3d(n, seed=data_seed)
    else:
        raise ValueError("make_config covers the single-cloud workloads 0..2")
    c0 = init_centroids(x, k, init_seed)
    cfg.update(n=n, k=k, data_seed=data_seed, init_seed=init_seed)
    return x, c0, cfg
