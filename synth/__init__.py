"""Seeded synthetic inputs for the exact k-means hot path.

This module only draws random numbers: it holds none of the clustering
arithmetic, and both the oracle side and the GPU side read what it makes.
The paper evaluates on 2D GPS trajectory sets and 3D lidar / CAD point
clouds (experimental section, dataset table); none of those datasets is
available here, so the generators below produce inputs of the same shape
and structure:

* ``gaussian_mixture_2d``  - isotropic Gaussian blobs (small plain-Lloyd case)
* ``geo_hotspots_2d``      - Zipf-weighted hotspots over a uniform background,
                             the shape of city-scale GPS point sets
* ``ellipsoid_surfaces_3d``- noisy samples of ellipsoid surfaces, the shape of
                             scanned object / street point clouds
* ``batched_clouds``       - thousands of independent small clouds
* ``distortion_batch``     - equal-sized clouds for the differentiable loss

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64), samples in
float64 and rounds once to the requested storage dtype.
"""

from .gen import (  # noqa: F401
    CONFIGS,
    batched_clouds,
    distortion_batch,
    ellipsoid_surfaces_3d,
    gaussian_mixture_2d,
    geo_hotspots_2d,
    init_centroids,
    make_config,
    sha256_of,
)
