"""Seeded synthetic LiDAR clouds that stand in for the paper's datasets.

The paper measures on public ALS / MLS / ULS / TLS datasets (Section 4.1,
Table 1) that are not available here.  These generators produce procedural
clouds with the same structure (terrain, buildings, vegetation with multiple
returns, range-dependent TLS density) from a numpy PCG64 generator, so that the
oracle and the GPU path read the very same FP64 coordinates.

This module draws random numbers only: it holds none of the index's
arithmetic (no grid, keys, distances or search) and is imported by both the
oracle-side tests and the GPU-side binding tests.
"""
from .als import (  # noqa: F401
    terrain_params,
    terrain_height,
    als_cloud,
    config0,
    config1,
    config3_tiles,
    config4,
    small_als,
)
from .tls import tls_cloud, config2  # noqa: F401
from .uniform import uniform_cube  # noqa: F401
