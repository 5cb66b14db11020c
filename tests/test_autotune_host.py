"""Host-side pieces of the autotuner (no GPU): cache keys, density
statistics and the density-preserving sample window."""
import math

import numpy as np
import torch

from paper_2502_11602_amd.autotune import Autotuner, compact_sample, tile_stats


def test_keys_bucket_size_density_and_aspect():
    k1 = Autotuner.key(100_000, 10.0, 1.0, 16)
    assert k1 == Autotuner.key(110_000, 10.5, 1.0, 16)
    assert k1 != Autotuner.key(400_000, 10.0, 1.0, 16)
    assert k1 != Autotuner.key(100_000, 40.0, 1.0, 16)
    assert k1 != Autotuner.key(100_000, 10.0, 2.0, 16)
    assert k1 == Autotuner.key(100_000, 10.0, 1.0, 16, aspect=1.2)
    assert k1 != Autotuner.key(100_000, 10.0, 1.0, 16, aspect=4.0)


def test_compact_sample_keeps_density():
    rng = np.random.default_rng(0)
    xyz = torch.from_numpy(np.c_[rng.uniform(0, 400, 400_000), rng.uniform(0, 100, 400_000),
                                 rng.uniform(0, 5, 400_000)])
    n, area, dens, ext = tile_stats(xyz)
    assert math.isclose(dens, 10.0, rel_tol=0.01)
    s = compact_sample(xyz, 50_000)
    sn, sa, sd, _ = tile_stats(s)
    assert 40_000 < sn < 60_000
    assert math.isclose(sd, dens, rel_tol=0.05)
    assert compact_sample(xyz[:1000], 50_000).shape[0] == 1000
