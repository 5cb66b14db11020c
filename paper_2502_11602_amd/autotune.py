"""Per-tile voxel-edge autotuner.

The paper names automatic cell-size selection as future work (Section 6) and
shows the edge is the key performance parameter, interacting with the search
radius (Section 5.1).  This tuner picks, per tile, the voxel edge s = f * r
(f from a small candidate set, or f * the k-NN radius estimate) and the
flavor by *timing the library's own kernels* -- radius count + fill at r and
k-NN at k -- on a spatially compact sample of the tile that keeps its point
density.  Decisions are cached in a JSON file keyed by the tile's size and
density buckets, r and k, so repeated batches reuse them."""
import json
import math
import os
import time

import torch

from .index import GridIndex

FACTORS = (0.5, 0.75, 1.0, 1.5, 2.0)
SAMPLE_POINTS = 200_000
DENSE_VOXEL_BUDGET = 1 << 27  # dense flavor while the grid has fewer voxels


def _bucket(v, step=0.5):
    return round(math.log2(max(v, 1e-9)) / step) * step


def tile_stats(xyz):
    """(points, xy area in m^2, density in points/m^2) of a float64 tile."""
    lo = xyz.min(0).values
    hi = xyz.max(0).values
    ext = (hi - lo).tolist()
    area = max(ext[0], 1e-3) * max(ext[1], 1e-3)
    return xyz.shape[0], area, xyz.shape[0] / area, ext


def compact_sample(xyz, npts=SAMPLE_POINTS):
    """A square window of the tile around its centre holding about npts
    points (keeps the local density and structure)."""
    n = xyz.shape[0]
    if n <= npts:
        return xyz
    lo = xyz[:, :2].min(0).values
    hi = xyz[:, :2].max(0).values
    c = (lo + hi) / 2
    half = (hi - lo) / 2 * math.sqrt(npts / n)
    m = ((xyz[:, 0] - c[0]).abs() <= half[0]) & ((xyz[:, 1] - c[1]).abs() <= half[1])
    return xyz[m].contiguous()


class Autotuner:
    def __init__(self, cache_path=None, repeats=3):
        self.cache_path = cache_path or os.environ.get(
            "CHS_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "chs_autotune.json"))
        self.repeats = repeats
        self.cache = {}
        if os.path.exists(self.cache_path):
            try:
                with open(self.cache_path) as fh:
                    self.cache = json.load(fh)
            except (OSError, ValueError):
                self.cache = {}
        self.trials = []

    def save(self):
        d = os.path.dirname(self.cache_path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    @staticmethod
    def key(n, density, r, k):
        return f"n{_bucket(n, 1.0)}_d{_bucket(density)}_r{r:g}_k{k}"

    def _time(self, sample, cell, flavor, r, k):
        ix = GridIndex(sample, cell=cell, flavor=flavor)
        best = math.inf
        for _ in range(self.repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            off, tot = ix.radius_count(r)
            ix.radius_fill(r, off, tot)
            ix.knn(k)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        ix.close()
        return best

    def tune(self, xyz, r, k):
        """Best (cell, flavor) for a tile (float64 [n,3] CUDA tensor)."""
        n, area, dens, ext = tile_stats(xyz)
        key = self.key(n, dens, r, k)
        if key in self.cache:
            e = self.cache[key]
            return e["cell"], e["flavor"]
        sample = compact_sample(xyz)
        # k-NN radius estimate on a surface of this density
        rk = math.sqrt(k / (math.pi * dens))
        cands = sorted({round(f * r, 4) for f in FACTORS} | {round(f * rk, 4) for f in (1.0, 2.0)})
        best = (math.inf, None, None)
        for cell in cands:
            vox = 1.0
            for e in ext:
                vox *= math.floor(e / cell) + 1
            flavor = "dense" if vox < DENSE_VOXEL_BUDGET else "sparse"
            t = self._time(sample, cell, flavor, r, k)
            self.trials.append(dict(key=key, cell=cell, flavor=flavor, seconds=t))
            if t < best[0]:
                best = (t, cell, flavor)
        self.cache[key] = {"cell": best[1], "flavor": best[2], "seconds": best[0],
                           "sample_points": int(sample.shape[0])}
        return best[1], best[2]

    def choose(self, tiles, r, k):
        """Per-tile voxel edges for a batch (list of float64 CUDA tensors).
        A batch has one flavor: dense while the concatenated grid stays
        within the dense budget and every tile chose dense, else sparse."""
        cells, flavors, total = [], [], 0.0
        for t in tiles:
            c, f = self.tune(t, r, k)
            cells.append(c)
            flavors.append(f)
            vox = 1.0
            for e in tile_stats(t)[3]:
                vox *= math.floor(e / c) + 1
            total += vox
        dense = "sparse" not in flavors and total < 4 * DENSE_VOXEL_BUDGET
        return cells, ("dense" if dense else "sparse")
