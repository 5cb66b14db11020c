"""Per-tile autotuner: voxel edge, flavor and query-tile size.

The paper names automatic cell-size selection as future work (Section 6) and
shows the edge is the key performance parameter, interacting with the search
radius (Section 5.1).  This tuner picks, per tile, the voxel edge s = f * r
(f from a small candidate set, or f * the k-NN radius estimate), the flavor
(dense, sparse, mixed) and the radius search's query-tile size (64-query
tiles or 8-query groups) by *timing the library's own kernels* -- build,
radius count + fill at r and k-NN at k -- on a spatially compact sample of the
tile that keeps its point density.  Edges and flavors are timed together,
then both query-tile sizes at the winner.  Decisions are cached in a JSON
file keyed by the tile's size, density and extent-aspect buckets, r and k,
so repeated batches reuse them; every decision is one of the timed trials
(the trials are kept in ``trials``)."""
import json
import math
import os
import time

import torch

from .index import GridIndex

FACTORS = (0.5, 0.75, 1.0, 1.5, 2.0)
SAMPLE_POINTS = 200_000
DENSE_VOXEL_BUDGET = 1 << 27  # the dense flavor is tried while the grid has fewer voxels
SCHEDULES = {"tiles": 64, "groups": 8}  # query-tile size of each radius schedule


def _bucket(v, step=0.5):
    return round(math.log2(max(v, 1e-9)) / step) * step


def tile_stats(xyz):
    """(points, xy area in m^2, density in points/m^2, extent) of a float64 tile."""
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


def _voxels(ext, cell):
    v = 1.0
    for e in ext:
        v *= math.floor(e / cell) + 1
    return v


class Autotuner:
    def __init__(self, cache_path=None, repeats=3, flavors=("dense", "sparse", "mixed")):
        self.cache_path = cache_path or os.environ.get(
            "CHS_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "chs_autotune.json"))
        self.repeats = repeats
        self.flavors = tuple(flavors)
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
    def key(n, density, r, k, aspect=1.0):
        return (f"n{_bucket(n, 1.0)}_d{_bucket(density)}_a{_bucket(max(aspect, 1.0), 1.0)}"
                f"_r{r:g}_k{k}")

    def _time(self, sample, cell, flavor, sched, r, k):
        """Best of `repeats` times of build + radius count + fill + k-NN on
        the sample (seconds)."""
        best = math.inf
        for _ in range(self.repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ix = GridIndex(sample, cell=cell, flavor=flavor)
            ix.set_radius_schedule(sched)
            off, tot = ix.radius_count(r)
            ix.radius_fill(r, off, tot)
            ix.knn(k)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
            ix.close()
        return best

    def _trial(self, key, sample, cell, flavor, sched, r, k):
        t = self._time(sample, cell, flavor, sched, r, k)
        self.trials.append(dict(key=key, cell=cell, flavor=flavor, schedule=sched,
                                query_tile=SCHEDULES.get(sched), seconds=t))
        return t

    def tune(self, xyz, r, k, flavors=None):
        """The best (cell, flavor, schedule) for a tile (float64 [n,3] CUDA
        tensor) and the sample's time of each schedule at that edge and
        flavor, {schedule: seconds per sample point}."""
        flavors = tuple(flavors or self.flavors)
        n, area, dens, ext = tile_stats(xyz)
        aspect = max(ext[0], 1e-3) / max(ext[1], 1e-3)
        key = self.key(n, dens, r, k, aspect if aspect >= 1 else 1 / aspect) + \
            "_f" + "".join(f[0] for f in flavors)
        if key in self.cache:
            e = self.cache[key]
            return e["cell"], e["flavor"], e["schedule"], e["sched_cost"]
        sample = compact_sample(xyz)
        ns = int(sample.shape[0])
        _, _, _, sext = tile_stats(sample)
        # k-NN radius estimate on a surface of this density
        rk = math.sqrt(k / (math.pi * dens))
        cands = sorted({round(f * r, 4) for f in FACTORS} | {round(f * rk, 4) for f in (1.0, 2.0)})
        best = (math.inf, None, None)
        for cell in cands:
            for fl in flavors:
                if fl == "dense" and _voxels(ext, cell) >= DENSE_VOXEL_BUDGET:
                    continue
                t = self._trial(key, sample, cell, fl, "auto", r, k)
                if t < best[0]:
                    best = (t, cell, fl)
        _, cell, fl = best
        cost = {s: self._trial(key, sample, cell, fl, s, r, k) / ns for s in SCHEDULES}
        sched = min(cost, key=cost.get)
        self.cache[key] = {"cell": cell, "flavor": fl, "schedule": sched, "sched_cost": cost,
                           "query_tile": SCHEDULES[sched], "seconds": cost[sched] * ns,
                           "sample_points": ns}
        return cell, fl, sched, cost

    def choose(self, tiles, r, k):
        """Per-tile voxel edges, and the flavor and radius schedule of a batch
        (list of float64 CUDA tensors).  A batched index has one flavor and
        one schedule: the flavor is the one most tiles chose (by points;
        dense only while the concatenated grid stays within the dense
        budget); the schedule minimises the tiles' summed estimated time (the
        sample's time per point at each schedule times the tile's points)."""
        cells, fl_pts, sched_cost, total_vox = [], {}, {s: 0.0 for s in SCHEDULES}, 0.0
        for t in tiles:
            c, f, s, cost = self.tune(t, r, k, flavors=("dense", "sparse"))
            cells.append(c)
            fl_pts[f] = fl_pts.get(f, 0) + t.shape[0]
            for sc in SCHEDULES:
                sched_cost[sc] += cost[sc] * t.shape[0]
            total_vox += _voxels(tile_stats(t)[3], c)
        flavor = max(fl_pts, key=fl_pts.get)
        if flavor == "dense" and total_vox >= 4 * DENSE_VOXEL_BUDGET:
            flavor = "sparse"
        schedule = min(sched_cost, key=sched_cost.get)
        return cells, flavor, schedule


def pick_radius_schedule(index, r, queries=None, kernel="sphere", reps=2):
    """Times the count pass of one query batch under both radius schedules
    (64-query tiles, 8-query groups) and leaves the faster set on the index.
    Returns (schedule, {schedule: ms}).  The best schedule depends on how
    densely the queries sample the cloud: sparse query sets whose 64-query
    tiles span little more than each query's own ball favour the tiles
    (each candidate fetched once per wave through the scalar unit), dense
    ones the groups' tighter candidate lists."""
    times = {}
    for sched in SCHEDULES:
        index.set_radius_schedule(sched)
        index.radius_count(r, queries, kernel=kernel, sync=False)
        torch.cuda.synchronize()
        best = math.inf
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            index.radius_count(r, queries, kernel=kernel, sync=False)
            b.record()
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b))
        times[sched] = best
    choice = min(times, key=times.get)
    index.set_radius_schedule(choice)
    return choice, times


def pick_knn_schedule(index, k, queries=None, reps=2, schedules=("rings", "solo"),
                      r_max=math.inf):
    """Times k-NN of one query batch under each schedule (by default the
    ring schedule, whose 64-query tiles share one visited box, and the
    one-query-at-a-time schedule) and leaves the faster set on the index.
    Returns (schedule, {schedule: ms}).  One query at a time wins for query
    sets that sample the cloud sparsely (10 M-point ALS tile, 1 % of the
    points as queries: 1.1 vs 5.0 ms at k = 8; the aggregation workload's
    250 k centres among 1 M points, k = 64 within 0.5 m: 1.3 vs 1.6 ms), the
    rings for dense ones and wherever queries must search far (the TLS
    scan's far field)."""
    times = {}
    for sched in schedules:
        index.set_knn_schedule(sched)
        index.knn(k, queries, r_max=r_max)
        torch.cuda.synchronize()
        best = math.inf
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            index.knn(k, queries, r_max=r_max)
            b.record()
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b))
        times[sched] = best
    choice = min(times, key=times.get)
    index.set_knn_schedule(choice)
    return choice, times
