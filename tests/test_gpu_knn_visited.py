"""GPU: the visited-voxel counts of k-NN (chs_knn_visited), the cost measure
by which Section 3.5 compares density growth with monotonic growth.

Per query: its own taboo box (Alg. 2 for it alone) and the wave's visited
box when its list became final.  Properties checked:
- the lists equal chs_knn's;
- the box holds the query's voxel and the voxels of all k neighbours found,
  so the count is at least the voxels of their bounding box, and at most
  the grid's;
- under density or monotonic growth on a dense map the query's own count
  is the oracle's, exactly (every voxel exists there, Section 3.5 "Voxels
  in dense Cheesemap"), and the 1 M-point statistic follows."""
import numpy as np
import pytest

import cloudgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _gi():
    from paper_2502_11602_amd import GridIndex
    return GridIndex


def _lower_bound(gi, qpts, idx):
    """Voxels of the bounding box of each query's voxel and its neighbours'
    (query and neighbour coordinates in the index's FP32 frame)."""
    inf = gi.info()
    s = np.array(inf["cell"], np.float64)
    n = np.array(inf["ncell"], np.int64)
    xyz = gi.coords().cpu().numpy().astype(np.float64)

    def vox(p):
        return np.clip(np.floor(p / s), 0, n - 1).astype(np.int64)

    qv = vox(qpts)
    lo = qv.copy(); hi = qv.copy()
    for t in range(idx.shape[1]):
        j = idx[:, t]
        ok = j >= 0
        v = vox(xyz[np.where(ok, j, 0)])
        lo = np.where(ok[:, None], np.minimum(lo, v), lo)
        hi = np.where(ok[:, None], np.maximum(hi, v), hi)
    dims = inf["dims"]
    return np.prod((hi - lo + 1)[:, :dims], axis=1), int(np.prod(n[:dims]))


@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("schedule", ["rings", "density", "monotonic"])
def test_visited_bounds_and_lists(flavor, schedule):
    dev = _dev()
    c = cloudgen.config0()
    gi = _gi()(torch.from_numpy(c["xyz"]).to(dev), cell=c["cell"], flavor=flavor)
    gi.set_knn_schedule(schedule)
    xyz32 = gi.coords().cpu().numpy().astype(np.float64)
    for k in (1, 16, 40):
        idx, d2 = gi.knn(k)
        i2, e2, vis = gi.knn_visited(k)
        assert torch.equal(idx, i2) and torch.equal(d2, e2)
        vis = vis.cpu().numpy()
        lb, grid = _lower_bound(gi, xyz32, i2.cpu().numpy())
        assert (vis[:, 1] >= lb).all(), (k, int(np.argmin(vis[:, 1] - lb)))
        assert (vis[:, 1] <= grid).all() and (vis[:, 0] >= 1).all()
        # the wave's box holds each query's own box
        assert (vis[:, 0] <= vis[:, 1]).all()
        if schedule == "rings":
            assert (vis[:, 0] == vis[:, 1]).all()
    # coordinate queries (recentred on the index's frame like the build)
    rng = np.random.default_rng(5)
    qa = rng.uniform(c["xyz"].min(0), c["xyz"].max(0), (3000, 3))
    idx, d2 = gi.knn(12, torch.from_numpy(qa).to(dev))
    i2, e2, vis = gi.knn_visited(12, torch.from_numpy(qa).to(dev))
    assert torch.equal(idx, i2) and torch.equal(d2, e2)
    q32 = (qa - np.array(gi.info()["origin"])).astype(np.float32).astype(np.float64)
    lb, grid = _lower_bound(gi, q32, i2.cpu().numpy())
    vis = vis.cpu().numpy()
    assert (vis[:, 1] >= lb).all() and (vis[:, 1] <= grid).all()


@pytest.mark.parametrize("schedule", ["density", "monotonic"])
@pytest.mark.parametrize("k", [1, 8, 32])
def test_own_visited_equals_oracle(schedule, k):
    """Dense map, uniform cube (scaled down): each query's own count is the
    oracle's count for the same schedule, exactly, and the wave's box holds
    it."""
    dev = _dev()
    xyz = cloudgen.uniform_cube(seed=11, n=40_000, side=20.0)
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=1.0, flavor="dense")
    gi.set_knn_schedule(schedule)
    idx, d2, vis = gi.knn_visited(k)
    ox = oracle.OracleIndex(xyz, 1.0, flavor="dense")
    oi, od, ov = ox.knn(k, nthreads=8, visited=True, schedule=schedule)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(d2.cpu().numpy(), od)
    vis = vis.cpu().numpy()
    np.testing.assert_array_equal(vis[:, 0], ov)
    assert (vis[:, 1] >= ov).all()


# the hand-worked lattice counts of the oracle's pins (Alg. 2 on unit voxels)
@pytest.mark.parametrize("k,dens,mono", [(1, 27, 27), (7, 125, 125), (20, 125, 343),
                                         (33, 343, 343)])
def test_own_visited_lattice(k, dens, mono):
    dev = _dev()
    g = np.arange(10, dtype=np.float64) + 0.5
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pts = np.vstack([pts, [[0.0, 0.0, 0.0], [10.0, 10.0, 10.0]]])
    q = int(np.flatnonzero((pts == 5.5).all(1))[0])
    gi = _gi()(torch.from_numpy(pts).to(dev), cell=1.0, flavor="dense")
    qi = torch.tensor([q], dtype=torch.int32, device=dev)
    got = []
    for sched in ("density", "monotonic"):
        gi.set_knn_schedule(sched)
        got.append(int(gi.knn_visited(k, qi)[2][0, 0]))
    assert got == [dens, mono]


def test_growth_statistic_full_size():
    """The 1 M-point statistic of Section 3.5 from the GPU's own counts
    equals the oracle's stored one, row by row (every voxel edge and k)."""
    from tests.conftest import golden
    dev = _dev()
    rows = {(float(c), int(v[0])): tuple(int(x) for x in v[1:])
            for c, vals in golden("knn_growth_stats.txt").items() for v in vals}
    x = torch.from_numpy(cloudgen.uniform_cube()).to(dev)
    for s in sorted({c for c, _ in rows}):
        gi = _gi()(x, cell=s, flavor="dense")
        for k in sorted(kk for c, kk in rows if c == s):
            vv = []
            for sched in ("density", "monotonic"):
                gi.set_knn_schedule(sched)
                vv.append(gi.knn_visited(k)[2][:, 0].cpu().numpy())
            vd, vm = vv
            got = (int((vd < vm).sum()), int((vd > vm).sum()), int((vd == vm).sum()),
                   int(vd.sum()), int(vm.sum()))
            assert got == rows[(s, k)], (s, k, got, rows[(s, k)])
        gi.close()


def test_visited_invalid_queries_and_rejects():
    dev = _dev()
    c = cloudgen.config0()
    GI = _gi()
    gi = GI(torch.from_numpy(c["xyz"]).to(dev), cell=c["cell"])
    n = c["xyz"].shape[0]
    q = torch.tensor([0, -1, n, 5], dtype=torch.int32, device=dev)
    idx, d2, vis = gi.knn_visited(4, q)
    vis = vis.cpu().numpy()
    assert (vis[1] == -1).all() and (vis[2] == -1).all()  # left as they were
    assert (vis[0] >= 1).all() and (vis[3] >= 1).all()
    assert (idx[1].cpu().numpy() == -1).all()
    # empty query set: nothing written, no error
    i0, e0, v0 = gi.knn_visited(4, torch.empty(0, dtype=torch.int32, device=dev))
    assert v0.numel() == 0
    # batched (persistent) index: unsupported
    xyz = torch.from_numpy(c["xyz"]).to(dev)
    h = n // 2
    gb = GI(xyz, cell=c["cell"], tile_off=[0, h, n])
    from paper_2502_11602_amd import ChsError
    with pytest.raises(ChsError):
        gb.knn_visited(4)
    gi.set_persistent(True)
    with pytest.raises(ChsError):
        gi.knn_visited(4)
    gi.set_persistent(False)
    gi.knn_visited(4)
