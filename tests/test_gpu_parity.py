"""GPU parity: the HIP library through its C ABI against the CPU oracle, on
the same seeded inputs.  Integer results (build arrays, neighbour sets, k-NN
indices) and the FP32 squared distances must be bit-exact."""
import math

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


def _walls(seed, n=3000, s=0.5):
    rng = np.random.default_rng(seed)
    g = rng.integers(0, 30, size=(n, 3)).astype(np.float64) * s
    g[: n // 10] = g[n // 10: 2 * (n // 10)]
    return g + np.array([1000.0, 2000.0, 10.0])


def _blob(seed, n=2000):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 0.5, (n, 3)) + 7.0


def _flat(seed, n=3000):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 40, (n, 3))
    p[:, 2] = 3.25
    return p


CLOUDS = {
    "als": lambda s: cloudgen.small_als(s, 30_000),
    "walls": _walls,
    "blob": _blob,
    "flat": _flat,
}


def _csr_pairs(off, nbr):
    off = np.asarray(off); nbr = np.asarray(nbr)
    rows = np.repeat(np.arange(len(off) - 1), np.diff(off))
    o = np.lexsort((nbr, rows))
    return rows[o], nbr[o]


def _assert_csr_equal(g_off, g_nbr, o_off, o_nbr):
    g_off = g_off.cpu().numpy() if hasattr(g_off, "cpu") else g_off
    g_nbr = g_nbr.cpu().numpy() if hasattr(g_nbr, "cpu") else g_nbr
    np.testing.assert_array_equal(g_off, o_off)
    gr, gn = _csr_pairs(g_off, g_nbr)
    orr, on = _csr_pairs(o_off, o_nbr)
    np.testing.assert_array_equal(gr, orr)
    np.testing.assert_array_equal(gn, on)


# ---------------------------------------------------------------- build
@pytest.mark.parametrize("name", sorted(CLOUDS))
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("dims,s", [(3, 1.0), (3, 0.3), (2, 2.5)])
def test_build_arrays(name, flavor, dims, s):
    dev = _dev()
    xyz = CLOUDS[name](3)
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=s, dims=dims, flavor=flavor)
    ox = oracle.OracleIndex(xyz, s, dims=dims, flavor=flavor)
    inf = gi.info()
    assert inf["origin"] == ox.origin.tolist()
    assert inf["ncell"] == ox.ncell.tolist()
    np.testing.assert_array_equal(np.array(inf["max32"], np.float32), ox.max32)
    assert inf["n_nonempty"] == ox.n_nonempty
    a = gi.arrays()
    o = ox.point_arrays()
    np.testing.assert_array_equal(a["perm"].cpu().numpy(), o["perm"])
    np.testing.assert_array_equal(a["sorted_xyz"].cpu().numpy(), o["sorted"])
    pts = a["points"].cpu().numpy()
    np.testing.assert_array_equal(pts[:, :3].T, o["sorted"])
    np.testing.assert_array_equal(pts[:, 3].view(np.int32), o["perm"])
    inv = a["inv_perm"].cpu().numpy()
    np.testing.assert_array_equal(inv[o["perm"]], np.arange(len(xyz)))
    uk, us = ox.cells()
    np.testing.assert_array_equal(a["cell_keys"].cpu().numpy(), uk)
    np.testing.assert_array_equal(a["cell_start"].cpu().numpy(), us)
    if flavor == "dense":
        np.testing.assert_array_equal(a["dense_start"].cpu().numpy(), ox.dense_start())
    else:
        assert a["dense_start"] is None
    if flavor == "mixed":
        ne, de = ox.slices()
        np.testing.assert_array_equal(a["slice_dense"].cpu().numpy().astype(bool), de)
        assert inf["n_dense_slices"] == int(de.sum())


def test_build_config0_and_determinism():
    dev = _dev()
    c = cloudgen.config0()
    x = torch.from_numpy(c["xyz"]).to(dev)
    a1 = _gi()(x, cell=1.0).arrays()
    a2 = _gi()(x, cell=1.0).arrays()
    for k in a1:
        if a1[k] is not None:
            assert torch.equal(a1[k], a2[k]), k
    ox = oracle.OracleIndex(c["xyz"], 1.0)
    np.testing.assert_array_equal(a1["perm"].cpu().numpy(), ox.point_arrays()["perm"])


# ---------------------------------------------------------------- radius
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("r", [0.0, 0.5, 1.0, 2.5])
def test_radius_config0(flavor, r):
    dev = _dev()
    c = cloudgen.config0()
    gi = _gi()(torch.from_numpy(c["xyz"]).to(dev), cell=c["cell"], flavor=flavor)
    ox = oracle.OracleIndex(c["xyz"], c["cell"], flavor=flavor)
    q = c["queries"]
    off, nbr = gi.radius(r, torch.from_numpy(q).to(dev))
    ooff, onbr = ox.radius(r, pidx=q, nthreads=8)
    _assert_csr_equal(off, nbr, ooff, onbr)


@pytest.mark.parametrize("sched", ["tiles", "groups"])
@pytest.mark.parametrize("name", sorted(CLOUDS))
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("dims,s", [(3, 1.0), (3, 0.3), (2, 2.5)])
def test_radius_all_points(name, flavor, dims, s, sched):
    dev = _dev()
    xyz = CLOUDS[name](4)
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=s, dims=dims, flavor=flavor)
    gi.set_radius_schedule(sched)
    ox = oracle.OracleIndex(xyz, s, dims=dims, flavor=flavor)
    r = 0.7 if name != "blob" else 0.05
    off, nbr = gi.radius(r)
    ooff, onbr = ox.radius(r, nthreads=8)
    _assert_csr_equal(off, nbr, ooff, onbr)


@pytest.mark.parametrize("sched", ["tiles", "groups"])
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
def test_radius_coordinate_queries(flavor, sched):
    dev = _dev()
    xyz = cloudgen.small_als(8, 40_000)
    rng = np.random.default_rng(11)
    qa = rng.uniform(xyz.min(0) - 4.0, xyz.max(0) + 4.0, (5000, 3))
    qa[:50] = xyz[:50]  # exactly on cloud points
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=1.0, flavor=flavor)
    gi.set_radius_schedule(sched)
    ox = oracle.OracleIndex(xyz, 1.0, flavor=flavor)
    for r in (0.6, 3.0):
        off, nbr = gi.radius(r, torch.from_numpy(qa).to(dev))
        ooff, onbr = ox.radius(r, qxyz=qa, nthreads=8)
        _assert_csr_equal(off, nbr, ooff, onbr)


def test_radius_edge_cases():
    dev = _dev()
    GI = _gi()
    # single point
    one = GI(torch.tensor([[5.0, 6.0, 7.0]], dtype=torch.float64, device=dev), cell=1.0)
    off, nbr = one.radius(0.0)
    assert off.tolist() == [0, 1] and nbr.tolist() == [0]
    # no queries
    xyz = _walls(1)
    gi = GI(torch.from_numpy(xyz).to(dev), cell=0.5)
    off, nbr = gi.radius(1.0, torch.empty(0, dtype=torch.int32, device=dev))
    assert off.tolist() == [0] and nbr.numel() == 0
    # out-of-range point indices give empty rows
    q = torch.tensor([0, -1, len(xyz), 5], dtype=torch.int32, device=dev)
    off, nbr = gi.radius(1.0, q)
    c = torch.diff(off).cpu().numpy()
    assert c[1] == 0 and c[2] == 0 and c[0] > 0 and c[3] > 0
    # radius beyond the bounding-box diagonal: every point
    off, nbr = gi.radius(1000.0, torch.arange(0, len(xyz), 97, dtype=torch.int32, device=dev))
    assert (torch.diff(off) == len(xyz)).all()
    # deterministic fill order
    o1, n1 = gi.radius(2.0)
    o2, n2 = gi.radius(2.0)
    assert torch.equal(o1, o2) and torch.equal(n1, n2)


@pytest.mark.parametrize("kernel", ["cube", "cylinder"])
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
def test_other_kernels_config0(kernel, flavor):
    """Cube and cylinder kernels of Alg. 1 on config 0: point queries at
    r = 0.5 and 1.5 m, coordinate queries (some far above the cloud)."""
    dev = _dev()
    c = cloudgen.config0()
    gi = _gi()(torch.from_numpy(c["xyz"]).to(dev), cell=c["cell"], flavor=flavor)
    ox = oracle.OracleIndex(c["xyz"], c["cell"], flavor=flavor)
    q = c["queries"]
    for r in (0.5, 1.5):
        off, nbr = gi.radius(r, torch.from_numpy(q).to(dev), kernel=kernel)
        ooff, onbr = ox.radius(r, pidx=q, nthreads=8, kernel=kernel)
        _assert_csr_equal(off, nbr, ooff, onbr)
    rng = np.random.default_rng(21)
    qa = c["xyz"][rng.choice(len(c["xyz"]), 3000, replace=False)].copy()
    qa[::3, 2] += 40.0
    off, nbr = gi.radius(1.0, torch.from_numpy(qa).to(dev), kernel=kernel)
    ooff, onbr = ox.radius(1.0, qxyz=qa, nthreads=8, kernel=kernel)
    _assert_csr_equal(off, nbr, ooff, onbr)


@pytest.mark.parametrize("sched", ["tiles", "groups"])
@pytest.mark.parametrize("kernel", ["cube", "cylinder"])
@pytest.mark.parametrize("name", sorted(CLOUDS))
@pytest.mark.parametrize("dims,s", [(3, 0.3), (2, 2.5)])
def test_other_kernels_all_points(kernel, name, dims, s, sched):
    dev = _dev()
    xyz = CLOUDS[name](4)
    for flavor in ("dense", "sparse", "mixed"):
        gi = _gi()(torch.from_numpy(xyz).to(dev), cell=s, dims=dims, flavor=flavor)
        gi.set_radius_schedule(sched)
        ox = oracle.OracleIndex(xyz, s, dims=dims, flavor=flavor)
        r = 0.7 if name != "blob" else 0.05
        off, nbr = gi.radius(r, kernel=kernel)
        ooff, onbr = ox.radius(r, nthreads=8, kernel=kernel)
        _assert_csr_equal(off, nbr, ooff, onbr)


def test_radius_rejects_bad_kernel():
    import ctypes
    from paper_2502_11602_amd._lib import Queries, lib
    dev = _dev()
    gi = _gi()(torch.from_numpy(_walls(2)).to(dev), cell=0.5)
    q = Queries(None, None, gi.n)
    tot = ctypes.c_int64(0)
    off = torch.empty(gi.n + 1, dtype=torch.int64, device=dev)
    call = lambda kern: lib().chs_kernel_count(gi._h, ctypes.byref(q), kern,  # noqa: E731
                                               ctypes.c_float(1.0), off.data_ptr(),
                                               ctypes.byref(tot), None)
    assert call(1) == 0 and tot.value > 0
    assert call(7) == 1 and b"kernel" in lib().chs_last_error()
    with pytest.raises(KeyError):
        gi.radius(1.0, kernel="torus")


def test_radius_rejects_bad_radius():
    from paper_2502_11602_amd import ChsError
    dev = _dev()
    gi = _gi()(torch.from_numpy(_walls(2)).to(dev), cell=0.5)
    for r in (-1.0, float("nan"), float("inf")):
        with pytest.raises(ChsError):
            gi.radius(r)


# ---------------------------------------------------------------- k-NN
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("k", [1, 5, 16, 33, 64])
def test_knn_config0(flavor, k):
    dev = _dev()
    c = cloudgen.config0()
    gi = _gi()(torch.from_numpy(c["xyz"]).to(dev), cell=c["cell"], flavor=flavor)
    ox = oracle.OracleIndex(c["xyz"], c["cell"], flavor=flavor)
    q = c["queries"]
    idx, d2 = gi.knn(k, torch.from_numpy(q).to(dev))
    oi, od = ox.knn(k, pidx=q, nthreads=8)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(d2.cpu().numpy(), od)


@pytest.mark.parametrize("name", sorted(CLOUDS))
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("dims,s", [(3, 1.0), (3, 0.3), (2, 2.5)])
def test_knn_all_points(name, flavor, dims, s):
    dev = _dev()
    xyz = CLOUDS[name](6)
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=s, dims=dims, flavor=flavor)
    ox = oracle.OracleIndex(xyz, s, dims=dims, flavor=flavor)
    for k in (8, 20):
        idx, d2 = gi.knn(k)
        oi, od = ox.knn(k, nthreads=8)
        np.testing.assert_array_equal(idx.cpu().numpy(), oi)
        np.testing.assert_array_equal(d2.cpu().numpy(), od)


@pytest.mark.parametrize("flavor", ["dense", "sparse"])
def test_knn_coordinate_queries_and_rmax(flavor):
    dev = _dev()
    xyz = cloudgen.small_als(9, 30_000)
    rng = np.random.default_rng(12)
    qa = rng.uniform(xyz.min(0) - 6.0, xyz.max(0) + 6.0, (4000, 3))
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=1.0, flavor=flavor)
    ox = oracle.OracleIndex(xyz, 1.0, flavor=flavor)
    for rmax in (math.inf, 0.8, 3.0):
        idx, d2 = gi.knn(12, torch.from_numpy(qa).to(dev), r_max=rmax)
        oi, od = ox.knn(12, r_max=rmax, qxyz=qa, nthreads=8)
        np.testing.assert_array_equal(idx.cpu().numpy(), oi)
        np.testing.assert_array_equal(d2.cpu().numpy(), od)


@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
def test_knn_density_schedule(flavor):
    """Alg. 2's density-growth schedule (CHS_OPT_KNN_SCHEDULE = 1) returns
    the oracle's lists and the ring schedule's, exactly: config 0 at
    k = 1, 16, 40, coordinate queries with an r_max cap, the adversarial
    clouds."""
    dev = _dev()
    c = cloudgen.config0()
    gi = _gi()(torch.from_numpy(c["xyz"]).to(dev), cell=c["cell"], flavor=flavor)
    ox = oracle.OracleIndex(c["xyz"], c["cell"], flavor=flavor)
    q = torch.from_numpy(c["queries"]).to(dev)
    for k in (1, 16, 40):
        ir, dr = gi.knn(k, q)
        gi.set_knn_schedule("density")
        idx, d2 = gi.knn(k, q)
        gi.set_knn_schedule("rings")
        oi, od = ox.knn(k, pidx=c["queries"], nthreads=8)
        np.testing.assert_array_equal(idx.cpu().numpy(), oi)
        np.testing.assert_array_equal(d2.cpu().numpy(), od)
        assert torch.equal(idx, ir) and torch.equal(d2, dr)
    rng = np.random.default_rng(31)
    qa = rng.uniform(c["xyz"].min(0) - 5.0, c["xyz"].max(0) + 5.0, (2000, 3))
    gi.set_knn_schedule("density")
    idx, d2 = gi.knn(12, torch.from_numpy(qa).to(dev), r_max=1.5)
    oi, od = ox.knn(12, r_max=1.5, qxyz=qa, nthreads=8)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(d2.cpu().numpy(), od)
    for name in sorted(CLOUDS):
        xyz = CLOUDS[name](4)
        g2 = _gi()(torch.from_numpy(xyz).to(dev), cell=0.3, flavor=flavor)
        g2.set_knn_schedule("density")
        i2, d2 = g2.knn(20)
        o2 = oracle.OracleIndex(xyz, 0.3, flavor=flavor)
        oi, od = o2.knn(20, nthreads=8)
        np.testing.assert_array_equal(i2.cpu().numpy(), oi)
        np.testing.assert_array_equal(d2.cpu().numpy(), od)


def _holes_sets(xyz, seed):
    """Index query sets with holes in config 0: 64 points from two opposite
    corners (one wave holding both), 100 and 130 of them (a compact wave
    beside a split one), a strip along each of two opposite edges, and
    clusters of 3 alternating between the corners (many small clusters)."""
    rel = xyz[:, :2] - xyz[:, :2].min(0)
    ext = rel.max(0)
    near_a = np.flatnonzero((rel < 6.0).all(1))
    near_b = np.flatnonzero((rel > ext - 6.0).all(1))
    rng = np.random.default_rng(seed)
    sets = []
    for na, nb in ((32, 32), (50, 50), (70, 60)):
        sets.append(np.concatenate([rng.choice(near_a, na, replace=False),
                                    rng.choice(near_b, nb, replace=False)]))
    strip_a = np.flatnonzero(rel[:, 0] < 3.0)
    strip_b = np.flatnonzero(rel[:, 0] > ext[0] - 3.0)
    sets.append(np.concatenate([rng.choice(strip_a, 400, replace=False),
                                rng.choice(strip_b, 400, replace=False)]))
    alt = []
    for i in range(12):
        src = near_a if i % 2 == 0 else near_b
        alt.append(rng.choice(src, 3, replace=False))
    sets.append(np.concatenate(alt))
    return [q.astype(np.int32) for q in sets]


@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("kernel", ["sphere", "cube", "cylinder"])
def test_radius_query_sets_with_holes(flavor, kernel):
    """Radius tiles whose queries lie far apart are counted and filled
    cluster by cluster (a second launch): CSR rows equal the oracle's, for
    the whole set and range by range."""
    dev = _dev()
    c = cloudgen.config0()
    xyz = c["xyz"]
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=c["cell"], flavor=flavor)
    gi.set_radius_schedule("tiles")
    ox = oracle.OracleIndex(xyz, c["cell"], flavor=flavor)
    for q in _holes_sets(xyz, 43):
        for r in (0.5, 1.5):
            qt = torch.from_numpy(q).to(dev)
            off, nbr = gi.radius(r, qt, kernel=kernel)
            ooff, onbr = ox.radius(r, pidx=q, nthreads=8, kernel=kernel)
            _assert_csr_equal(off, nbr, ooff, onbr)
    q = _holes_sets(xyz, 44)[3]
    qt = torch.from_numpy(q).to(dev)
    off, nbr = gi.radius(1.0, qt)
    parts = [part.clone() for _, _, part in gi.radius_chunked(1.0, qt, int(off[-1]) // 3 + 1,
                                                              offsets=off)]
    assert torch.equal(torch.cat(parts), nbr)


@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("schedule", ["rings", "density"])
def test_knn_query_sets_with_holes(flavor, schedule):
    """Waves whose queries lie far apart (more than 16 voxels) are searched
    cluster by cluster, each cluster with its own box: the lists equal the
    oracle's.  Query sets: 64 points from two opposite corners of config 0
    (one wave holding both), the same at 100 and 130 queries (a compact
    wave beside a split one), a strip along each of two opposite edges,
    and clusters of 3 alternating between corners (many small clusters)."""
    dev = _dev()
    c = cloudgen.config0()
    xyz = c["xyz"]
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=c["cell"], flavor=flavor)
    gi.set_knn_schedule(schedule)
    ox = oracle.OracleIndex(xyz, c["cell"], flavor=flavor)
    rel = xyz[:, :2] - xyz[:, :2].min(0)
    ext = rel.max(0)
    near_a = np.flatnonzero((rel < 6.0).all(1))
    near_b = np.flatnonzero((rel > ext - 6.0).all(1))
    rng = np.random.default_rng(41)
    sets = []
    for na, nb in ((32, 32), (50, 50), (70, 60)):
        sets.append(np.concatenate([rng.choice(near_a, na, replace=False),
                                    rng.choice(near_b, nb, replace=False)]))
    strip_a = np.flatnonzero(rel[:, 0] < 3.0)
    strip_b = np.flatnonzero(rel[:, 0] > ext[0] - 3.0)
    sets.append(np.concatenate([rng.choice(strip_a, 400, replace=False),
                                rng.choice(strip_b, 400, replace=False)]))
    alt = []
    for i in range(12):
        src = near_a if i % 2 == 0 else near_b
        alt.append(rng.choice(src, 3, replace=False))
    sets.append(np.concatenate(alt))
    for q in sets:
        q = q.astype(np.int32)
        for k in (1, 8, 16, 32, 64):
            idx, d2 = gi.knn(k, torch.from_numpy(q).to(dev))
            oi, od = ox.knn(k, pidx=q, nthreads=8)
            np.testing.assert_array_equal(idx.cpu().numpy(), oi, err_msg=f"nq={len(q)} k={k}")
            np.testing.assert_array_equal(d2.cpu().numpy(), od, err_msg=f"nq={len(q)} k={k}")
    # visited counts through the split launch: the lists are the same and
    # every count lies between the query's own box and the grid
    q = sets[0].astype(np.int32)
    i2, e2, vis = gi.knn_visited(16, torch.from_numpy(q).to(dev))
    oi, od = ox.knn(16, pidx=q, nthreads=8)
    np.testing.assert_array_equal(i2.cpu().numpy(), oi)
    vis = vis.cpu().numpy()
    assert (vis[:, 0] >= 1).all() and (vis[:, 0] <= vis[:, 1]).all()
    # a cluster's box is far smaller than the box over both corners
    n = np.array(gi.info()["ncell"], np.int64)
    assert (vis[:, 1] < np.prod(n) // 20).all(), (vis[:, 1].max(), np.prod(n))


@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
def test_knn_solo_schedule(flavor):
    """The one-query-at-a-time schedule (CHS_OPT_KNN_SCHEDULE = 3) returns
    the oracle's lists and the ring schedule's, exactly: config 0 at
    k = 1, 16, 40, 64, sparse index queries, coordinate queries (inside and
    outside the box) with an r_max cap, the adversarial clouds in 3D and
    2D."""
    dev = _dev()
    c = cloudgen.config0()
    gi = _gi()(torch.from_numpy(c["xyz"]).to(dev), cell=c["cell"], flavor=flavor)
    ox = oracle.OracleIndex(c["xyz"], c["cell"], flavor=flavor)
    q = torch.from_numpy(c["queries"]).to(dev)
    for k in (1, 16, 40, 64):
        ir, dr = gi.knn(k, q)
        gi.set_knn_schedule("solo")
        idx, d2 = gi.knn(k, q)
        gi.set_knn_schedule("rings")
        oi, od = ox.knn(k, pidx=c["queries"], nthreads=8)
        np.testing.assert_array_equal(idx.cpu().numpy(), oi)
        np.testing.assert_array_equal(d2.cpu().numpy(), od)
        assert torch.equal(idx, ir) and torch.equal(d2, dr)
    rng = np.random.default_rng(32)
    qa = rng.uniform(c["xyz"].min(0) - 5.0, c["xyz"].max(0) + 5.0, (2000, 3))
    gi.set_knn_schedule("solo")
    idx, d2 = gi.knn(12, torch.from_numpy(qa).to(dev), r_max=1.5)
    oi, od = ox.knn(12, r_max=1.5, qxyz=qa, nthreads=8)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(d2.cpu().numpy(), od)
    idx, d2 = gi.knn(9, torch.from_numpy(qa).to(dev))
    oi, od = ox.knn(9, qxyz=qa, nthreads=8)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(d2.cpu().numpy(), od)
    for name in sorted(CLOUDS):
        for dims, s in ((3, 0.3), (2, 2.5)):
            xyz = CLOUDS[name](4)
            g2 = _gi()(torch.from_numpy(xyz).to(dev), cell=s, dims=dims, flavor=flavor)
            g2.set_knn_schedule("solo")
            i2, e2 = g2.knn(20)
            o2 = oracle.OracleIndex(xyz, s, dims=dims, flavor=flavor)
            oi, od = o2.knn(20, nthreads=8)
            np.testing.assert_array_equal(i2.cpu().numpy(), oi)
            np.testing.assert_array_equal(e2.cpu().numpy(), od)


def test_knn_edge_cases():
    dev = _dev()
    GI = _gi()
    # fewer points than k
    xyz = np.random.default_rng(0).uniform(0, 3, (10, 3))
    gi = GI(torch.from_numpy(xyz).to(dev), cell=1.0)
    idx, d2 = gi.knn(16)
    oi, od = oracle.OracleIndex(xyz, 1.0).knn(16)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(d2.cpu().numpy(), od)
    assert (idx[:, 10:] == -1).all()
    # duplicates: ties broken by original index
    w = _walls(5)
    gi = GI(torch.from_numpy(w).to(dev), cell=0.5)
    idx, d2 = gi.knn(24)
    oi, od = oracle.OracleIndex(w, 0.5).knn(24)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(d2.cpu().numpy(), od)
    # invalid point indices give (-1, inf) rows
    q = torch.tensor([3, -7, len(w)], dtype=torch.int32, device=dev)
    idx, d2 = gi.knn(4, q)
    assert (idx[1:] == -1).all() and torch.isinf(d2[1:]).all() and (idx[0] >= 0).all()
    # k-prefix property and determinism
    i8, _ = gi.knn(8)
    i32, _ = gi.knn(32)
    assert torch.equal(i32[:, :8], i8)
    assert torch.equal(gi.knn(32)[0], i32)


# ---------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def config1_oracle():
    c = cloudgen.config1()
    return c, oracle.OracleIndex(c["xyz"], 1.0)


@pytest.mark.slow
def test_config1_full_size_sampled(config1_oracle):
    """The 10 M-point ALS tile, every point a query, in the launch
    configuration the benchmark times; a seeded sample of rows is checked
    against the oracle exactly, and the whole radius relation for symmetry."""
    dev = _dev()
    c, ox = config1_oracle
    xyz = c["xyz"]
    n = len(xyz)
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=1.0)
    samp = np.sort(np.random.default_rng(42).choice(n, 3000, replace=False)).astype(np.int32)
    st = torch.from_numpy(samp.astype(np.int64)).to(dev)
    for r in c["radii"]:
        off, nbr = gi.radius(r)
        counts = torch.diff(off)
        ooff, onbr = ox.radius(r, pidx=samp, nthreads=8)
        np.testing.assert_array_equal(counts[st].cpu().numpy(), np.diff(ooff))
        rows = []
        offc = off.cpu().numpy()
        nb = nbr.cpu().numpy() if r <= 1.0 else None
        for t, p in enumerate(samp):
            g = nb[offc[p]:offc[p + 1]] if nb is not None else \
                nbr[int(offc[p]):int(offc[p + 1])].cpu().numpy()
            rows.append(np.sort(g))
        got = np.concatenate(rows)
        want = np.concatenate([np.sort(onbr[ooff[t]:ooff[t + 1]]) for t in range(len(samp))])
        np.testing.assert_array_equal(got, want)
        if r == 1.0:
            # symmetry of the whole relation: the multiset of pairs is closed
            # under swapping (compared through two order-independent sums)
            rowi = torch.repeat_interleave(torch.arange(n, device=dev), counts)
            a = rowi.to(torch.int64) * 1_000_003 + nbr.to(torch.int64)
            b = nbr.to(torch.int64) * 1_000_003 + rowi.to(torch.int64)
            h = lambda v: ((v * 0x9E3779B97F4A7C15) >> 17) & 0xFFFFFFFF  # noqa: E731
            assert int(h(a).sum()) == int(h(b).sum())
        del off, nbr
    for k in c["ks"]:
        idx, d2 = gi.knn(k)
        oi, od = ox.knn(k, pidx=samp, nthreads=8)
        np.testing.assert_array_equal(idx[st].cpu().numpy(), oi)
        np.testing.assert_array_equal(d2[st].cpu().numpy(), od)


@pytest.mark.slow
def test_config1_full_size_knn_sampled(config1_oracle):
    """k-NN at k = 8, 16, 32 on the 10 M-point tile, every point a query (the
    benchmark's launches); a seeded sample of rows equals the oracle's, and
    each k's list is a prefix of the next one's."""
    dev = _dev()
    c, ox = config1_oracle
    xyz = c["xyz"]
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=1.0)
    samp = np.sort(np.random.default_rng(43).choice(len(xyz), 3000, replace=False)).astype(np.int32)
    st = torch.from_numpy(samp.astype(np.int64)).to(dev)
    prev = None
    for k in c["ks"]:
        idx, d2 = gi.knn(k)
        oi, od = ox.knn(k, pidx=samp, nthreads=8)
        np.testing.assert_array_equal(idx[st].cpu().numpy(), oi)
        np.testing.assert_array_equal(d2[st].cpu().numpy(), od)
        if prev is not None:
            assert torch.equal(idx[:, :prev.shape[1]], prev)
        prev = idx
        del d2


@pytest.fixture(scope="module")
def config2_oracle():
    c = cloudgen.config2()
    return c, oracle.OracleIndex(c["xyz"], 0.25, flavor="sparse")


@pytest.mark.slow
@pytest.mark.parametrize("flavor", ["sparse", "mixed"])
def test_config2_full_size_sampled(config2_oracle, flavor):
    """The 20 M-point TLS scan (density falling with range), 0.25 m voxels:
    k = 32 on all 2 M query indices, and radius at 0.1 / 0.25 / 0.5 m on
    every 100th of them (near the scanner a 0.5 m ball holds tens of
    thousands of points, so the CSR of all 2 M queries would not fit one
    GPU); seeded samples of 2000 rows checked against the oracle."""
    dev = _dev()
    c, ox = config2_oracle
    xyz = c["xyz"]
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=0.25, flavor=flavor)
    rq = c["queries"][::100]
    q = torch.from_numpy(rq).to(dev)
    sel = np.sort(np.random.default_rng(44).choice(len(rq), 2000, replace=False))
    samp = rq[sel]
    for r in c["radii"]:
        off, nbr = gi.radius(r, q)
        offc = off.cpu().numpy()
        ooff, onbr = ox.radius(r, pidx=samp, nthreads=8)
        np.testing.assert_array_equal(offc[sel + 1] - offc[sel], np.diff(ooff))
        got = np.concatenate([np.sort(nbr[int(offc[t]):int(offc[t + 1])].cpu().numpy()) for t in sel])
        want = np.concatenate([np.sort(onbr[ooff[j]:ooff[j + 1]]) for j in range(len(sel))])
        np.testing.assert_array_equal(got, want)
        del off, nbr
    qa = torch.from_numpy(c["queries"]).to(dev)
    idx, d2 = gi.knn(c["k"], qa)
    sel = np.sort(np.random.default_rng(45).choice(len(c["queries"]), 2000, replace=False))
    oi, od = ox.knn(c["k"], pidx=c["queries"][sel], nthreads=8)
    st = torch.from_numpy(sel.astype(np.int64)).to(dev)
    np.testing.assert_array_equal(idx[st].cpu().numpy(), oi)
    np.testing.assert_array_equal(d2[st].cpu().numpy(), od)


# ---------------------------------------------------------------- every query at full size
@pytest.fixture(scope="module")
def config1_cloud():
    return cloudgen.config1()


@pytest.mark.slow
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
def test_config1_every_query_digests(config1_cloud, flavor):
    """The 10 M-point ALS tile, every point a query, in the launch
    configuration the benchmark times: every query's neighbour count and
    order-independent neighbour hash (sphere at 0.5-4 m, cube and cylinder at
    2 and 3 m: fills with 16-, 24- and 32-entry stages), and every k-NN row
    (k = 8, 16, 32) in order, summarised per block of 2^18 queries, equal the
    oracle's digests written by tests/golden/make_config1_digests.py."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import _digest as D
    from tests.conftest import ROOT
    dev = _dev()
    meta, sets = D.read_golden(os.path.join(ROOT, "tests", "golden", "config1_digests.txt"))
    xyz = config1_cloud["xyz"]
    assert D.fingerprint(xyz) == meta["input"][0], "the generator no longer gives the digested cloud"
    assert int(meta["block"][0]) == D.BLOCK
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=1.0, flavor=flavor)
    for name, want in sets.items():
        if name.startswith("knn_"):
            idx, d2 = gi.knn(int(name[4:]))
            cnt, h = D.row_hash_knn_t(idx, d2)
            del idx, d2
        else:
            kern, r = name.split("_")
            off, nbr = gi.radius(float(r), kernel=kern)
            cnt, h = D.row_hash_csr_t(off, nbr)
            del off, nbr
        got = D.block_digests_t(cnt, h)
        bad = [w[0] for g, w in zip(got, want) if g != w]
        assert len(got) == len(want) and not bad, f"{flavor} {name}: blocks {bad[:10]} differ"


# ---------------------------------------------------------------- every fill stage
@pytest.mark.parametrize("n", [3000, 9000])
@pytest.mark.parametrize("flavor", ["dense", "sparse"])
def test_fill_long_rows_streaming(n, flavor):
    """Rows of thousands of entries take the fill stages whose flushes use
    non-temporal stores (mean row >= 2048: the 32-entry stage, >= 8192: the
    64-entry one): a blob of n points in a 0.5 m cube, every point a query
    at r = 1 m (rows of n entries), against the oracle."""
    dev = _dev()
    xyz = _blob(6, n)
    g = _gi()(torch.from_numpy(xyz).to(dev), cell=0.1, flavor=flavor)
    g.set_radius_schedule("tiles")
    off, nbr = g.radius(1.0)
    ooff, onbr = oracle.OracleIndex(xyz, 0.1, flavor=flavor).radius(1.0, nthreads=8)
    assert int(ooff[-1]) == n * n
    _assert_csr_equal(off, nbr, ooff, onbr)


@pytest.mark.parametrize("stage", [16, 24, 32, 64])
@pytest.mark.parametrize("kernel", ["sphere", "cube", "cylinder"])
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
def test_fill_stages(stage, kernel, flavor):
    """Each LDS stage size of the 64-query tiles' radius fill (16, 24, 32,
    64 entries per query, forced with CHS_OPT_FILL_STAGE) with each kernel
    and flavor: config 0 at r = 2.5 m (rows of tens of entries, several
    flushes per wave), the duplicate-heavy walls cloud and the blob (rows of
    2000 entries), all points, against the oracle."""
    dev = _dev()
    c = cloudgen.config0()
    gi = _gi()(torch.from_numpy(c["xyz"]).to(dev), cell=c["cell"], flavor=flavor)
    gi.set_radius_schedule("tiles")
    gi.set_fill_stage(stage)
    ox = oracle.OracleIndex(c["xyz"], c["cell"], flavor=flavor)
    q = c["queries"]
    off, nbr = gi.radius(2.5, torch.from_numpy(q).to(dev), kernel=kernel)
    ooff, onbr = ox.radius(2.5, pidx=q, nthreads=8, kernel=kernel)
    assert stage > 32 or np.diff(ooff).max() > 2 * stage
    _assert_csr_equal(off, nbr, ooff, onbr)
    for xyz, s, r in ((_walls(7), 0.5, 1.2), (_blob(5), 0.1, 1.0)):
        gw = _gi()(torch.from_numpy(xyz).to(dev), cell=s, flavor=flavor)
        gw.set_radius_schedule("tiles")
        gw.set_fill_stage(stage)
        off, nbr = gw.radius(r, kernel=kernel)
        ooff, onbr = oracle.OracleIndex(xyz, s, flavor=flavor).radius(r, nthreads=8, kernel=kernel)
        _assert_csr_equal(off, nbr, ooff, onbr)


@pytest.mark.parametrize("kernel", ["sphere", "cube", "cylinder"])
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
def test_query_groups(kernel, flavor):
    """The 8-query-group schedule (CHS_OPT_RADIUS_SCHEDULE = 2) with each
    kernel and flavor: config 0 at r = 0.5, 2.5 and 6 m (packed lists of a
    few to several thousand candidates, so more than one LDS piece), the
    walls cloud (duplicates, points on voxel walls), against the oracle."""
    dev = _dev()
    c = cloudgen.config0()
    gi = _gi()(torch.from_numpy(c["xyz"]).to(dev), cell=c["cell"], flavor=flavor)
    gi.set_radius_schedule("groups")
    ox = oracle.OracleIndex(c["xyz"], c["cell"], flavor=flavor)
    q = c["queries"]
    for r in (0.5, 2.5, 6.0):
        off, nbr = gi.radius(r, torch.from_numpy(q).to(dev), kernel=kernel)
        ooff, onbr = ox.radius(r, pidx=q, nthreads=8, kernel=kernel)
        _assert_csr_equal(off, nbr, ooff, onbr)
    w = _walls(8)
    gw = _gi()(torch.from_numpy(w).to(dev), cell=0.5, flavor=flavor)
    gw.set_radius_schedule("groups")
    off, nbr = gw.radius(1.2, kernel=kernel)
    ooff, onbr = oracle.OracleIndex(w, 0.5, flavor=flavor).radius(1.2, nthreads=8, kernel=kernel)
    _assert_csr_equal(off, nbr, ooff, onbr)


@pytest.mark.slow
@pytest.mark.parametrize("flavor", ["sparse", "mixed"])
def test_config2_every_query_digests(config2_oracle, flavor):
    """The 20 M-point TLS scan, 2 M query points, 0.25 m voxels, in the
    launch configuration the benchmark times: the queries in the searches'
    processing order, each radius counted over all of them, then filled
    range by range within 2^32 entries per range (at 0.5 m the relation
    holds 1.5e11 pairs), each range's rows hashed as it is filled; every
    query's count and order-independent neighbour hash (sphere at 0.1, 0.25,
    0.5 m) and every k = 32 row in order, summarised per block of 2^18
    queries in the caller's order, equal the oracle's digests written by
    tests/golden/make_config2_digests.py."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import _digest as D
    from tests.conftest import ROOT
    dev = _dev()
    meta, sets = D.read_golden(os.path.join(ROOT, "tests", "golden", "config2_digests.txt"))
    c = config2_oracle[0]
    xyz, qidx = c["xyz"], c["queries"]
    assert D.fingerprint(xyz) == meta["input"][0], "the generator no longer gives the digested cloud"
    assert D.fingerprint(qidx.astype(np.float64)) == meta["input"][2]
    assert int(meta["block"][0]) == D.BLOCK
    gi = _gi()(torch.from_numpy(xyz).to(dev), cell=0.25, flavor=flavor)
    from paper_2502_11602_amd.autotune import pick_radius_schedule
    q = torch.from_numpy(qidx).to(dev)
    order = gi.query_order(q).long()
    qs = q[order]
    nq = len(qidx)
    for name, want in sets.items():
        if name.startswith("knn_"):
            idx, d2 = gi.knn(int(name[4:]), q)
            cnt, h = D.row_hash_knn_t(idx, d2)
            del idx, d2
        else:
            r = float(name.split("_")[1])
            pick_radius_schedule(gi, r, qs)
            off, _ = gi.radius_count(r, qs)
            cnt = torch.empty(nq, dtype=torch.int64, device=dev)
            h = torch.empty(nq, dtype=torch.int64, device=dev)
            for a, b, part in gi.radius_chunked(r, qs, 1 << 32, offsets=off):
                ca, ha = D.row_hash_csr_t(off[a:b + 1] - off[a], part)
                cnt[order[a:b]] = ca
                h[order[a:b]] = ha
                del part
            del off
        got = D.block_digests_t(cnt, h)
        bad = [w[0] for g, w in zip(got, want) if g != w]
        assert len(got) == len(want) and not bad, f"{flavor} {name}: blocks {bad[:10]} differ"
