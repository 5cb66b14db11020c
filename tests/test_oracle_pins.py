"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code (worked numbers printed in the
paper, brute force on small clouds, library routines for the build arrays,
invariants of the neighbour relations, finite differences for gradients)."""
import math

import numpy as np
import pytest

import cloudgen
import oracle
from tests._brute import brute_kernel, brute_knn, brute_radius, csr_rows, sq_dist_rows
from tests.conftest import golden

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# --------------------------------------------------------------------------
# clouds
# --------------------------------------------------------------------------
def _als(seed, n=1500):
    return cloudgen.small_als(seed, n)


def _walls(seed, n=1200, s=0.5):
    """Coordinates on exact voxel walls (integer multiples of s) plus duplicates."""
    rng = np.random.default_rng(seed)
    g = rng.integers(0, 12, size=(n, 3)).astype(np.float64) * s
    g[: n // 10] = g[n // 10: 2 * (n // 10)]  # exact duplicates
    return g + np.array([1000.0, 2000.0, 10.0])


def _blob(seed, n=800):
    """Everything inside a single 1 m voxel."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 0.5, (n, 3)) + 7.0


def _flat(seed, n=1000):
    """Zero extent along z (n_z = 1)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 20, (n, 3))
    p[:, 2] = 3.25
    return p


CLOUDS = {"als": _als, "walls": _walls, "blob": _blob, "flat": _flat}


def _q32(ix, xyz):
    return (np.asarray(xyz, np.float64) - ix.origin).astype(np.float32)


# --------------------------------------------------------------------------
# Eq. 3 -- grid size -- pinned by the voxel counts printed in Section 5.2
# --------------------------------------------------------------------------
def _box_cloud(ex, ey, ez, n=2000, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 1, (n, 3)) * np.array([ex, ey, ez])
    p[0] = 0.0
    p[1] = [ex, ey, ez]  # the two bounding-box corners
    return p + np.array([5.0e5, 5.4e6, 0.0])


@pytest.mark.parametrize("row", golden("voxel_counts.txt")["dales_3d"] +
                         golden("voxel_counts.txt")["dales_2d"])
def test_grid_size_matches_paper_voxel_counts(row):
    ex, ey, ez, s, dims, printed, digits = row
    ex, ey, ez, s, dims = float(ex), float(ey), float(ez), float(s), int(dims)
    xyz = _box_cloud(ex, ey, ez)
    ix = oracle.OracleIndex(xyz, s, dims=dims, flavor="sparse")
    count = int(np.prod(ix.ncell))
    mant, exp = printed.split("e")
    scale = 10.0 ** int(exp)
    assert round(count / scale, int(digits)) == float(mant), (count, printed)


def test_grid_size_rules_out_ceil():
    # a ceil-based grid would give 500 * 500 * 169 = 42.25e6 for the DALES box
    ix = oracle.OracleIndex(_box_cloud(500.0, 500.0, 168.4), 1.0, flavor="sparse")
    assert list(ix.ncell) == [501, 501, 169]
    assert int(np.prod(ix.ncell)) == 42_419_169


def test_grid_size_lille_ratio():
    # Section 5.2: Lille Dense<2> 798.43e3 voxels, Dense<3> 34.33e6, i.e. n_z = 43,
    # which Eq. 3 gives for any z extent in [42, 43) m at s = 1 m.
    for ez in (42.0, 42.5, 42.999):
        ix = oracle.OracleIndex(_box_cloud(1000.0, 797.0, ez), 1.0, flavor="sparse")
        assert ix.ncell[2] == 43
    assert round(798_430 * 43 / 1e6, 2) == 34.33


# --------------------------------------------------------------------------
# Eq. 5 / Eq. 7 -- voxel of a point and global order -- invariants
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", sorted(CLOUDS))
@pytest.mark.parametrize("s", [0.3, 1.0, 2.5])
@pytest.mark.parametrize("dims", [2, 3])
def test_build_arrays(name, s, dims):
    xyz = CLOUDS[name](11)
    ix = oracle.OracleIndex(xyz, s, dims=dims, flavor="dense")
    a = ix.point_arrays()
    x32 = a["x32"]
    # recentring: FP64 subtraction of the exact minimum, then FP32
    np.testing.assert_array_equal(x32.T, (xyz - xyz.min(axis=0)).astype(np.float32))
    np.testing.assert_array_equal(ix.max32, x32.max(axis=1))
    assert ix.origin.tolist() == xyz.min(axis=0).tolist()
    keys = a["keys"].astype(np.int64)
    nc = ix.ncell
    # decode g with divmod only (no geometry) and check the voxel bounds
    i = keys // (nc[1] * nc[2]); j = (keys // nc[2]) % nc[1]; k = keys % nc[2]
    assert (i < nc[0]).all() and (j < nc[1]).all() and (k < nc[2]).all()
    for axis, c in ((0, i), (1, j), (2, k)):
        if axis == 2 and dims == 2:
            assert (c == 0).all() and nc[2] == 1
            continue
        v = x32[axis].astype(np.float64)
        assert (c * s <= v * (1 + 1e-12) + 1e-12).all()
        top = c == nc[axis] - 1
        assert ((v < (c + 1) * s * (1 + 1e-12)) | top).all()
        assert (nc[axis] - 1) * s <= ix.max32[axis] * (1 + 1e-12)
    # counting sort == stable argsort; stored coordinates follow it
    np.testing.assert_array_equal(a["perm"], np.argsort(keys, kind="stable"))
    np.testing.assert_array_equal(a["sorted"], x32[:, a["perm"]])
    # global order: x slowest, then y, then z (Eq. 7)
    ijk = np.stack([i, j, k], 1)[a["perm"]]
    lex = np.lexsort((ijk[:, 2], ijk[:, 1], ijk[:, 0]))
    np.testing.assert_array_equal(ijk[lex], ijk)
    # non-empty voxels and their starts == np.unique on the sorted keys
    uk, us = ix.cells()
    sk = keys[a["perm"]]
    u, first = np.unique(sk, return_index=True)
    np.testing.assert_array_equal(uk.astype(np.int64), u)
    np.testing.assert_array_equal(us, np.append(first, len(sk)))
    # dense start table == searchsorted over every voxel, empty ones included
    ds = ix.dense_start()
    np.testing.assert_array_equal(ds, np.searchsorted(sk, np.arange(int(np.prod(nc)) + 1)))


def test_sparse_fig2_example():
    f = golden("sparse_fig2.txt")
    nx, ny = map(int, f["grid"][0])
    empty = {(int(a), int(b)) for a, b in f["empty"]}
    pts = []
    rng = np.random.default_rng(2)
    for i in range(nx):
        for j in range(ny):
            if (i, j) in empty:
                continue
            pts.append(np.c_[rng.uniform(i + 0.05, i + 0.95, 5), rng.uniform(j + 0.05, j + 0.95, 5),
                             np.zeros(5)])
    xyz = np.concatenate(pts)
    xyz[0, :2] = 0.0
    xyz[1, :2] = [nx - 0.01, ny - 0.01]
    ix = oracle.OracleIndex(xyz, 1.0, dims=2, flavor="sparse")
    assert list(ix.ncell[:2]) == [nx, ny]
    assert ix.n_nonempty == int(f["nonempty"][0][0])
    uk, _ = ix.cells()
    stored = {(int(g) // ny, int(g) % ny) for g in uk}
    assert stored.isdisjoint(empty)


def test_kernel_box_fig3_example():
    f = golden("kernel_box_fig3.txt")
    nx, ny = map(int, f["grid"][0])
    cx, cy = map(float, f["centre"][0])
    r = float(f["radius"][0][0])
    rng = np.random.default_rng(3)
    xyz = np.c_[rng.uniform(0, nx - 0.01, 4000), rng.uniform(0, ny - 0.01, 4000), np.zeros(4000)]
    xyz[0] = 0.0
    xyz[1, :2] = [nx - 0.01, ny - 0.01]
    ix = oracle.OracleIndex(xyz, 1.0, dims=2, flavor="dense")
    assert list(ix.ncell[:2]) == [nx, ny]
    off, nbr, vis = ix.radius(r, qxyz=np.array([[cx, cy, 0.0]]), visited=True)
    assert vis[0] == int(f["box_voxels"][0][0])
    i0, i1 = map(int, f["box_i"][0]); j0, j1 = map(int, f["box_j"][0])
    assert (i1 - i0 + 1) * (j1 - j0 + 1) == vis[0]
    # every neighbour lies in a voxel that meets the circle (dark grey)
    miss = {(int(a), int(b)) for a, b in f["sphere_miss"]}
    cells = {(int(xyz[p, 0]), int(xyz[p, 1])) for p in nbr}
    assert cells.isdisjoint(miss) and len(cells) <= int(f["sphere_voxels"][0][0])
    assert all(i0 <= a <= i1 and j0 <= b <= j1 for a, b in cells)


# --------------------------------------------------------------------------
# Alg. 1 -- radius search == brute force
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", sorted(CLOUDS))
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("dims", [2, 3])
@pytest.mark.parametrize("s", [0.5, 1.0, 2.5])
def test_radius_equals_brute_force(name, flavor, dims, s):
    xyz = CLOUDS[name](5)
    ix = oracle.OracleIndex(xyz, s, dims=dims, flavor=flavor)
    pts = ix.point_arrays()["x32"].T
    rng = np.random.default_rng(1)
    q = rng.choice(len(xyz), 120, replace=False).astype(np.int32)
    for r in (0.0, 0.35, 1.0, 2.5):
        off, nbr = ix.radius(r, pidx=q)
        got = csr_rows(off, nbr)
        want = brute_radius(pts, pts[q], r)
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("kernel", ["cube", "cylinder"])
@pytest.mark.parametrize("name", sorted(CLOUDS))
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("dims,s", [(3, 0.5), (3, 1.0), (2, 2.5)])
def test_other_kernels_equal_brute_force(kernel, name, flavor, dims, s):
    """Alg. 1 with the cube and cylinder kernels (Section 2, Section 3.4.1)
    against brute force, point and coordinate queries, r = 0 included."""
    xyz = CLOUDS[name](6)
    ix = oracle.OracleIndex(xyz, s, dims=dims, flavor=flavor)
    pts = ix.point_arrays()["x32"].T
    rng = np.random.default_rng(3)
    q = rng.choice(len(xyz), 100, replace=False).astype(np.int32)
    qa = rng.uniform(xyz.min(0) - 2.0, xyz.max(0) + 2.0, (60, 3))
    for r in (0.0, 0.35, 1.0, 2.5):
        off, nbr = ix.radius(r, pidx=q, kernel=kernel)
        for a, b in zip(csr_rows(off, nbr), brute_kernel(pts, pts[q], r, kernel)):
            np.testing.assert_array_equal(a, b)
        off, nbr = ix.radius(r, qxyz=qa, kernel=kernel)
        for a, b in zip(csr_rows(off, nbr), brute_kernel(pts, _q32(ix, qa), r, kernel)):
            np.testing.assert_array_equal(a, b)


def test_cylinder_ignores_z_and_contains_the_sphere():
    """A cylinder query's rows do not depend on the query's z, even far
    outside the cloud's z range; the sphere's rows are subsets (exactly, in
    FP32: adding fl32(dz^2) >= 0 cannot lower the sum)."""
    xyz = _als(9)
    ix = oracle.OracleIndex(xyz, 1.0)
    rng = np.random.default_rng(4)
    qa = xyz[rng.choice(len(xyz), 150, replace=False)].copy()
    for r in (0.5, 2.0):
        off0, nbr0 = ix.radius(r, qxyz=qa, kernel="cylinder")
        for dz in (-37.0, 55.5):
            qz = qa.copy()
            qz[:, 2] += dz
            off1, nbr1 = ix.radius(r, qxyz=qz, kernel="cylinder")
            for a, b in zip(csr_rows(off0, nbr0), csr_rows(off1, nbr1)):
                np.testing.assert_array_equal(a, b)
        offs, nbrs = ix.radius(r, qxyz=qa)
        for a, b in zip(csr_rows(offs, nbrs), csr_rows(off0, nbr0)):
            assert np.isin(a, b).all()
        assert (np.diff(off0) >= np.diff(offs)).all()


@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
def test_radius_coordinate_queries_outside_bbox(flavor):
    xyz = _als(7)
    ix = oracle.OracleIndex(xyz, 1.0, flavor=flavor)
    pts = ix.point_arrays()["x32"].T
    rng = np.random.default_rng(2)
    lo, hi = xyz.min(0), xyz.max(0)
    qa = rng.uniform(lo - 3.0, hi + 3.0, (200, 3))
    for r in (0.5, 2.0, 4.0):
        off, nbr = ix.radius(r, qxyz=qa)
        want = brute_radius(pts, _q32(ix, qa), r)
        for a, b in zip(csr_rows(off, nbr), want):
            np.testing.assert_array_equal(a, b)


def test_radius_degenerate_cases():
    xyz = _walls(3)
    ix = oracle.OracleIndex(xyz, 0.5)
    pts = ix.point_arrays()["x32"].T
    n = len(xyz)
    # r larger than the bounding-box diagonal: every point
    off, nbr = ix.radius(100.0, pidx=np.arange(0, n, 37, dtype=np.int32))
    assert (np.diff(off) == n).all()
    # r = 0: the point itself plus its exact duplicates
    q = np.arange(n, dtype=np.int32)
    off, nbr = ix.radius(0.0, pidx=q)
    for t, row in enumerate(csr_rows(off, nbr)):
        same = np.nonzero((pts == pts[t]).all(1))[0]
        np.testing.assert_array_equal(row, same)
    # a single-point cloud
    one = oracle.OracleIndex(np.array([[1.0, 2.0, 3.0]]), 1.0)
    assert list(one.ncell) == [1, 1, 1]
    off, nbr = one.radius(0.0, pidx=np.array([0], np.int32))
    assert off.tolist() == [0, 1] and nbr.tolist() == [0]


def test_radius_symmetry_and_monotonicity():
    xyz = _als(9, 3000)
    ix = oracle.OracleIndex(xyz, 1.0)
    n = len(xyz)
    prev = None
    for r in (0.3, 0.7, 1.5, 3.0):
        off, nbr = ix.radius(r)
        rows = np.repeat(np.arange(n), np.diff(off))
        pairs = set(zip(rows.tolist(), nbr.tolist()))
        assert all((b, a) in pairs for a, b in pairs)  # j in N(i) <=> i in N(j)
        assert all((a, a) in pairs for a in range(n))  # self included
        if prev is not None:
            assert prev <= pairs  # monotone in r
        prev = pairs


def test_distance_error_bound():
    # the FP32 distance stays within a few ulps of the exact FP64 value
    rng = np.random.default_rng(0)
    a = rng.uniform(0, 1000, (5000, 3)).astype(np.float32)
    b = (a + rng.normal(0, 3, a.shape)).astype(np.float32)
    D = np.array([sq_dist_rows(a[t:t + 1], b[t:t + 1])[0, 0] for t in range(len(a))])
    exact = ((a.astype(np.float64) - b.astype(np.float64)) ** 2).sum(1)
    assert (np.abs(D - exact) <= 4 * 2.0 ** -24 * exact + 1e-30).all()


# --------------------------------------------------------------------------
# Alg. 2 -- k-NN == brute force (stable sort by (D, index))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", sorted(CLOUDS))
@pytest.mark.parametrize("flavor", ["dense", "sparse", "mixed"])
@pytest.mark.parametrize("dims", [2, 3])
@pytest.mark.parametrize("s", [0.5, 2.5])
def test_knn_equals_brute_force(name, flavor, dims, s):
    xyz = CLOUDS[name](4)
    ix = oracle.OracleIndex(xyz, s, dims=dims, flavor=flavor)
    pts = ix.point_arrays()["x32"].T
    rng = np.random.default_rng(3)
    q = rng.choice(len(xyz), 100, replace=False).astype(np.int32)
    for k in (1, 8, 33):
        idx, d2 = ix.knn(k, pidx=q)
        bi, bd = brute_knn(pts, pts[q], k)
        np.testing.assert_array_equal(idx, bi)
        np.testing.assert_array_equal(d2, bd)


def test_knn_coordinate_queries_and_rmax():
    xyz = _als(8)
    ix = oracle.OracleIndex(xyz, 1.0, flavor="sparse")
    pts = ix.point_arrays()["x32"].T
    rng = np.random.default_rng(5)
    qa = rng.uniform(xyz.min(0) - 5.0, xyz.max(0) + 5.0, (150, 3))
    for rmax in (math.inf, 0.7, 2.0):
        idx, d2 = ix.knn(12, r_max=rmax, qxyz=qa)
        bi, bd = brute_knn(pts, _q32(ix, qa), 12, r_max=rmax)
        np.testing.assert_array_equal(idx, bi)
        np.testing.assert_array_equal(d2, bd)


def test_knn_invariants():
    xyz = _walls(6, 600)
    n = len(xyz)
    ix = oracle.OracleIndex(xyz, 0.5, flavor="mixed")
    q = np.arange(0, n, 7, dtype=np.int32)
    i8, d8 = ix.knn(8, pidx=q)
    i20, d20 = ix.knn(20, pidx=q)
    np.testing.assert_array_equal(i20[:, :8], i8)  # k-prefix
    np.testing.assert_array_equal(d20[:, :8], d8)
    # k > N: all N points, then padding
    ib, db = ix.knn(n + 5, pidx=q[:3])
    assert (ib[:, :n] >= 0).all() and (ib[:, n:] == -1).all() and np.isinf(db[:, n:]).all()
    assert all(sorted(row[:n].tolist()) == list(range(n)) for row in ib)
    # d2[k-1] <= R  <=>  |N_r| >= k
    r = 0.8
    off, _ = ix.radius(r, pidx=q)
    R = np.float32(r) * np.float32(r)
    np.testing.assert_array_equal(d20[:, 19] <= R, np.diff(off) >= 20)
    # first neighbour is the point itself unless a duplicate has a lower index
    pts = ix.point_arrays()["x32"].T
    for t, p in enumerate(q):
        dup = np.nonzero((pts == pts[p]).all(1))[0]
        assert i8[t, 0] == dup.min() and d8[t, 0] == 0.0


# --------------------------------------------------------------------------
# mixed flavor: a slice is dense once 80 % of its voxels hold points
# --------------------------------------------------------------------------
def test_mixed_slice_rule():
    nx, ny = 10, 10
    need = math.ceil(0.8 * nx * ny)  # 80 voxels
    for filled, dense in ((need, True), (need - 1, False)):
        cells = [(i, j) for i in range(nx) for j in range(ny)][:filled]
        pts = [[i + 0.5, j + 0.5, 0.5] for i, j in cells]
        pts += [[0.0, 0.0, 0.0], [nx - 0.01, ny - 0.01, 1.99]]  # corners; slice 1 sparse
        ix = oracle.OracleIndex(np.array(pts), 1.0, flavor="mixed")
        ne, de = ix.slices()
        assert list(ix.ncell) == [nx, ny, 2]
        assert ne[0] == filled + (0 if (0, 0) in cells else 1)
        assert bool(de[0]) == dense and not de[1]


# --------------------------------------------------------------------------
# aggregation (project addition): FP64 forward and analytic gradient
# --------------------------------------------------------------------------
def _agg_case(seed=0, n=60, q=15, k=6, c=4):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1.0, (n, 3))
    f = rng.standard_normal((n, c))
    qidx = rng.choice(n, q, replace=False).astype(np.int32)
    nbr = rng.integers(-1, n, (q, k)).astype(np.int32)
    nbr[:, 0] = qidx  # self in the list
    return x, f, qidx, nbr


def test_agg_special_cases():
    x, f, qidx, nbr = _agg_case()
    # sigma -> infinity: every weight is 1, out = plain sum of the features
    out = oracle.agg_forward(x, qidx, nbr, f, 1e9)
    want = np.stack([f[row[row >= 0]].sum(0) for row in nbr])
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=1e-12)
    # a neighbour list holding only the centre itself returns its feature
    only = np.full_like(nbr, -1); only[:, 0] = qidx
    np.testing.assert_array_equal(oracle.agg_forward(x, qidx, only, f, 0.3), f[qidx])
    # two points at distance d: out = f[q] + exp(-d^2 / (2 sigma^2)) f[j]
    x2 = np.array([[0.0, 0, 0], [0.3, 0.4, 0]]); f2 = np.array([[1.0, 2.0], [3.0, -1.0]])
    o = oracle.agg_forward(x2, np.array([0], np.int32), np.array([[0, 1]], np.int32), f2, 0.5)
    w = math.exp(-0.25 / 0.5)
    np.testing.assert_allclose(o[0], [1 + 3 * w, 2 - w], rtol=1e-14)


def test_agg_gradient_finite_differences():
    x, f, qidx, nbr = _agg_case(1)
    sigma = 0.35
    rng = np.random.default_rng(9)
    g = rng.standard_normal((len(qidx), f.shape[1]))
    gx, gf = oracle.agg_backward(x, qidx, nbr, f, sigma, g)

    def L(xx, ff):
        return float((oracle.agg_forward(xx, qidx, nbr, ff, sigma) * g).sum())

    h = 1e-6
    num_x = np.zeros_like(x)
    for p in range(x.shape[0]):
        for a in range(3):
            e = np.zeros_like(x); e[p, a] = h
            num_x[p, a] = (L(x + e, f) - L(x - e, f)) / (2 * h)
    num_f = np.zeros_like(f)
    for p in range(f.shape[0]):
        for c in range(f.shape[1]):
            e = np.zeros_like(f); e[p, c] = h
            num_f[p, c] = (L(x, f + e) - L(x, f - e)) / (2 * h)
    np.testing.assert_allclose(gx, num_x, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(gf, num_f, rtol=1e-6, atol=1e-7)


def test_invalid_queries_are_empty():
    """A point index outside the cloud or a non-finite coordinate names no
    centre: an empty radius row and a k-NN row of (-1, +inf)."""
    rng = np.random.default_rng(77)
    xyz = rng.uniform(0, 10, (500, 3))
    ox = oracle.OracleIndex(xyz, 1.0)
    q = np.array([3, -1, 500, 10**6, 7], np.int32)
    off, nbr = ox.radius(2.0, pidx=q)
    c = np.diff(off)
    assert c[0] > 0 and c[4] > 0 and (c[1:4] == 0).all()
    idx, d2 = ox.knn(5, pidx=q)
    assert (idx[1:4] == -1).all() and np.isinf(d2[1:4]).all() and (idx[[0, 4]] >= 0).all()
    qa = np.array([[1.0, 2.0, 3.0], [np.nan, 1.0, 1.0], [1.0, np.inf, 0.0]])
    off, nbr = ox.radius(2.0, qxyz=qa)
    assert np.diff(off)[0] > 0 and (np.diff(off)[1:] == 0).all()
    idx, d2 = ox.knn(4, qxyz=qa)
    assert (idx[1:] == -1).all() and (idx[0] >= 0).all()


@pytest.mark.parametrize("name", ["als", "walls"])
def test_knn_monotonic_schedule_same_lists(name):
    """Alg. 2 with monotonic radius growth (the baseline of Section 3.5)
    returns brute force's lists, like density growth, and both count the
    voxels they visit."""
    xyz = CLOUDS[name](12)
    ox = oracle.OracleIndex(xyz, 0.5)
    q = np.arange(0, len(xyz), 7, dtype=np.int32)
    i1, d1, v1 = ox.knn(10, pidx=q, visited=True)
    i2, d2, v2 = ox.knn(10, pidx=q, visited=True, schedule="monotonic")
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_array_equal(d1, d2)
    pts = ox.point_arrays()["x32"].T
    bi, bd = brute_knn(pts, pts[q], 10)
    np.testing.assert_array_equal(i2, bi)
    np.testing.assert_array_equal(d2, bd)
    assert (v1 > 0).all() and (v2 > 0).all()


def _lattice():
    """Points at the centres of a 10 x 10 x 10 block of unit voxels, plus
    two frame points at (0,0,0) and (10,10,10) so that p- = 0 and voxel
    walls lie on the integers; query: the point at (5.5, 5.5, 5.5)."""
    g = np.arange(10, dtype=np.float64) + 0.5
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pts = np.vstack([pts, [[0.0, 0.0, 0.0], [10.0, 10.0, 10.0]]])
    q = int(np.flatnonzero((pts == 5.5).all(1))[0])
    return pts, q


# Worked by hand from Alg. 2 (Section 3.4.2) on the lattice above, voxel
# edge 1: the start radius is the distance to the nearest wall, 0.5 (Eq. 11);
# the box of B(c, r), padded by 2^-18 r, spans voxels floor(5.5 - r') ..
# floor(5.5 + r'), i.e. 3, 5, 7 per axis at r = 0.5, 1.5, 2.5, and 5 at the
# density radii 1.54 (k = 7) and 2.19 (k = 20).  Lattice neighbours at
# squared distance <= 0, 2, 4, 6 number 1, 19, 33, 81.  Density growth:
# r = (k / rho)^(1/3) with rho = 1 / ((4/3) pi 0.5^3) (Eq. 12).  Monotonic
# growth: r = 0.5, 1.5, 2.5, ...
@pytest.mark.parametrize("k,dens,mono", [(1, 27, 27), (7, 125, 125), (20, 125, 343),
                                         (33, 343, 343)])
def test_knn_visited_voxels_lattice(k, dens, mono):
    pts, q = _lattice()
    ox = oracle.OracleIndex(pts, 1.0, flavor="dense")
    _, _, vd = ox.knn(k, pidx=np.array([q], np.int32), visited=True)
    _, _, vm = ox.knn(k, pidx=np.array([q], np.int32), visited=True, schedule="monotonic")
    assert (int(vd[0]), int(vm[0])) == (dens, mono)


def test_knn_growth_stats_file_current():
    """The stored density-vs-monotonic statistic (written by the oracle-only
    script beside it) is what the oracle gives now, on its row closest to
    the split Section 3.5 reports (voxel edge 2 m, k = 8)."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "mkstats", os.path.join(os.path.dirname(__file__), "golden", "make_knn_growth_stats.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    rows = {(float(c), int(v[0])): tuple(int(x) for x in v[1:])
            for c, vals in golden("knn_growth_stats.txt").items() for v in vals}
    got = next(mk.rows(8, cells=[2.0], ks=[8]))
    assert rows[(2.0, 8)] == tuple(got[2:])
    assert sum(rows[(2.0, 8)][:3]) == 1_000_000
