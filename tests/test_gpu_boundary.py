"""The C ABI's contract on the GPU: fills never write outside nbr[0, total),
allocation failures leak nothing and leave outputs untouched, capacity
limits are reported, calls on a non-current stream and concurrent searches
on one index give the same results, and the exported FP32 frame is the
oracle's recentring (Section 3.1, Eq. 1)."""
import ctypes

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


def _cloud(seed=5, n=30_000):
    return cloudgen.small_als(seed, n)


def test_fill_clipped_to_total():
    """Offsets from a larger radius with the total of a smaller one: the fill
    writes inside nbr[0, total) only; the guard region behind it (the same
    allocation) keeps its sentinel."""
    from paper_2502_11602_amd import GridIndex
    from paper_2502_11602_amd._lib import Queries, lib
    dev = _dev()
    gi = GridIndex(torch.from_numpy(_cloud()).to(dev), cell=1.0)
    off_big, tot_big = gi.radius_count(2.0)
    _, tot_small = gi.radius_count(0.5)
    assert tot_big > 4 * tot_small > 0
    guard = 1 << 16
    buf = torch.full((tot_small + guard,), -7, dtype=torch.int32, device=dev)
    q = Queries(None, None, gi.n)
    st = lib().chs_radius_fill(gi._h, ctypes.byref(q), ctypes.c_float(2.0), off_big.data_ptr(),
                               buf.data_ptr(), tot_small, None)
    assert st == 0
    torch.cuda.synchronize()
    assert bool((buf[tot_small:] == -7).all())
    assert bool((buf[:tot_small] >= 0).all())  # the rows that fit were written
    # garbage offsets (negative, decreasing, beyond total): nothing outside
    bad = off_big.clone()
    bad[1::3] = -5
    bad[2::7] = tot_big * 4
    buf.fill_(-7)
    st = lib().chs_radius_fill(gi._h, ctypes.byref(q), ctypes.c_float(2.0), bad.data_ptr(),
                               buf.data_ptr(), tot_small, None)
    assert st == 0
    torch.cuda.synchronize()
    assert bool((buf[tot_small:] == -7).all())
    # the binding checks what it can on the host
    with pytest.raises(ValueError):
        gi.radius_fill(2.0, off_big.to(torch.int32), tot_big)
    with pytest.raises(ValueError):
        gi.radius_fill(2.0, off_big, tot_big, out=torch.empty(tot_big - 1, dtype=torch.int32,
                                                               device=dev))


class _CountingAllocator:
    """chs_allocator over torch's caching allocator that fails on the n-th
    request (0: never) and tracks what is live."""

    def __init__(self, device, fail_at=0):
        from paper_2502_11602_amd import _lib
        self.device = device
        self.fail_at = fail_at
        self.calls = 0
        self.live = set()

        def _alloc(nbytes, ctx):
            self.calls += 1
            if self.fail_at and self.calls == self.fail_at:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                   torch.cuda.current_stream(self.device))
            self.live.add(p)
            return p

        def _free(p, ctx):
            if p:
                self.live.discard(p)
                torch.cuda.caching_allocator_delete(p)

        self._a = _lib.ALLOC_FN(_alloc)
        self._f = _lib.FREE_FN(_free)
        self.struct = _lib.Allocator(self._a, self._f, None)


def _build(xyz_t, al, flavor=0, max_dense=0):
    from paper_2502_11602_amd._lib import BuildParams, lib
    p = BuildParams(flavor, 3, (ctypes.c_double * 3)(1.0, 1.0, 1.0), 80, 0, max_dense)
    h = ctypes.c_void_p()
    st = lib().chs_build(xyz_t.data_ptr(), xyz_t.shape[0], ctypes.byref(p), ctypes.byref(al.struct),
                         None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("flavor", [0, 1, 2])
def test_build_nomem_every_allocation(flavor):
    """A build whose n-th allocation fails returns CHS_E_NOMEM, leaves *out
    NULL and releases everything it had allocated, for every n."""
    from paper_2502_11602_amd._lib import lib
    dev = _dev()
    xyz = torch.from_numpy(_cloud(6, 20_000)).to(dev)
    ok = _CountingAllocator(dev)
    st, h = _build(xyz, ok, flavor)
    assert st == 0 and h.value
    n_calls = ok.calls
    lib().chs_free(h)
    torch.cuda.synchronize()
    assert not ok.live
    assert n_calls > 5
    for n in range(1, n_calls + 1):
        al = _CountingAllocator(dev, fail_at=n)
        st, h = _build(xyz, al, flavor)
        torch.cuda.synchronize()
        assert st == 2, (n, st)
        assert not h.value
        assert not al.live, f"allocation {n} failing leaked {len(al.live)} buffers"
        assert b"NULL" in lib().chs_last_error()


def test_search_nomem_leaves_outputs():
    """k-NN and radius searches whose temporaries cannot be allocated return
    CHS_E_NOMEM, write nothing to idx / d2 / *nbr and leak nothing."""
    from paper_2502_11602_amd._lib import Queries, lib
    dev = _dev()
    xyz = torch.from_numpy(_cloud(7, 20_000)).to(dev)
    al = _CountingAllocator(dev)
    st, h = _build(xyz, al)
    assert st == 0
    base = set(al.live)
    qi = torch.arange(0, 20_000, 7, dtype=torch.int32, device=dev)
    q = Queries(None, qi.data_ptr(), qi.numel())
    for n in (1, 2, 3, 5):
        al.fail_at, al.calls = n, 0
        idx = torch.full((qi.numel(), 8), -9, dtype=torch.int32, device=dev)
        d2 = torch.full((qi.numel(), 8), -9.0, dtype=torch.float32, device=dev)
        st = lib().chs_knn(h, ctypes.byref(q), 8, ctypes.c_float(float("inf")), idx.data_ptr(),
                           d2.data_ptr(), None)
        torch.cuda.synchronize()
        if al.calls < n:  # fewer allocations than n: the call succeeded
            assert st == 0
            continue
        assert st == 2, (n, st)
        assert bool((idx == -9).all()) and bool((d2 == -9.0).all())
        assert al.live == base
    # chs_radius_search: the neighbour array's allocation fails
    al.fail_at, al.calls = 0, 0
    off = torch.empty(qi.numel() + 1, dtype=torch.int64, device=dev)
    nbr_p = ctypes.c_void_p(0x5)
    tot = ctypes.c_int64(-3)
    fail_out = _CountingAllocator(dev, fail_at=1)
    st = lib().chs_radius_search(h, ctypes.byref(q), ctypes.c_float(1.0), ctypes.byref(fail_out.struct),
                                 off.data_ptr(), ctypes.byref(nbr_p), ctypes.byref(tot), None)
    torch.cuda.synchronize()
    assert st == 2 and nbr_p.value == 0x5 and tot.value == -3
    assert not fail_out.live and al.live == base
    lib().chs_free(h)
    torch.cuda.synchronize()
    assert not al.live


def test_dense_capacity():
    """A dense grid above max_dense_cells is refused with CHS_E_CAPACITY (the
    sparse flavor of the same cloud builds)."""
    from paper_2502_11602_amd._lib import lib
    dev = _dev()
    xyz = torch.from_numpy(_cloud(8, 5_000)).to(dev)
    al = _CountingAllocator(dev)
    st, h = _build(xyz, al, flavor=0, max_dense=1000)
    torch.cuda.synchronize()
    assert st == 3 and not h.value and b"exceeds" in lib().chs_last_error()
    assert not al.live
    st, h = _build(xyz, al, flavor=1, max_dense=1000)
    assert st == 0
    lib().chs_free(h)


def test_non_current_stream_and_concurrent_searches():
    """Searches handed a stream that is not current, with allocations and
    frees on the default stream meanwhile, and two persistent searches of
    one index in flight on two streams, return the default-stream results."""
    from paper_2502_11602_amd import GridIndex
    dev = _dev()
    gi = GridIndex(torch.from_numpy(_cloud(9, 60_000)).to(dev), cell=1.0)
    qi = torch.arange(0, 60_000, 3, dtype=torch.int32, device=dev)
    ref_i, ref_d = gi.knn(16, qi)
    ref_o, ref_n = gi.radius(1.5)
    gi.set_persistent(True)
    s1, s2 = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    for _ in range(3):
        i1, d1 = gi.knn(16, qi, stream=s1)
        o2, t2 = gi.radius_count(1.5, stream=s2)
        junk = [torch.empty(1 << 20, device=dev) for _ in range(8)]  # default stream churn
        del junk
        n2 = gi.radius_fill(1.5, o2, t2, stream=s2)
        i2, d2 = gi.knn(16, qi, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(i1, ref_i) and torch.equal(d1, ref_d)
        assert torch.equal(i2, ref_i) and torch.equal(d2, ref_d)
        assert torch.equal(o2, ref_o)
        # (row order inside a CSR row is deterministic)
        assert torch.equal(n2, ref_n)


def test_coords_are_the_oracle_frame():
    from paper_2502_11602_amd import GridIndex
    dev = _dev()
    xyz = _cloud(10, 25_000)
    gi = GridIndex(torch.from_numpy(xyz).to(dev), cell=1.0)
    x32 = gi.coords().cpu().numpy()
    o = oracle.OracleIndex(xyz, 1.0).point_arrays()["x32"]
    np.testing.assert_array_equal(x32, o.T)


def test_fill_by_ranges():
    """A counted query set filled range by range (chs_fill_chunks picks the
    ranges under an entry budget; each range fills with the queries and
    offsets advanced to its start) gives the rows of one whole fill, for
    index and coordinate queries and both radius schedules."""
    from paper_2502_11602_amd import GridIndex
    dev = _dev()
    xyz = _cloud()
    gi = GridIndex(torch.from_numpy(xyz).to(dev), cell=1.0)
    rng = np.random.default_rng(3)
    qi = torch.from_numpy(rng.choice(len(xyz), 5000, replace=False).astype(np.int32)).to(dev)
    qa = torch.from_numpy(rng.uniform(xyz.min(0), xyz.max(0), (4000, 3))).to(dev)
    for sched in ("tiles", "groups"):
        gi.set_radius_schedule(sched)
        for q in (qi, qa):
            off, nbr = gi.radius(2.0, q)
            total = int(off[-1])
            for budget in (total, total // 7 + 1, 1000):
                bounds, eb = gi.fill_chunks(off, budget)
                offc = off.cpu().numpy()
                assert bounds[0] == 0 and bounds[-1] == len(q)
                assert eb == [int(offc[b]) for b in bounds]
                sizes = np.diff(eb)
                assert (sizes <= budget).all()
                # fewest ranges: no range could take the next query too
                for i in range(len(bounds) - 2):
                    assert offc[bounds[i + 1] + 1] - offc[bounds[i]] > budget
                parts = []
                for a, b, part in gi.radius_chunked(2.0, q, budget, offsets=off):
                    rows = np.split(part.cpu().numpy(), offc[a + 1:b] - offc[a])
                    parts += [np.sort(r) for r in rows]
                want = np.split(nbr.cpu().numpy(), offc[1:-1])
                assert len(parts) == len(want)
                for g, w in zip(parts, want):
                    np.testing.assert_array_equal(g, np.sort(w))


def test_fill_chunks_rejects():
    from paper_2502_11602_amd import ChsError
    from paper_2502_11602_amd._lib import lib
    dev = _dev()
    off = torch.tensor([0, 5, 9, 30, 31], dtype=torch.int64, device=dev)
    from paper_2502_11602_amd import GridIndex
    gi = GridIndex(torch.from_numpy(_cloud(n=2000)).to(dev), cell=1.0)
    assert gi.fill_chunks(off, 22) == ([0, 2, 4], [0, 9, 31])
    assert gi.fill_chunks(off, 21) == ([0, 2, 3, 4], [0, 9, 30, 31])
    assert gi.fill_chunks(off, 1000) == ([0, 4], [0, 31])
    with pytest.raises(ChsError):  # query 2 alone holds 21 entries
        gi.fill_chunks(off, 20)
    with pytest.raises(ChsError):  # decreasing offsets
        gi.fill_chunks(torch.tensor([0, 5, 4], dtype=torch.int64, device=dev), 10)
    m = ctypes.c_int64(0)
    b = (ctypes.c_int64 * 2)()
    e = (ctypes.c_int64 * 2)()
    st = lib().chs_fill_chunks(off.data_ptr(), 4, 22, b, e, 2, ctypes.byref(m), None)
    assert st == 3 and m.value == 2  # CHS_E_CAPACITY: 2 ranges need 3 bounds
    st = lib().chs_fill_chunks(off.data_ptr(), 4, 0, None, None, 0, ctypes.byref(m), None)
    assert st == 1
    # an empty set is one bound and no range
    z = torch.zeros(1, dtype=torch.int64, device=dev)
    assert gi.fill_chunks(z, 10) == ([0], [0])


def test_query_order_and_ordered_ranges():
    """chs_query_order is a permutation of the batch; counting and filling
    the reordered queries range by range gives each query its own row."""
    from paper_2502_11602_amd import GridIndex
    dev = _dev()
    xyz = _cloud()
    gi = GridIndex(torch.from_numpy(xyz).to(dev), cell=1.0, flavor="sparse")
    rng = np.random.default_rng(4)
    q = torch.from_numpy(rng.choice(len(xyz), 6000, replace=False).astype(np.int32)).to(dev)
    order = gi.query_order(q)
    assert sorted(order.cpu().tolist()) == list(range(len(q)))
    qs = q[order.long()]
    off, nbr = gi.radius(2.0, q)
    offc, nb = off.cpu().numpy(), nbr.cpu().numpy()
    oc = order.cpu().numpy()
    got = {}
    offs = None
    gen = gi.radius_chunked(2.0, qs, 3000)
    for a, b, part in gen:
        if offs is None:
            offs, _ = gi.radius_count(2.0, qs)
            so = offs.cpu().numpy()
        p = part.cpu().numpy()
        for t in range(a, b):
            got[oc[t]] = np.sort(p[so[t] - so[a]:so[t + 1] - so[a]])
    assert len(got) == len(q)
    for i in range(0, len(q), 7):
        np.testing.assert_array_equal(got[i], np.sort(nb[offc[i]:offc[i + 1]]))
    # every-point queries: the build's plan order, a permutation of the points
    allo = gi.query_order()
    assert sorted(allo.cpu().tolist()) == list(range(len(xyz)))
