"""chs_knn_noalloc, the k-NN entry point that allocates nothing: through the
C ABI its lists equal chs_knn's (Section 3.4.2) on two calls in a row, the
second smaller, for index, coordinate and every-point queries, plain and
persistent launches; the index's allocator is never called; batches beyond
the stated limit are refused before any device work."""
import ctypes
import math

import numpy as np
import pytest

import cloudgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


class _Counting:
    """Allocator that records every request (torch's caching allocator)."""

    def __init__(self, device):
        from paper_2502_11602_amd import _lib
        self.calls = 0

        def _alloc(nbytes, ctx):
            self.calls += 1
            return torch.cuda.caching_allocator_alloc(int(nbytes), device,
                                                      torch.cuda.current_stream(device))

        def _free(p, ctx):
            if p:
                torch.cuda.caching_allocator_delete(p)

        self._a = _lib.ALLOC_FN(_alloc)
        self._f = _lib.FREE_FN(_free)
        self.struct = _lib.Allocator(self._a, self._f, None)


def _noalloc(h, q, k, r_max, nq):
    from paper_2502_11602_amd._lib import lib
    idx = torch.full((nq, k), -5, dtype=torch.int32, device="cuda:0")
    d2 = torch.full((nq, k), -5.0, dtype=torch.float32, device="cuda:0")
    st = lib().chs_knn_noalloc(h, ctypes.byref(q), k, ctypes.c_float(r_max),
                               idx.data_ptr() if nq else None, d2.data_ptr() if nq else None, None)
    return st, idx, d2


def _plain(h, q, k, r_max, nq):
    from paper_2502_11602_amd._lib import lib
    idx = torch.empty((nq, k), dtype=torch.int32, device="cuda:0")
    d2 = torch.empty((nq, k), dtype=torch.float32, device="cuda:0")
    st = lib().chs_knn(h, ctypes.byref(q), k, ctypes.c_float(r_max), idx.data_ptr(),
                       d2.data_ptr(), None)
    assert st == 0
    return idx, d2


@pytest.mark.parametrize("persistent", [False, True])
def test_noalloc_matches_knn(persistent):
    from paper_2502_11602_amd._lib import BuildParams, Queries, lib
    dev = _dev()
    xyz = cloudgen.small_als(21, 60_000)
    x = torch.from_numpy(xyz).to(dev)
    al = _Counting(dev)
    p = BuildParams(0, 3, (ctypes.c_double * 3)(1.0, 1.0, 1.0), 80, 0, 0)
    h = ctypes.c_void_p()
    assert lib().chs_build(x.data_ptr(), x.shape[0], ctypes.byref(p), ctypes.byref(al.struct),
                           None, ctypes.byref(h)) == 0
    assert lib().chs_index_set_option(h, 1, 1 if persistent else 0) == 0
    rng = np.random.default_rng(3)
    # two calls in a row, the second smaller: index queries, then coordinates
    for nq, k, r_max in ((40_000, 16, math.inf), (7_000, 33, 1.5)):
        qi = torch.from_numpy(rng.choice(len(xyz), nq, replace=False).astype(np.int32)).to(dev)
        q = Queries(None, qi.data_ptr(), nq)
        want = _plain(h, q, k, r_max, nq)
        torch.cuda.synchronize()
        before = al.calls
        st, idx, d2 = _noalloc(h, q, k, r_max, nq)
        torch.cuda.synchronize()
        assert st == 0, lib().chs_last_error()
        assert al.calls == before, "chs_knn_noalloc called the allocator"
        assert torch.equal(idx, want[0]) and torch.equal(d2, want[1])
    for nq, k in ((30_000, 8), (3_000, 20)):
        qa = torch.from_numpy(rng.uniform(xyz.min(0) - 2, xyz.max(0) + 2, (nq, 3))).to(dev)
        q = Queries(qa.data_ptr(), None, nq)
        want = _plain(h, q, k, math.inf, nq)
        before = al.calls
        st, idx, d2 = _noalloc(h, q, k, math.inf, nq)
        torch.cuda.synchronize()
        assert st == 0 and al.calls == before
        assert torch.equal(idx, want[0]) and torch.equal(d2, want[1])
    # every point
    q = Queries(None, None, len(xyz))
    want = _plain(h, q, 12, math.inf, len(xyz))
    before = al.calls
    st, idx, d2 = _noalloc(h, q, 12, math.inf, len(xyz))
    torch.cuda.synchronize()
    assert st == 0 and al.calls == before
    assert torch.equal(idx, want[0]) and torch.equal(d2, want[1])
    lib().chs_free(h)


def test_noalloc_limit_and_binding():
    from paper_2502_11602_amd import ChsError, GridIndex
    dev = _dev()
    xyz = cloudgen.small_als(22, 20_000)
    gi = GridIndex(torch.from_numpy(xyz).to(dev), cell=1.0)
    nq = (1 << 19) + 1
    qi = torch.zeros(nq, dtype=torch.int32, device=dev)
    idx = torch.full((nq, 4), -5, dtype=torch.int32, device=dev)
    d2 = torch.full((nq, 4), -5.0, dtype=torch.float32, device=dev)
    with pytest.raises(ChsError, match="CHS_E_CAPACITY"):
        gi.knn_noalloc(4, idx, d2, qi)
    torch.cuda.synchronize()
    assert bool((idx == -5).all())
    qi = torch.arange(0, 20_000, 5, dtype=torch.int32, device=dev)
    a = gi.knn(10, qi)
    b = gi.knn_noalloc(10, torch.empty_like(a[0]), torch.empty_like(a[1]), qi)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
