"""Python face of the GPU grid index: marshals torch device tensors into the
C ABI of libchs.so.  PyTorch provides device memory, streams and (for the
aggregation) autograd glue; the index, the searches and their results are
computed by the library's HIP kernels."""
import contextlib
import ctypes
import math

import torch

from . import _lib
from ._lib import BuildParams, IndexArrays, IndexInfo, Queries, check, lib


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


@contextlib.contextmanager
def _on(device, stream=None):
    """Make `device` and `stream` current for a library call: the allocator
    then hands out (and takes back) temporaries on the stream the call's
    kernels run on."""
    with torch.cuda.device(device):
        if stream is None:
            yield
        else:
            with torch.cuda.stream(stream):
                yield


class TorchAllocator:
    """chs_allocator backed by PyTorch's caching allocator on the current
    stream, so library temporaries and index memory are stream-ordered (the
    methods below make the call's stream current around every call)."""

    def __init__(self, device):
        self.device = device
        self._live = {}

        def _alloc(nbytes, ctx):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                       torch.cuda.current_stream(self.device))
                return p
            except Exception:  # out of memory -> NULL -> CHS_E_NOMEM
                return None

        def _free(p, ctx):
            if p:
                torch.cuda.caching_allocator_delete(p)

        self._cb_alloc = _lib.ALLOC_FN(_alloc)
        self._cb_free = _lib.FREE_FN(_free)
        self.struct = _lib.Allocator(self._cb_alloc, self._cb_free, None)


class _DevView:
    """A borrowed device array exposed through __cuda_array_interface__."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 2}


def _view(ptr, shape, typestr, device):
    if not ptr or any(s == 0 for s in shape):
        return None
    return torch.as_tensor(_DevView(ptr, shape, typestr), device=device)


def _queries(queries, n):
    """Build a chs_queries struct; returns (struct, nq, keepalive)."""
    if queries is None:
        return Queries(None, None, n), n, None
    if not queries.is_cuda:
        raise ValueError("queries must be a CUDA (HIP) tensor")
    if queries.dtype == torch.int32 and queries.dim() == 1:
        q = queries.contiguous()
        return Queries(None, q.data_ptr() if q.numel() else None, q.numel()), q.numel(), q
    if queries.dtype == torch.float64 and queries.dim() == 2 and queries.shape[1] == 3:
        q = queries.contiguous()
        return Queries(q.data_ptr() if q.numel() else None, None, q.shape[0]), q.shape[0], q
    raise ValueError("queries: int32 [nq] point indices or float64 [nq,3] coordinates")


def _params(cell, dims, flavor, mixed_dense_pct, max_dense_cells):
    c = [float(cell)] * 3 if not hasattr(cell, "__len__") else [float(v) for v in cell]
    return BuildParams(_lib.FLAVORS[flavor], dims, (ctypes.c_double * 3)(*c), mixed_dense_pct, 0,
                       max_dense_cells)


class GridIndex:
    """Cheesemap grid index over a cloud ``xyz`` (float64 [n,3] on the GPU).

    flavor: "dense" | "sparse" | "mixed" (Section 3.3); dims: 3 or 2;
    cell: voxel edge in metres (scalar or per axis).

    With ``tile_off`` (host sequence of ntiles+1 point offsets) the index is
    a batch of independent tiles stored back to back in ``xyz``; ``cell``
    may then be one value per tile.  Searches on a batched index take every
    point as a query (of its own tile) and return tile-local indices.
    ``frames`` (per tile: min x, y, z, max x, y, z) makes the batched build
    read nothing back from the device (it can be captured in a graph)."""

    def __init__(self, xyz, cell=1.0, dims=3, flavor="dense", mixed_dense_pct=80,
                 max_dense_cells=0, stream=None, tile_off=None, frames=None):
        if not (isinstance(xyz, torch.Tensor) and xyz.is_cuda and xyz.dtype == torch.float64):
            raise ValueError("xyz must be a float64 CUDA tensor [n,3]")
        if xyz.dim() != 2 or xyz.shape[1] != 3:
            raise ValueError("xyz must have shape [n,3]")
        self.device = xyz.device
        self._alloc = TorchAllocator(self.device)
        xyz = xyz.contiguous()
        h = ctypes.c_void_p()
        self._h = None
        self.ntiles = 1
        self._build_stream = stream
        with _on(self.device, stream):
            if tile_off is None:
                p = _params(cell, dims, flavor, mixed_dense_pct, max_dense_cells)
                st = lib().chs_build(xyz.data_ptr(), xyz.shape[0], ctypes.byref(p),
                                     ctypes.byref(self._alloc.struct), _stream(stream),
                                     ctypes.byref(h))
                check(st, "chs_build")
            else:
                toff = [int(v) for v in tile_off]
                T = len(toff) - 1
                cells = list(cell) if (hasattr(cell, "__len__") and len(cell) == T) else [cell] * T
                arr = (BuildParams * T)(*[_params(c, dims, flavor, mixed_dense_pct,
                                                  max_dense_cells) for c in cells])
                toff_c = (ctypes.c_int64 * (T + 1))(*toff)
                if frames is None:
                    st = lib().chs_build_batch(xyz.data_ptr(), xyz.shape[0], toff_c, T, arr,
                                               ctypes.byref(self._alloc.struct), _stream(stream),
                                               ctypes.byref(h))
                    check(st, "chs_build_batch")
                else:
                    fr = [float(v) for f in frames for v in f]
                    if len(fr) != 6 * T:
                        raise ValueError("frames: 6 values (min x, y, z, max x, y, z) per tile")
                    fr_c = (ctypes.c_double * (6 * T))(*fr)
                    st = lib().chs_build_batch_framed(xyz.data_ptr(), xyz.shape[0], toff_c, T, arr,
                                                      fr_c, ctypes.byref(self._alloc.struct),
                                                      _stream(stream), ctypes.byref(h))
                    check(st, "chs_build_batch_framed")
                self.ntiles = T
                self.tile_off = toff
        self._h = h
        self.n = xyz.shape[0]
        self.flavor = flavor
        self.dims = dims

    def set_persistent(self, on=True):
        """Persistent searches: one wave per hardware slot pulling 64-query
        work items from a device counter (default for batched indexes)."""
        check(lib().chs_index_set_option(self._h, 1, 1 if on else 0), "chs_index_set_option")

    def set_knn_schedule(self, schedule="rings"):
        """k-NN voxel schedule: "rings" (default), "density" (Alg. 2's
        density-growth radius), "monotonic" (the radius grows by the
        smallest voxel edge per step) or "solo" (one query at a time, for
        sparse query sets); the results are identical."""
        check(lib().chs_index_set_option(self._h, 4, {"rings": 0, "density": 1,
                                                      "monotonic": 2, "solo": 3}[schedule]),
              "chs_index_set_option")

    def tile_info(self, t):
        inf = IndexInfo()
        check(lib().chs_tile_info(self._h, t, ctypes.byref(inf)), "chs_tile_info")
        return dict(origin=list(inf.origin), max32=list(inf.max32), cell=list(inf.cell),
                    ncell=list(inf.ncell), n_points=inf.n_points, dims=inf.dims)

    def set_radius_schedule(self, schedule="auto"):
        """Work sharing of the kernel-based searches: "tiles" (64 queries
        per union box), "groups" (8 queries per box) or "auto"; results are
        identical."""
        check(lib().chs_index_set_option(self._h, 6, {"auto": 0, "tiles": 1, "groups": 2}[schedule]),
              "chs_index_set_option")

    def set_fill_stage(self, entries=0):
        """LDS entries per query of the radius fill (16, 24, 32, 64; 0 = by
        the mean row length); results are identical."""
        check(lib().chs_index_set_option(self._h, 5, int(entries)), "chs_index_set_option")

    def coords(self, stream=None):
        """The index's FP32 coordinates in input order ([n,3] float32): the
        library's recentring fl32(p - p-) (each tile in its own frame)."""
        out = torch.empty((self.n, 3), dtype=torch.float32, device=self.device)
        with _on(self.device, stream):
            check(lib().chs_index_coords(self._h, out.data_ptr(), _stream(stream)),
                  "chs_index_coords")
        return out

    def close(self):
        if getattr(self, "_h", None):
            with _on(self.device, self._build_stream):
                lib().chs_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        inf = IndexInfo()
        check(lib().chs_index_info(self._h, ctypes.byref(inf)), "chs_index_info")
        return dict(origin=list(inf.origin), max32=list(inf.max32), cell=list(inf.cell),
                    ncell=list(inf.ncell), n_points=inf.n_points, n_nonempty=inf.n_nonempty,
                    n_dense_slices=inf.n_dense_slices, device_bytes=inf.device_bytes,
                    flavor=inf.flavor, dims=inf.dims, ntiles=inf.ntiles)

    def arrays(self):
        """Copies of the index's device arrays (for inspection and tests)."""
        a = IndexArrays()
        check(lib().chs_index_arrays(self._h, ctypes.byref(a)), "chs_index_arrays")
        inf = self.info()
        n, m, d = self.n, inf["n_nonempty"], self.device
        nc = inf["ncell"][0] * inf["ncell"][1] * inf["ncell"][2]
        out = dict(
            perm=_view(a.perm, (n,), "<i4", d),
            inv_perm=_view(a.inv_perm, (n,), "<i4", d),
            sorted_xyz=_view(a.sorted_xyz, (3, n), "<f4", d),
            points=_view(a.points, (n, 4), "<f4", d),
            cell_keys=_view(a.cell_keys, (m,), "<u8", d),
            cell_start=_view(a.cell_start, (m + 1,), "<i4", d),
            dense_start=_view(a.dense_start, (nc + 1,), "<i4", d) if a.dense_start else None,
            slice_dense=_view(a.slice_dense, (inf["ncell"][2],), "|u1", d) if a.slice_dense else None,
        )
        torch.cuda.current_stream(d).synchronize()
        return {k: (None if v is None else v.clone()) for k, v in out.items()}

    # ---- fixed-radius search (Alg. 1)
    KERNELS = {"sphere": 0, "cube": 1, "cylinder": 2}

    def radius_count(self, r, queries=None, stream=None, kernel="sphere", sync=True, out=None):
        """Row offsets (int64 [nq+1]) and total of a kernel search; kernel is
        "sphere", "cube" (half side r) or "cylinder" (radius r, any z).  With
        sync=False the total is not read back (None; it is offsets[-1]) and
        nothing waits for the stream.  ``out``: preallocated offsets."""
        q, nq, keep = _queries(queries, self.n)
        off = out if out is not None else torch.empty(nq + 1, dtype=torch.int64, device=self.device)
        tot = ctypes.c_int64(0)
        with _on(self.device, stream):
            check(lib().chs_kernel_count(self._h, ctypes.byref(q), self.KERNELS[kernel],
                                         ctypes.c_float(r), off.data_ptr(),
                                         ctypes.byref(tot) if sync else None,
                                         _stream(stream)), "chs_kernel_count")
        return off, (tot.value if sync else None)

    def radius_fill(self, r, offsets, total, queries=None, out=None, stream=None, kernel="sphere"):
        """Fill pass into ``out`` (int32, at least ``total`` entries) or a new
        tensor; ``offsets`` as returned by radius_count."""
        q, nq, keep = _queries(queries, self.n)
        total = int(total)
        if not (isinstance(offsets, torch.Tensor) and offsets.dtype == torch.int64
                and offsets.shape == (nq + 1,) and offsets.device == self.device
                and offsets.is_contiguous()):
            raise ValueError(f"offsets must be a contiguous int64 [{nq + 1}] tensor on {self.device}")
        if total < 0:
            raise ValueError("total must be >= 0")
        if out is not None and not (out.dtype == torch.int32 and out.device == self.device
                                    and out.is_contiguous() and out.numel() >= total):
            raise ValueError(f"out must be a contiguous int32 tensor on {self.device} "
                             f"with at least {total} entries")
        nbr = out if out is not None else torch.empty(total, dtype=torch.int32,
                                                      device=self.device)
        with _on(self.device, stream):
            check(lib().chs_kernel_fill(self._h, ctypes.byref(q), self.KERNELS[kernel],
                                        ctypes.c_float(r), offsets.data_ptr(),
                                        nbr.data_ptr() if total else None, total,
                                        _stream(stream)), "chs_kernel_fill")
        return nbr

    def query_order(self, queries=None, stream=None):
        """int32 [nq]: the caller's query indices in the order the searches
        process them (spatially coherent; chs_query_order)."""
        q, nq, keep = _queries(queries, self.n)
        order = torch.empty(nq, dtype=torch.int32, device=self.device)
        with _on(self.device, stream):
            check(lib().chs_query_order(self._h, ctypes.byref(q), order.data_ptr() if nq else None,
                                        _stream(stream)), "chs_query_order")
        return order

    def fill_chunks(self, offsets, max_entries, stream=None):
        """Query ranges whose fills each hold at most max_entries entries
        (chs_fill_chunks): host lists bounds [q_0 = 0, ..., q_m = nq] and
        entry_bounds [offsets[q_i]]."""
        nq = offsets.numel() - 1
        m = ctypes.c_int64(0)
        with _on(self.device, stream):
            check(lib().chs_fill_chunks(offsets.data_ptr(), nq, int(max_entries), None, None, 0,
                                        ctypes.byref(m), _stream(stream)), "chs_fill_chunks")
            b = (ctypes.c_int64 * (m.value + 1))()
            e = (ctypes.c_int64 * (m.value + 1))()
            check(lib().chs_fill_chunks(offsets.data_ptr(), nq, int(max_entries), b, e,
                                        m.value + 1, ctypes.byref(m), _stream(stream)),
                  "chs_fill_chunks")
        return list(b), list(e)

    def radius_chunked(self, r, queries, max_entries, stream=None, kernel="sphere",
                       offsets=None):
        """Count all queries (index or coordinate queries), then yield
        (a, b, nbr) per range of queries [a, b) whose neighbour rows fit
        max_entries entries: nbr is a view of one reused int32 buffer holding
        the range's CSR rows (offsets[a:b+1] - offsets[a]); it is overwritten
        by the next range.  Returns the offsets of all queries when exhausted
        (StopIteration.value)."""
        if queries is None:
            raise ValueError("ranges need explicit queries (point indices or coordinates)")
        if offsets is None:
            offsets, _ = self.radius_count(r, queries, stream, kernel)
        bounds, ebounds = self.fill_chunks(offsets, max_entries, stream)
        buf = torch.empty(max(1, min(int(max_entries), ebounds[-1])), dtype=torch.int32,
                          device=self.device)
        for i in range(len(bounds) - 1):
            a, b = bounds[i], bounds[i + 1]
            tot = ebounds[i + 1] - ebounds[i]
            nbr = self.radius_fill(r, offsets[a:b + 1], tot, queries[a:b], out=buf,
                                   stream=stream, kernel=kernel)
            yield a, b, nbr[:tot]
        return offsets

    def radius(self, r, queries=None, stream=None, kernel="sphere"):
        """CSR neighbour lists: (offsets int64 [nq+1], nbr int32 [total]) of
        original point indices inside the kernel around each query (the
        sphere: D <= fl32(r*r))."""
        off, tot = self.radius_count(r, queries, stream, kernel)
        nbr = self.radius_fill(r, off, tot, queries, stream=stream, kernel=kernel)
        return off, nbr

    # ---- per-tile query sets on a batched index
    def _qoff(self, q_off, nq):
        qo = [int(v) for v in q_off]
        if len(qo) != self.ntiles + 1:
            raise ValueError(f"q_off needs {self.ntiles + 1} entries")
        return (ctypes.c_int64 * len(qo))(*qo)

    def radius_tiles(self, r, queries, q_off, stream=None, kernel="sphere"):
        """CSR lists of per-tile query sets: queries[q_off[t]:q_off[t+1]]
        (tile-local int32 point indices or float64 [.,3] coordinates) search
        tile t; neighbour indices are tile-local."""
        q, nq, keep = _queries(queries, self.n)
        qo = self._qoff(q_off, nq)
        off = torch.empty(nq + 1, dtype=torch.int64, device=self.device)
        tot = ctypes.c_int64(0)
        with _on(self.device, stream):
            check(lib().chs_kernel_count_tiles(self._h, ctypes.byref(q), qo, self.KERNELS[kernel],
                                               ctypes.c_float(r), off.data_ptr(), ctypes.byref(tot),
                                               _stream(stream)), "chs_kernel_count_tiles")
            nbr = torch.empty(tot.value, dtype=torch.int32, device=self.device)
            check(lib().chs_kernel_fill_tiles(self._h, ctypes.byref(q), qo, self.KERNELS[kernel],
                                              ctypes.c_float(r), off.data_ptr(),
                                              nbr.data_ptr() if tot.value else None, tot.value,
                                              _stream(stream)), "chs_kernel_fill_tiles")
        return off, nbr

    def knn_tiles(self, k, queries, q_off, r_max=math.inf, stream=None):
        """k-NN of per-tile query sets (as radius_tiles)."""
        q, nq, keep = _queries(queries, self.n)
        qo = self._qoff(q_off, nq)
        idx = torch.empty((nq, k), dtype=torch.int32, device=self.device)
        d2 = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        with _on(self.device, stream):
            check(lib().chs_knn_tiles(self._h, ctypes.byref(q), qo, k, ctypes.c_float(r_max),
                                      idx.data_ptr() if nq else None,
                                      d2.data_ptr() if nq else None, _stream(stream)),
                  "chs_knn_tiles")
        return idx, d2

    # ---- k-NN (Section 3.4.2)
    def knn_into(self, k, idx, d2, queries=None, r_max=math.inf, stream=None):
        """k-NN into preallocated idx [nq,k] int32 and d2 [nq,k] float32
        (no allocation: usable inside a captured graph)."""
        q, nq, keep = _queries(queries, self.n)
        if idx.shape != (nq, k) or d2.shape != (nq, k) or idx.dtype != torch.int32 \
                or d2.dtype != torch.float32 or not (idx.is_contiguous() and d2.is_contiguous()):
            raise ValueError("idx / d2 must be contiguous [nq,k] int32 / float32")
        with _on(self.device, stream):
            check(lib().chs_knn(self._h, ctypes.byref(q), k, ctypes.c_float(r_max),
                                idx.data_ptr() if nq else None, d2.data_ptr() if nq else None,
                                _stream(stream)), "chs_knn")
        return idx, d2

    def knn_visited(self, k, queries=None, r_max=math.inf, stream=None):
        """(idx, d2, visited): knn's lists plus, per query, int64 [nq, 2]:
        [:, 0] the voxels of the query's own taboo box (Alg. 2 run for it
        alone; rings: as [:, 1]), [:, 1] the voxels of its wave's visited box
        when its list became final; -1 for invalid queries."""
        q, nq, keep = _queries(queries, self.n)
        idx = torch.empty((nq, k), dtype=torch.int32, device=self.device)
        d2 = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        vis = torch.full((nq, 2), -1, dtype=torch.int64, device=self.device)
        with _on(self.device, stream):
            check(lib().chs_knn_visited(self._h, ctypes.byref(q), k, ctypes.c_float(r_max),
                                        idx.data_ptr() if nq else None,
                                        d2.data_ptr() if nq else None,
                                        vis.data_ptr() if nq else None, _stream(stream)),
                  "chs_knn_visited")
        return idx, d2, vis

    def knn_noalloc(self, k, idx, d2, queries=None, r_max=math.inf, stream=None):
        """k-NN into preallocated idx / d2 through chs_knn_noalloc: the library
        allocates nothing (its temporaries live in a fixed device array shared
        by every such call on the GPU; calls must not overlap)."""
        q, nq, keep = _queries(queries, self.n)
        if idx.shape != (nq, k) or d2.shape != (nq, k) or idx.dtype != torch.int32 \
                or d2.dtype != torch.float32 or not (idx.is_contiguous() and d2.is_contiguous()):
            raise ValueError("idx / d2 must be contiguous [nq,k] int32 / float32")
        with _on(self.device, stream):
            check(lib().chs_knn_noalloc(self._h, ctypes.byref(q), k, ctypes.c_float(r_max),
                                        idx.data_ptr() if nq else None,
                                        d2.data_ptr() if nq else None, _stream(stream)),
                  "chs_knn_noalloc")
        return idx, d2

    def knn(self, k, queries=None, r_max=math.inf, stream=None):
        """(idx int32 [nq,k], d2 float32 [nq,k]) sorted by (d2, index);
        missing entries are (-1, +inf)."""
        q, nq, keep = _queries(queries, self.n)
        idx = torch.empty((nq, k), dtype=torch.int32, device=self.device)
        d2 = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        with _on(self.device, stream):
            check(lib().chs_knn(self._h, ctypes.byref(q), k, ctypes.c_float(r_max),
                                idx.data_ptr() if nq else None, d2.data_ptr() if nq else None,
                                _stream(stream)), "chs_knn")
        return idx, d2
