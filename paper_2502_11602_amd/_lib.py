"""ctypes declarations of the C ABI in include/chs.h (argument marshalling
only: every step of the computation runs in libchs.so)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchs.so")

c_void_p, c_int32, c_int64, c_float, c_double = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                                 ctypes.c_float, ctypes.c_double)

STATUS = {0: "CHS_OK", 1: "CHS_E_INVALID", 2: "CHS_E_NOMEM", 3: "CHS_E_CAPACITY",
          4: "CHS_E_DEVICE", 5: "CHS_E_UNSUPPORTED"}
FLAVORS = {"dense": 0, "sparse": 1, "mixed": 2}

ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", c_void_p)]


class BuildParams(ctypes.Structure):
    _fields_ = [("flavor", c_int32), ("dims", c_int32), ("cell", c_double * 3),
                ("mixed_dense_pct", c_int32), ("reserved", c_int32), ("max_dense_cells", c_int64)]


class Queries(ctypes.Structure):
    _fields_ = [("xyz", c_void_p), ("point_idx", c_void_p), ("nq", c_int64)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("origin", c_double * 3), ("max32", c_float * 3), ("cell", c_double * 3),
                ("ncell", c_int64 * 3), ("n_points", c_int64), ("n_nonempty", c_int64),
                ("n_dense_slices", c_int64), ("device_bytes", c_int64), ("flavor", c_int32),
                ("dims", c_int32), ("ntiles", c_int32), ("reserved", c_int32)]


class IndexArrays(ctypes.Structure):
    _fields_ = [("perm", c_void_p), ("inv_perm", c_void_p), ("sorted_xyz", c_void_p),
                ("points", c_void_p), ("cell_keys", c_void_p), ("cell_start", c_void_p),
                ("dense_start", c_void_p), ("slice_dense", c_void_p)]


# name -> (restype, argtypes); the set the header declares
SIGNATURES = {
    "chs_build": (c_int32, [c_void_p, c_int64, ctypes.POINTER(BuildParams),
                            ctypes.POINTER(Allocator), c_void_p, ctypes.POINTER(c_void_p)]),
    "chs_index_info": (c_int32, [c_void_p, ctypes.POINTER(IndexInfo)]),
    "chs_build_batch": (c_int32, [c_void_p, c_int64, c_void_p, c_int32, c_void_p,
                                  ctypes.POINTER(Allocator), c_void_p, ctypes.POINTER(c_void_p)]),
    "chs_build_batch_framed": (c_int32, [c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_void_p,
                                         ctypes.POINTER(Allocator), c_void_p,
                                         ctypes.POINTER(c_void_p)]),
    "chs_tile_info": (c_int32, [c_void_p, c_int32, ctypes.POINTER(IndexInfo)]),
    "chs_index_set_option": (c_int32, [c_void_p, c_int32, c_int64]),
    "chs_index_arrays": (c_int32, [c_void_p, ctypes.POINTER(IndexArrays)]),
    "chs_index_coords": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "chs_radius_count": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_float, c_void_p,
                                   ctypes.POINTER(c_int64), c_void_p]),
    "chs_radius_fill": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_float, c_void_p, c_void_p,
                                  c_int64, c_void_p]),
    "chs_radius_search": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_float,
                                    ctypes.POINTER(Allocator), c_void_p, ctypes.POINTER(c_void_p),
                                    ctypes.POINTER(c_int64), c_void_p]),
    "chs_kernel_count": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_int32, c_float, c_void_p,
                                   ctypes.POINTER(c_int64), c_void_p]),
    "chs_kernel_fill": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_int32, c_float, c_void_p,
                                  c_void_p, c_int64, c_void_p]),
    "chs_kernel_search": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_int32, c_float,
                                    ctypes.POINTER(Allocator), c_void_p, ctypes.POINTER(c_void_p),
                                    ctypes.POINTER(c_int64), c_void_p]),
    "chs_kernel_count_tiles": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_void_p, c_int32,
                                         c_float, c_void_p, ctypes.POINTER(c_int64), c_void_p]),
    "chs_kernel_fill_tiles": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_void_p, c_int32,
                                        c_float, c_void_p, c_void_p, c_int64, c_void_p]),
    "chs_query_order": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_void_p, c_void_p]),
    "chs_fill_chunks": (c_int32, [c_void_p, c_int64, c_int64, c_void_p, c_void_p, c_int64,
                                  ctypes.POINTER(c_int64), c_void_p]),
    "chs_knn_tiles": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_void_p, c_int32, c_float,
                                c_void_p, c_void_p, c_void_p]),
    "chs_knn": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_int32, c_float, c_void_p, c_void_p,
                          c_void_p]),
    "chs_knn_visited": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_int32, c_float, c_void_p,
                                  c_void_p, c_void_p, c_void_p]),
    "chs_knn_noalloc": (c_int32, [c_void_p, ctypes.POINTER(Queries), c_int32, c_float, c_void_p,
                                  c_void_p, c_void_p]),
    "chs_gauss_agg_fwd": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int64, c_int32,
                                    c_void_p, c_int32, c_double, c_int32, c_int32, c_void_p,
                                    c_void_p]),
    "chs_gauss_agg_bwd": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int64, c_int32,
                                    c_void_p, c_int32, c_double, c_int32, c_int32, c_void_p,
                                    c_void_p, c_void_p, ctypes.POINTER(Allocator), c_void_p]),
    "chs_free": (None, [c_void_p]),
    "chs_last_error": (ctypes.c_char_p, []),
    "chs_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libchs.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class ChsError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib().chs_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


def check(status, where):
    if status != 0:
        raise ChsError(status, where)
