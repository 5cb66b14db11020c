"""CPU oracle for the Cheesemap grid index -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the GPU library
computes, written from the paper (Section 3: Eq. 1-7, Alg. 1, Alg. 2 and the
remarks of Section 3.5) in ``chs_oracle.cpp`` and driven from here through
ctypes.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may use it; the GPU library neither imports nor links it, and the
two share no code.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chs_oracle.cpp")
_SO = os.path.join(_HERE, "liboracle.so")
CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-pthread", "-Wall"]

FLAVORS = {"dense": 0, "sparse": 1, "mixed": 2}


def compile_oracle():
    """Compile the oracle with the host compiler (no FMA contraction)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["g++", *CXXFLAGS, "-o", tmp, _SRC])
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            compile_oracle()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, i32, f32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_double
        L.orc_build.restype = P
        L.orc_build.argtypes = [P, i64, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, i64, P]
        L.orc_free.argtypes = [P]
        L.orc_geometry.argtypes = [P, P, P, P]
        L.orc_n_nonempty.restype = i64
        L.orc_n_nonempty.argtypes = [P]
        L.orc_point_arrays.argtypes = [P, P, P, P, P]
        L.orc_cells.argtypes = [P, P, P]
        L.orc_dense_start.restype = i64
        L.orc_dense_start.argtypes = [P, P]
        L.orc_slices.restype = i64
        L.orc_slices.argtypes = [P, P, P]
        L.orc_radius.restype = P
        L.orc_radius.argtypes = [P, P, P, i64, f32, ctypes.c_int, P, P]
        L.orc_kernel_search.restype = P
        L.orc_kernel_search.argtypes = [P, P, P, i64, ctypes.c_int, f32, ctypes.c_int, P, P]
        L.orc_radius_copy.argtypes = [P, P]
        L.orc_radius_free.argtypes = [P]
        L.orc_knn.restype = ctypes.c_int
        L.orc_knn.argtypes = [P, P, P, i64, ctypes.c_int, f32, ctypes.c_int, P, P, P, ctypes.c_int]
        L.orc_agg_fwd.argtypes = [P, P, P, i64, i64, i32, P, i32, f64, P]
        L.orc_agg_bwd.argtypes = [P, P, P, i64, i64, i32, P, i32, f64, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


class OracleIndex:
    """The grid index built on the CPU from FP64 coordinates ``xyz`` [n,3]."""

    def __init__(self, xyz, cell=1.0, dims=3, flavor="dense", mixed_pct=80,
                 max_dense_cells=1 << 31):
        L = lib()
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.n = self.xyz.shape[0]
        c = np.broadcast_to(np.asarray(cell, dtype=np.float64), (3,)).copy()
        self.cell = c
        self.dims = dims
        self.flavor = flavor
        st = ctypes.c_int(0)
        self._h = L.orc_build(_p(self.xyz), self.n, dims, FLAVORS[flavor], _p(c), mixed_pct,
                              int(max_dense_cells), ctypes.byref(st))
        if not self._h:
            raise OracleError(f"orc_build failed with status {st.value}")
        o = np.zeros(3); m = np.zeros(3, np.float32); nc = np.zeros(3, np.int64)
        L.orc_geometry(self._h, _p(o), _p(m), _p(nc))
        self.origin, self.max32, self.ncell = o, m, nc
        self.n_nonempty = L.orc_n_nonempty(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    def point_arrays(self):
        n = self.n
        x32 = np.zeros((3, n), np.float32); keys = np.zeros(n, np.uint64)
        perm = np.zeros(n, np.int32); srt = np.zeros((3, n), np.float32)
        lib().orc_point_arrays(self._h, _p(x32), _p(keys), _p(perm), _p(srt))
        return dict(x32=x32, keys=keys, perm=perm, sorted=srt)

    def cells(self):
        m = self.n_nonempty
        uk = np.zeros(m, np.uint64); us = np.zeros(m + 1, np.int64)
        lib().orc_cells(self._h, _p(uk), _p(us))
        return uk, us

    def dense_start(self):
        L = lib()
        ln = L.orc_dense_start(self._h, None)
        if ln < 0:
            return None
        out = np.zeros(ln, np.int64)
        L.orc_dense_start(self._h, _p(out))
        return out

    def slices(self):
        L = lib()
        nz = L.orc_slices(self._h, None, None)
        if nz < 0:
            return None
        ne = np.zeros(nz, np.int64); de = np.zeros(nz, np.uint8)
        L.orc_slices(self._h, _p(ne), _p(de))
        return ne, de.astype(bool)

    @staticmethod
    def _queries(pidx, qxyz):
        if pidx is not None:
            pidx = np.ascontiguousarray(pidx, dtype=np.int32)
            return pidx, None, pidx.shape[0]
        if qxyz is not None:
            qxyz = np.ascontiguousarray(qxyz, dtype=np.float64)
            return None, qxyz, qxyz.shape[0]
        return None, None, None

    KERNELS = {"sphere": 0, "cube": 1, "cylinder": 2}

    def radius(self, r, pidx=None, qxyz=None, nthreads=1, visited=False, kernel="sphere"):
        """Alg. 1 per query with a closed sphere of radius ``r`` (FP32), or a
        cube of half side r, or a vertical cylinder of radius r (z ignored);
        returns CSR (offsets [nq+1], original point indices)."""
        pidx, qxyz, nq = self._queries(pidx, qxyz)
        if nq is None:
            nq = self.n
        L = lib()
        off = np.zeros(nq + 1, np.int64)
        vis = np.zeros(nq, np.int64) if visited else None
        res = L.orc_kernel_search(self._h, _p(pidx), _p(qxyz), nq, self.KERNELS[kernel],
                                  ctypes.c_float(r), nthreads, _p(off), _p(vis))
        nbr = np.zeros(int(off[-1]), np.int32)
        L.orc_radius_copy(res, _p(nbr))
        L.orc_radius_free(res)
        if visited:
            return off, nbr, vis
        return off, nbr

    def knn(self, k, r_max=math.inf, pidx=None, qxyz=None, nthreads=1, visited=False,
            schedule="density"):
        """Alg. 2 per query; returns idx [nq,k] int32 (-1 padded) and squared
        distances d2 [nq,k] FP32 (+inf padded), sorted by (d2, index).
        schedule: "density" (Alg. 2's growth, Eq. 12) or "monotonic" (the
        radius grows by the smallest voxel edge per step); with visited=True
        also the non-empty voxels each query's search visited."""
        pidx, qxyz, nq = self._queries(pidx, qxyz)
        if nq is None:
            nq = self.n
        idx = np.zeros((nq, k), np.int32)
        d2 = np.zeros((nq, k), np.float32)
        vis = np.zeros(nq, np.int64) if visited else None
        rc = lib().orc_knn(self._h, _p(pidx), _p(qxyz), nq, k, ctypes.c_float(r_max), nthreads,
                           _p(idx), _p(d2), _p(vis), {"density": 0, "monotonic": 1}[schedule])
        if rc != 0:
            raise OracleError("orc_knn: invalid argument")
        if visited:
            return idx, d2, vis
        return idx, d2


def agg_forward(x, qidx, nbr, f, sigma):
    """FP64 Gaussian-weighted aggregation over fixed neighbour lists."""
    x = np.ascontiguousarray(x, np.float64); f = np.ascontiguousarray(f, np.float64)
    qidx = np.ascontiguousarray(qidx, np.int32); nbr = np.ascontiguousarray(nbr, np.int32)
    Q, K = nbr.shape
    C = f.shape[1]
    out = np.zeros((Q, C), np.float64)
    lib().orc_agg_fwd(_p(x), _p(qidx), _p(nbr), x.shape[0], Q, K, _p(f), C, float(sigma), _p(out))
    return out


def agg_backward(x, qidx, nbr, f, sigma, gout):
    """FP64 analytic gradients (grad_x [N,3], grad_f [N,C]) of sum(gout * out)."""
    x = np.ascontiguousarray(x, np.float64); f = np.ascontiguousarray(f, np.float64)
    qidx = np.ascontiguousarray(qidx, np.int32); nbr = np.ascontiguousarray(nbr, np.int32)
    gout = np.ascontiguousarray(gout, np.float64)
    Q, K = nbr.shape
    C = f.shape[1]
    gx = np.zeros_like(x); gf = np.zeros_like(f)
    lib().orc_agg_bwd(_p(x), _p(qidx), _p(nbr), x.shape[0], Q, K, _p(f), C, float(sigma),
                      _p(gout), _p(gx), _p(gf))
    return gx, gf


def recentre32(xyz):
    """FP64 recentring to the per-axis minimum, then FP32 (Eq. 1)."""
    xyz = np.asarray(xyz, np.float64)
    return (xyz - xyz.min(axis=0)).astype(np.float32)
