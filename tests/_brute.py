"""Brute-force neighbour search in numpy (the naive method of Section 2: every
point is checked against every query).  Used only to pin the grid oracle; it
shares no code with the oracle and has no grid at all.

The squared distance follows the fixed arithmetic of the method: FP32
operands, dx = fl32(qx - px), and D = fl32(fl32(fl32(dx^2) + fl32(dy^2)) +
fl32(dz^2)); numpy float32 ufuncs round every operation to binary32 and never
fuse.
"""
import numpy as np


def sq_dist_rows(q, pts):
    """D between each query row q [m,3] float32 and all points pts [n,3]."""
    q = np.asarray(q, np.float32)
    pts = np.asarray(pts, np.float32)
    dx = np.subtract(q[:, None, 0], pts[None, :, 0], dtype=np.float32)
    dy = np.subtract(q[:, None, 1], pts[None, :, 1], dtype=np.float32)
    dz = np.subtract(q[:, None, 2], pts[None, :, 2], dtype=np.float32)
    s = np.add(np.multiply(dx, dx, dtype=np.float32), np.multiply(dy, dy, dtype=np.float32),
               dtype=np.float32)
    return np.add(s, np.multiply(dz, dz, dtype=np.float32), dtype=np.float32)


def brute_radius(pts32, q32, r, block=256):
    """List of ascending index arrays: points with D <= fl32(r*r)."""
    R = np.float32(r) * np.float32(r)
    out = []
    for a in range(0, q32.shape[0], block):
        D = sq_dist_rows(q32[a:a + block], pts32)
        for row in D:
            out.append(np.nonzero(row <= R)[0].astype(np.int32))
    return out


def brute_knn(pts32, q32, k, r_max=np.inf, block=256):
    """First k points by (D, index); (-1, inf) padding; r_max filter."""
    n = pts32.shape[0]
    Rm = np.float32(np.inf) if np.isinf(r_max) else np.float32(r_max) * np.float32(r_max)
    idx = np.full((q32.shape[0], k), -1, np.int32)
    d2 = np.full((q32.shape[0], k), np.inf, np.float32)
    ar = np.arange(n)
    for a in range(0, q32.shape[0], block):
        D = sq_dist_rows(q32[a:a + block], pts32)
        for t, row in enumerate(D):
            order = np.lexsort((ar, row))[:k]
            keep = row[order] <= Rm
            m = int(keep.sum())
            idx[a + t, :m] = order[:m]
            d2[a + t, :m] = row[order[:m]]
    return idx, d2


def csr_rows(off, nbr):
    return [np.sort(nbr[off[i]:off[i + 1]]) for i in range(len(off) - 1)]


def brute_kernel(pts32, q32, r, kernel, block=256):
    """Like brute_radius for the other kernels of Alg. 1: a cube of half side
    r (|dx|, |dy|, |dz| <= r) or a vertical cylinder of radius r
    (fl32(dx^2 + dy^2) <= fl32(r*r), z ignored); dx = fl32(qx - px)."""
    if kernel == "sphere":
        return brute_radius(pts32, q32, r, block)
    r32 = np.float32(r)
    R = r32 * r32
    pts = np.asarray(pts32, np.float32)
    out = []
    for a in range(0, q32.shape[0], block):
        q = np.asarray(q32[a:a + block], np.float32)
        dx = np.subtract(q[:, None, 0], pts[None, :, 0], dtype=np.float32)
        dy = np.subtract(q[:, None, 1], pts[None, :, 1], dtype=np.float32)
        if kernel == "cube":
            dz = np.subtract(q[:, None, 2], pts[None, :, 2], dtype=np.float32)
            m = (np.abs(dx) <= r32) & (np.abs(dy) <= r32) & (np.abs(dz) <= r32)
        elif kernel == "cylinder":
            h = np.add(np.multiply(dx, dx, dtype=np.float32), np.multiply(dy, dy, dtype=np.float32),
                       dtype=np.float32)
            m = h <= R
        else:
            raise ValueError(kernel)
        for row in m:
            out.append(np.nonzero(row)[0].astype(np.int32))
    return out
