"""Differentiable Gaussian-weighted neighbourhood aggregation.

out[q, c] = sum_t exp(-|x_j - x_q|^2 / (2 sigma^2)) f[j_t, c] over fixed
neighbour lists (the k nearest points within a radius, from the grid index).
Forward and backward both run in libchs.so; this module is the
``torch.autograd.Function`` glue around chs_gauss_agg_fwd / _bwd."""
import ctypes
import math

import torch

from ._lib import check, lib
from .index import TorchAllocator, _stream

_DT = {torch.float32: 0, torch.float64: 1, torch.bfloat16: 2}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else None


class GaussAgg(torch.autograd.Function):
    """x [N,3] (float32 or float64), f [N,C] (same dtype, or bfloat16 with
    float32 x), qidx [Q] int32 centre points, nbr [Q,K] int32 (-1 padded)."""

    @staticmethod
    def forward(ctx, x, f, qidx, nbr, sigma):
        x = x.contiguous(); f = f.contiguous()
        qidx = qidx.contiguous(); nbr = nbr.contiguous()
        N, C = f.shape
        Q, K = nbr.shape
        out = torch.empty((Q, C), dtype=f.dtype, device=f.device)
        with torch.cuda.device(f.device):
            check(lib().chs_gauss_agg_fwd(_ptr(x), _ptr(qidx), _ptr(nbr), N, Q, K, _ptr(f), C,
                                          float(sigma), _DT[x.dtype], _DT[f.dtype], _ptr(out),
                                          _stream()), "chs_gauss_agg_fwd")
        ctx.save_for_backward(x, f, qidx, nbr)
        ctx.sigma = float(sigma)
        return out

    @staticmethod
    def backward(ctx, gout):
        x, f, qidx, nbr = ctx.saved_tensors
        gout = gout.contiguous().to(f.dtype)
        N, C = f.shape
        Q, K = nbr.shape
        gx = torch.empty_like(x)
        gf = torch.empty_like(f)
        al = TorchAllocator(f.device)
        with torch.cuda.device(f.device):
            check(lib().chs_gauss_agg_bwd(_ptr(x), _ptr(qidx), _ptr(nbr), N, Q, K, _ptr(f), C,
                                          ctx.sigma, _DT[x.dtype], _DT[f.dtype], _ptr(gout),
                                          _ptr(gx), _ptr(gf), ctypes.byref(al.struct),
                                          _stream()), "chs_gauss_agg_bwd")
        return gx, gf, None, None, None


def gauss_aggregate(x, f, qidx, nbr, sigma=0.25):
    return GaussAgg.apply(x, f, qidx, nbr, sigma)


def neighbour_lists(index, qidx, k=64, r_max=0.5):
    """The k nearest points within r_max of every centre (point indices into
    the indexed cloud), as [Q,k] int32 padded with -1; computed without
    gradient by the grid index."""
    with torch.no_grad():
        idx, _ = index.knn(k, qidx, r_max=r_max)
    return idx


def recentred(index):
    """FP32 coordinates in the index's frame, in input order: the library's
    own recentring (Section 3.1, Eq. 1), the same values its searches use."""
    return index.coords()
