"""Order-independent digests of neighbour relations and k-NN lists, for
parity at sizes where the oracle's results cannot be stored whole.

Per query q of a CSR relation: c_q = the row's length and h_q = the sum
(mod 2^64) of fmix64(j + 1) over its neighbours j, which does not depend on
the order inside the row (rows are sets).  Per query of a k-NN result: h_q =
the sum of fmix64(w_i + (i + 1) * G) over the row's slots i, with w_i =
(bits of d2 << 32) | index as uint32, which does depend on the order (k-NN
rows are sorted lists).  A block of consecutive queries is summarised by the
sum of its counts and the sum of fmix64(h_q + fmix64(q << 32 | c_q)).

fmix64 is the 64-bit finaliser of MurmurHash3.  The numpy functions serve
the script that writes the oracle's digests; the torch functions compute
the same values for the GPU's results on the GPU (int64 arithmetic, which
wraps like uint64).  This file is test infrastructure only."""
import hashlib

import numpy as np

_F1 = 0xFF51AFD7ED558CCD
_F2 = 0xC4CEB9FE1A85EC53
_G = 0x9E3779B97F4A7C15
BLOCK = 1 << 18


def fingerprint(xyz):
    """First 32 hex digits of the SHA-256 of an FP64 cloud's bytes."""
    return hashlib.sha256(np.ascontiguousarray(xyz, np.float64).tobytes()).hexdigest()[:32]


def read_golden(path):
    """(meta, sets) of a digest file: meta[key] = values of the 'input' and
    'block' lines; sets[name] = [(block, count sum, digest)]."""
    meta, sets = {}, {}
    with open(path) as fh:
        for line in fh:
            f = line.split("#", 1)[0].split()
            if not f:
                continue
            if f[0] in ("input", "block"):
                meta[f[0]] = f[1:]
            else:
                sets.setdefault(f[0], []).append((int(f[1]), int(f[2]), int(f[3], 16)))
    return meta, sets


# ---------------------------------------------------------------- numpy (uint64)
def fmix64_np(x):
    x = np.asarray(x, np.uint64).copy()
    x ^= x >> np.uint64(33)
    x *= np.uint64(_F1)
    x ^= x >> np.uint64(33)
    x *= np.uint64(_F2)
    x ^= x >> np.uint64(33)
    return x


def row_hash_csr_np(off, nbr):
    """(counts [nq] int64, h [nq] uint64) of a CSR relation."""
    off = np.asarray(off, np.int64)
    m = fmix64_np(np.asarray(nbr, np.int64).astype(np.uint64) + np.uint64(1))
    cs = np.zeros(len(m) + 1, np.uint64)
    np.cumsum(m, out=cs[1:])
    return np.diff(off), cs[off[1:]] - cs[off[:-1]]


def row_hash_knn_np(idx, d2):
    idx = np.asarray(idx, np.int32)
    d2 = np.ascontiguousarray(d2, np.float32)
    k = idx.shape[1]
    w = (d2.view(np.uint32).astype(np.uint64) << np.uint64(32)) | idx.view(np.uint32).astype(np.uint64)
    pos = (np.arange(1, k + 1, dtype=np.uint64) * np.uint64(_G))[None, :]
    h = fmix64_np(w + pos).sum(axis=1, dtype=np.uint64)
    return np.zeros(idx.shape[0], np.int64), h


def query_digest_np(q0, counts, h):
    """Per-query digests of queries q0, q0+1, ..."""
    q = np.arange(q0, q0 + len(h), dtype=np.uint64)
    tag = fmix64_np((q << np.uint64(32)) | np.asarray(counts, np.int64).astype(np.uint64))
    return fmix64_np(np.asarray(h, np.uint64) + tag)


# ---------------------------------------------------------------- torch (int64)
def _c(v):
    return v - (1 << 64) if v >= (1 << 63) else v


def fmix64_t(x):
    import torch
    x = x.to(torch.int64)
    mask = (1 << 31) - 1  # keeps the low 31 bits of an arithmetic >> 33
    x = x ^ ((x >> 33) & mask)
    x = x * _c(_F1)
    x = x ^ ((x >> 33) & mask)
    x = x * _c(_F2)
    x = x ^ ((x >> 33) & mask)
    return x


def row_hash_csr_t(off, nbr, chunk=1 << 28):
    """Same as row_hash_csr_np for device tensors, in chunks of entries."""
    import torch
    off = off.to(torch.int64)
    nq = off.numel() - 1
    at = torch.zeros(nq + 1, dtype=torch.int64, device=off.device)  # prefix sums at offsets
    carry = torch.zeros((), dtype=torch.int64, device=off.device)
    total = int(off[-1])
    for a in range(0, total, chunk):
        b = min(total, a + chunk)
        cs = torch.cumsum(fmix64_t(nbr[a:b].to(torch.int64) + 1), 0) + carry
        lo = int(torch.searchsorted(off, torch.tensor(a + 1, device=off.device)))
        hi = int(torch.searchsorted(off, torch.tensor(b, device=off.device), right=True))
        if hi > lo:
            at[lo:hi] = cs[off[lo:hi] - 1 - a]
        carry = cs[-1].clone()
        del cs
    return torch.diff(off), at[1:] - at[:-1]


def row_hash_knn_t(idx, d2):
    import torch
    k = idx.shape[1]
    w = (d2.contiguous().view(torch.int32).to(torch.int64) << 32) | \
        (idx.to(torch.int64) & 0xFFFFFFFF)
    pos = torch.arange(1, k + 1, dtype=torch.int64, device=idx.device) * _c(_G)
    h = fmix64_t(w + pos[None, :]).sum(dim=1)
    return torch.zeros(idx.shape[0], dtype=torch.int64, device=idx.device), h


def query_digest_t(q0, counts, h):
    import torch
    q = torch.arange(q0, q0 + h.numel(), dtype=torch.int64, device=h.device)
    return fmix64_t(h + fmix64_t((q << 32) | counts.to(torch.int64)))


# ---------------------------------------------------------------- blocks
def block_digests_np(counts, h, q0=0, block=BLOCK):
    """[(block index, count sum, digest as uint64)] for queries q0.. (q0 a
    multiple of block)."""
    d = query_digest_np(q0, counts, h)
    out = []
    for s in range(0, len(d), block):
        b = (q0 + s) // block
        out.append((b, int(np.asarray(counts[s:s + block], np.int64).sum()),
                    int(d[s:s + block].sum(dtype=np.uint64))))
    return out


def block_digests_t(counts, h, block=BLOCK):
    import torch
    d = query_digest_t(0, counts, h)
    nb = (d.numel() + block - 1) // block
    pad = nb * block - d.numel()
    if pad:
        d = torch.cat([d, torch.zeros(pad, dtype=torch.int64, device=d.device)])
        counts = torch.cat([counts, torch.zeros(pad, dtype=counts.dtype, device=d.device)])
    ds = d.view(nb, block).sum(dim=1).cpu().tolist()
    cs = counts.view(nb, block).to(torch.int64).sum(dim=1).cpu().tolist()
    return [(b, int(cs[b]), ds[b] & ((1 << 64) - 1)) for b in range(nb)]
