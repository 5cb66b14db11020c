"""Writes config2_digests.txt: the oracle's per-block digests of every
query's result on the 20 M-point TLS scan (cloudgen.config2(): 2 M query
points in the generator's order, 0.25 m voxels, 3D).

The neighbour sets follow Alg. 1 (Section 3.4.1) with the sphere at 0.1,
0.25 and 0.5 m; the k-NN lists (k = 32) follow Alg. 2 (Section 3.4.2).  At
0.5 m the relation holds about 1.5e11 pairs, so the oracle's CSR is built
for a few thousand queries at a time and reduced to per-query digests
(tests/_digest.py) before the next.  Only the oracle computes them: this
script imports oracle/ and the seeded generator, nothing of the GPU library.
Sets already in the file (same cloud) are kept, so an interrupted run
resumes.  Run from the repository root:

    python tests/golden/make_config2_digests.py [nthreads]

(about an hour on 8 threads, most of it the 0.5 m set)."""
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path[:0] = [ROOT, os.path.join(ROOT, "tests")]

import cloudgen  # noqa: E402
import oracle  # noqa: E402
import _digest as D  # noqa: E402

CELL = 0.25
SETS_RADIUS = [(0.1, 16384), (0.25, 4096), (0.5, 1024)]  # (r, queries per oracle call)
SETS_KNN = [32]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_digests.txt")
HEAD = ["# Oracle digests of every query's result on the 20 M-point TLS scan",
        "# (cloudgen.config2(): 2 M query points in the generator's order, 0.25 m",
        "# voxels, 3D).  Radius sets: Alg. 1 (Section 3.4.1) with the sphere;",
        "# k-NN: Alg. 2 (Section 3.4.2), rows sorted by (D, index).",
        "# Written by tests/golden/make_config2_digests.py (oracle only); digests",
        "# as defined in tests/_digest.py.  Line format:",
        "#   input <sha256 prefix of the FP64 cloud> <n> <sha256 prefix of the queries>",
        "#   <set> <block> <sum of counts> <digest, hex>"]


def row_hash_parallel(pool, parts, off, nbr):
    """D.row_hash_csr_np over row ranges in parallel threads (numpy releases
    the interpreter lock inside its array loops); the same values."""
    nq = len(off) - 1
    bounds = np.linspace(0, nq, parts + 1).astype(np.int64)

    def work(i):
        a, b = int(bounds[i]), int(bounds[i + 1])
        return D.row_hash_csr_np(off[a:b + 1] - off[a], nbr[off[a]:off[b]])

    res = list(pool.map(work, range(parts)))
    return np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res])


def main():
    nth = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    c = cloudgen.config2()
    xyz, queries = c["xyz"], c["queries"]
    n, nq = len(xyz), len(queries)
    qfp = D.fingerprint(queries.astype(np.float64))
    meta_line = f"input {D.fingerprint(xyz)} {n} {qfp}"
    done = {}
    if os.path.exists(OUT):
        meta, sets = D.read_golden(OUT)
        if " ".join(["input"] + meta.get("input", [])) == meta_line:
            nb = (nq + D.BLOCK - 1) // D.BLOCK
            done = {k: v for k, v in sets.items() if len(v) == nb}
    ox = oracle.OracleIndex(xyz, CELL, flavor="sparse")
    pool = ThreadPoolExecutor(nth)

    def write():
        lines = HEAD + [meta_line, f"block {D.BLOCK}"]
        for name in sorted(done, key=lambda s: (s.startswith("knn"), float(s.split("_")[1]))):
            lines += [f"{name} {b} {cs} {dg:016x}" for b, cs, dg in done[name]]
        with open(OUT + ".tmp", "w") as fh:
            fh.write("\n".join(lines) + "\n")
        os.replace(OUT + ".tmp", OUT)

    for r, step in SETS_RADIUS:
        name = f"sphere_{r:g}"
        if name in done:
            continue
        t = time.time()
        rows = []
        for q0 in range(0, nq, D.BLOCK):
            cnt_b, h_b = [], []
            for a in range(q0, min(nq, q0 + D.BLOCK), step):
                b = min(nq, q0 + D.BLOCK, a + step)
                off, nbr = ox.radius(r, pidx=queries[a:b], nthreads=nth)
                cnt, h = row_hash_parallel(pool, nth, off, nbr)
                cnt_b.append(cnt)
                h_b.append(h)
                del off, nbr
            rows += D.block_digests_np(np.concatenate(cnt_b), np.concatenate(h_b), q0=q0)
            print(f"{name}: block {q0 // D.BLOCK} done, {time.time() - t:.0f} s", flush=True)
        done[name] = rows
        write()
    for k in SETS_KNN:
        name = f"knn_{k}"
        if name in done:
            continue
        rows = []
        for q0 in range(0, nq, D.BLOCK):
            idx, d2 = ox.knn(k, pidx=queries[q0:q0 + D.BLOCK], nthreads=nth)
            cnt, h = D.row_hash_knn_np(idx, d2)
            rows += D.block_digests_np(cnt, h, q0=q0)
        done[name] = rows
        write()
    print(OUT)


if __name__ == "__main__":
    main()
