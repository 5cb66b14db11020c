"""Writes config1_digests.txt: the oracle's per-block digests of every
query's result on the 10 M-point ALS tile (every point a query, 1 m voxels).

The neighbour sets follow Alg. 1 (Section 3.4.1) with the sphere, the cube
and the cylinder kernels; the k-NN lists follow Alg. 2 (Section 3.4.2).
Only the oracle computes them: this script imports oracle/ and the seeded
generator, nothing of the GPU library.  Digests are defined in
tests/_digest.py.  Run from the repository root:

    python tests/golden/make_config1_digests.py [nthreads]

(about 8 minutes on 8 threads)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path[:0] = [ROOT, os.path.join(ROOT, "tests")]

import cloudgen  # noqa: E402
import oracle  # noqa: E402
import _digest as D  # noqa: E402

# (set name, kernel, r) -- the sphere at 4 m has more than 256 neighbours per
# query on average; the cube and the cylinder at 2 and 3 m span 96 to 340
SETS_RADIUS = [("sphere", 0.5), ("sphere", 1.0), ("sphere", 2.0), ("sphere", 3.0),
               ("sphere", 4.0), ("cube", 2.0), ("cube", 3.0), ("cylinder", 2.0),
               ("cylinder", 3.0)]
SETS_KNN = [8, 16, 32]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config1_digests.txt")


def main():
    nth = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    c = cloudgen.config1()
    xyz = c["xyz"]
    n = len(xyz)
    ox = oracle.OracleIndex(xyz, 1.0)
    lines = ["# Oracle digests of every query's result on the 10 M-point ALS tile",
             "# (cloudgen.config1(), every point a query in index order, 1 m voxels, 3D).",
             "# Radius sets: Alg. 1 (Section 3.4.1) with the sphere, cube and cylinder",
             "# kernels; k-NN: Alg. 2 (Section 3.4.2), rows sorted by (D, index).",
             "# Written by tests/golden/make_config1_digests.py (oracle only); digests",
             "# as defined in tests/_digest.py.  Line format:",
             "#   input <sha256 prefix of the FP64 cloud> <n>",
             "#   <set> <block> <sum of counts> <digest, hex>",
             f"input {D.fingerprint(xyz)} {n}",
             f"block {D.BLOCK}"]
    for kern, r in SETS_RADIUS:
        t = time.time()
        name = f"{kern}_{r:g}"
        tot = 0
        for q0 in range(0, n, D.BLOCK):
            q = np.arange(q0, min(n, q0 + D.BLOCK), dtype=np.int32)
            off, nbr = ox.radius(r, pidx=q, nthreads=nth, kernel=kern)
            cnt, h = D.row_hash_csr_np(off, nbr)
            for b, cs, dg in D.block_digests_np(cnt, h, q0=q0):
                lines.append(f"{name} {b} {cs} {dg:016x}")
            tot += int(off[-1])
        print(f"{name}: {tot} neighbours, {time.time() - t:.1f} s", flush=True)
    for k in SETS_KNN:
        t = time.time()
        name = f"knn_{k}"
        for q0 in range(0, n, D.BLOCK):
            q = np.arange(q0, min(n, q0 + D.BLOCK), dtype=np.int32)
            idx, d2 = ox.knn(k, pidx=q, nthreads=nth)
            cnt, h = D.row_hash_knn_np(idx, d2)
            for b, cs, dg in D.block_digests_np(cnt, h, q0=q0):
                lines.append(f"{name} {b} {cs} {dg:016x}")
        print(f"{name}: {time.time() - t:.1f} s", flush=True)
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(OUT)


if __name__ == "__main__":
    main()
