"""Writes knn_growth_stats.txt: the oracle's voxels visited per k-NN query
under density growth (Alg. 2, Eq. 12) and under monotonic growth (radius +
smallest voxel edge per step), on the 1 M uniform random points of
cloudgen.uniform_cube (Section 3.5, "Density-based growth in k-NN"), every
point a query, dense map, for several voxel edges and k.

Per row: voxel edge s, k, the number of queries where density growth visits
fewer, more and as many voxels as monotonic growth, and the sums of the
visited voxels of each schedule.  Only the oracle computes them: this script
imports oracle/ and the seeded generator, nothing of the GPU library.  Run
from the repository root:

    python tests/golden/make_knn_growth_stats.py [nthreads]

(about a minute on 8 threads)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path[:0] = [ROOT]

import cloudgen  # noqa: E402
import oracle  # noqa: E402

CELLS = [0.5, 1.0, 2.0, 4.0]
KS = [4, 8, 16, 32]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "knn_growth_stats.txt")


def rows(nth, cells=CELLS, ks=KS):
    xyz = cloudgen.uniform_cube()
    for s in cells:
        ox = oracle.OracleIndex(xyz, s, flavor="dense")
        for k in ks:
            _, _, vd = ox.knn(k, nthreads=nth, visited=True, schedule="density")
            _, _, vm = ox.knn(k, nthreads=nth, visited=True, schedule="monotonic")
            yield (s, k, int((vd < vm).sum()), int((vd > vm).sum()), int((vd == vm).sum()),
                   int(vd.sum()), int(vm.sum()))


def main():
    nth = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    with open(OUT, "w") as f:
        f.write("# Section 3.5 density vs monotonic growth, 1e6 uniform points "
                "(cloudgen.uniform_cube, seed 7, side 100 m), dense map, every point a query\n")
        f.write("# written by tests/golden/make_knn_growth_stats.py (oracle only)\n")
        f.write("# cell k n_fewer n_more n_equal sum_visited_density sum_visited_monotonic\n")
        for r in rows(nth):
            f.write(" ".join(str(v) for v in r) + "\n")
            f.flush()
            print(r, flush=True)


if __name__ == "__main__":
    main()
