// Declarations shared by the search translation units (search.hip: query
// planning and the entry points; radius.hip: the kernel-based search of
// Section 3.4.1; knn.hip: the k-NN search of Section 3.4.2): work items,
// the geometry of query tiles and voxel boxes, the inside tests and the
// kernels' argument blocks.
#pragma once

#include <cmath>

#include "common.h"

#pragma clang fp contract(off)

namespace chs {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;
constexpr uint32_t kInactive = 0x80000000u;
constexpr double kPadRel = 1.0 / 262144.0;              // 2^-18
constexpr double kPadAbs = 8.673617379884035e-19;       // 2^-60

// ---------------------------------------------------------------- work items
// A work item is one wave of at most 64 queries of one tile.
struct Waves {
  const float4* __restrict__ q4;  // processing order
  int64_t nq;
  int64_t nwaves;
  const int32_t* __restrict__ wave_tile;   // NULL: one tile, waves of 64
  const int32_t* __restrict__ wave_start;
  const int32_t* __restrict__ tile_qend;
  const Grid* __restrict__ tiles;
  int32_t* counter;  // persistent launches: next work item
};

struct Item {
  int tile;
  int64_t t0, tend;
};

__device__ __forceinline__ Item item_of(const Waves& W, int64_t w) {
  Item it;
  if (W.wave_tile) {
    // wave-uniform values: keep them in scalar registers
    it.tile = uniform(W.wave_tile[w]);
    it.t0 = uniform(W.wave_start[w]);
    const int64_t e = uniform(W.tile_qend[it.tile]);
    it.tend = it.t0 + kWave < e ? it.t0 + kWave : e;
  } else {
    it.tile = 0;
    it.t0 = w * kWave;
    it.tend = it.t0 + kWave < W.nq ? it.t0 + kWave : W.nq;
  }
  return it;
}

// Next work item of this wave: persistent waves take one from the counter
// (a single lane performs the atomic), others own exactly one.
__device__ __forceinline__ int64_t next_item(const Waves& W, int64_t* own, int lane) {
  if (W.counter) {
    int v = 0;
    if (lane == 0) v = atomicAdd(W.counter, 1);
    return (int64_t)uniform(__shfl(v, 0, kWave));
  }
  const int64_t w = *own;
  *own = W.nwaves;  // the next request finds nothing left
  return w;
}

// Inclusive prefix sum over the wave.
__device__ __forceinline__ int32_t wave_incl_scan(int32_t v, int lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// ---------------------------------------------------------------- tile geometry
struct Tile {
  bool any;             // at least one active lane
  float lo[3], hi[3];   // bounding box of the active queries
};

__device__ __forceinline__ Tile tile_bounds(float4 q, bool active) {
  Tile t;
  const float inf = INFINITY;
  t.lo[0] = wave_min(active ? q.x : inf);
  t.lo[1] = wave_min(active ? q.y : inf);
  t.lo[2] = wave_min(active ? q.z : inf);
  t.hi[0] = wave_max(active ? q.x : -inf);
  t.hi[1] = wave_max(active ? q.y : -inf);
  t.hi[2] = wave_max(active ? q.z : -inf);
  t.any = __ballot(active) != 0ull;
  return t;
}

// ---------------------------------------------------------------- lane clusters
// A wave's queries come in processing order, which can leave a sparse
// query set's region and re-enter it far away: one box over both stretches
// would cover the gap (and, for k-NN, every ring would grow it).  The lanes
// still to be searched (todo) are therefore cut into clusters of
// consecutive lanes: a cluster takes lanes until the next query's voxel
// column lies more than kClusterGap voxels (Chebyshev distance in x and y)
// from the cluster's columns, and more than twice the cluster's extent.
// The clusters are searched one after the other, each with its own box.  Heights are not compared: a column's ground and canopy points
// share their column runs, and splitting them was slower.
constexpr int32_t kClusterGap = 32;

// The query's voxel column (x and y voxel coordinates, clamped).
__device__ __forceinline__ void query_column(const Grid& g, const float (&qc)[3], int32_t (&qv)[2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a) qv[a] = (int32_t)voxel_clamped((double)qc[a], g.s[a], g.n[a]);
}

// Whether the lanes in todo (not empty) hold a compact set of queries: every
// query's voxel column, in FP32 voxel units, within kClusterGap of the
// first such lane's along x and y.  Uniform; both launches of a search
// evaluate it alike, and it costs one ballot (the launch that searches the
// other waves evaluates it for every wave).
__device__ __forceinline__ bool lanes_compact(uint64_t todo, const Grid& g, const float (&qc)[3],
                                              int lane) {
  const bool mine = (todo >> lane) & 1ull;
  const int src = __builtin_ctzll(todo);
  const float cx = floorf(qc[0] * (float)(1.0 / g.s[0]));
  const float cy = floorf(qc[1] * (float)(1.0 / g.s[1]));
  const float x0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cx), src));
  const float y0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cy), src));
  const float h = (float)kClusterGap;
  return __ballot(mine && (fabsf(cx - x0) > h || fabsf(cy - y0) > h)) == 0ull;
}

__device__ __forceinline__ uint64_t lane_cluster(uint64_t todo, const Grid& g,
                                                 const float (&qc)[3], int lane) {
  if (lanes_compact(todo, g, qc, lane)) return todo;
  int32_t qv[2];
  query_column(g, qc, qv);
  int l = __builtin_ctzll(todo);
  uint64_t cm = 1ull << l;
  uint64_t rest = todo & (todo - 1);
  int32_t lo[2], hi[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) lo[a] = hi[a] = __builtin_amdgcn_readlane(qv[a], l);
  while (rest) {
    l = __builtin_ctzll(rest);
    int32_t v[2], d = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      v[a] = __builtin_amdgcn_readlane(qv[a], l);
      const int32_t da = v[a] < lo[a] ? lo[a] - v[a] : (v[a] > hi[a] ? v[a] - hi[a] : 0);
      d = da > d ? da : d;
    }
    // a jump counts only if it is also long against the cluster's extent
    // (far-field queries spread over many voxels search best with one box)
    const int32_t ext = (hi[0] - lo[0]) > (hi[1] - lo[1]) ? (hi[0] - lo[0]) : (hi[1] - lo[1]);
    if (d > kClusterGap && d > 2 * ext) break;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      lo[a] = v[a] < lo[a] ? v[a] : lo[a];
      hi[a] = v[a] > hi[a] ? v[a] : hi[a];
    }
    cm |= 1ull << l;
    rest &= rest - 1;
  }
  return cm;
}

// Which waves a launch of the 64-query k-NN or radius tiles searches:
// kClAll every item with one box (the persistent form), kClCompact the
// items whose queries are compact or form one cluster (one box, no cluster
// loop, so the registers are those of the plain search; the others go to a
// list), kClSplit the listed items, cluster by cluster, with a grid of at
// most kSplitBlocks blocks.  The last two run as two launches.
constexpr int kClAll = 0, kClCompact = 1, kClSplit = 2;
constexpr unsigned kSplitBlocks = 2048;

struct VBox {
  int64_t lo[3], hi[3];
  bool empty;
};
struct IBox {
  int32_t lo[3], hi[3];
};

// Search kernels of Alg. 1 (Section 3.4.1; the cube and the cylinder of
// Section 2): each gives the box around the queries and an inside test.
enum KernelShape { kSphere = 0, kCube = 1, kCylinder = 2 };

// Voxel box covering [lo - pad, hi + pad] along every indexed axis, clamped
// to the grid; empty when it misses the grid.  KS: the cylinder's box spans
// every z voxel.
template <int KS = kSphere>
__device__ __forceinline__ VBox voxel_box(const Grid& g, const float* lo, const float* hi,
                                          double pad) {
  VBox b;
  b.empty = false;
  for (int a = 0; a < 3; ++a) {
    if (a >= g.dims) {
      b.lo[a] = 0;
      b.hi[a] = 0;
      continue;
    }
    if (KS == kCylinder && a == 2) {
      b.lo[2] = 0;
      b.hi[2] = g.n[2] - 1;
      continue;
    }
    const double clo = floor(((double)lo[a] - pad) / g.s[a]);
    const double chi = floor(((double)hi[a] + pad) / g.s[a]);
    // uniform values computed on the vector unit (there is no scalar FP64)
    // are moved back to scalar registers, so the loops they bound are not
    // divergent
    if (first_lane((int32_t)(chi < 0.0 || clo > (double)(g.n[a] - 1)))) {
      b.empty = true;
      b.lo[a] = 0;
      b.hi[a] = -1;
      continue;
    }
    b.lo[a] = first_lane(clo < 0.0 ? (int64_t)0 : (int64_t)clo);
    b.hi[a] = first_lane(chi > (double)(g.n[a] - 1) ? g.n[a] - 1 : (int64_t)chi);
  }
  return b;
}

// Lower bound of the horizontal distance between the tile's query box and
// column (i, j); columns farther than the search radius are skipped.  The
// column's extent is widened by a relative 1e-9 so that the FP64 rounding of
// the voxel function can never make this test drop a candidate.
__device__ __forceinline__ bool column_near(const Grid& g, const Tile& t, int64_t i, int64_t j,
                                            double pad) {
  const double x0 = (double)i * g.s[0], x1 = (double)(i + 1) * g.s[0];
  const double y0 = (double)j * g.s[1], y1 = (double)(j + 1) * g.s[1];
  const double ex = 1e-9 * (fabs(x1) + g.s[0]), ey = 1e-9 * (fabs(y1) + g.s[1]);
  double dx = fmax(0.0, fmax((x0 - ex) - (double)t.hi[0], (double)t.lo[0] - (x1 + ex)));
  double dy = fmax(0.0, fmax((y0 - ey) - (double)t.hi[1], (double)t.lo[1] - (y1 + ey)));
  return dx * dx + dy * dy <= pad * pad;
}

// As column_near, also giving hz, the largest height difference between a
// point within the padded radius of the box and the box's z range at this
// horizontal distance (in FP64, from the padded radius).
__device__ __forceinline__ bool column_near_z(const Grid& g, const Tile& t, int64_t i, int64_t j,
                                              double pad, double* hz) {
  const double x0 = (double)i * g.s[0], x1 = (double)(i + 1) * g.s[0];
  const double y0 = (double)j * g.s[1], y1 = (double)(j + 1) * g.s[1];
  const double ex = 1e-9 * (fabs(x1) + g.s[0]), ey = 1e-9 * (fabs(y1) + g.s[1]);
  double dx = fmax(0.0, fmax((x0 - ex) - (double)t.hi[0], (double)t.lo[0] - (x1 + ex)));
  double dy = fmax(0.0, fmax((y0 - ey) - (double)t.hi[1], (double)t.lo[1] - (y1 + ey)));
  const double h2 = pad * pad - (dx * dx + dy * dy);
  // widened (relatively, and absolutely by a 2^-18 share of the padded
  // radius, far above the FP64 rounding of the z bounds for any radius the
  // FP32 test can resolve): the z bounds then never cut a point the test
  // could admit
  *hz = (h2 > 0.0 ? sqrt(h2) * (1.0 + kPadRel) : 0.0) + pad * kPadRel;
  return h2 >= 0.0;
}

// ---------------------------------------------------------------- radius search
// Inside test in FP32 with unfused operations, differences fl32(q - p):
// sphere (dx*dx + dy*dy) + dz*dz <= R, cube |dx|, |dy|, |dz| <= r, cylinder
// dx*dx + dy*dy <= R, where R = fl32(r*r).  Lanes without a valid query pass
// r = R = -1, which nothing satisfies.
template <int KS>
__device__ __forceinline__ bool inside(float4 q, float4 P, float r, float R) {
  const float dx = q.x - P.x, dy = q.y - P.y;
  if (KS == kCube) {
    const float dz = q.z - P.z;
    return fabsf(dx) <= r && fabsf(dy) <= r && fabsf(dz) <= r;
  }
  if (KS == kCylinder) return dx * dx + dy * dy <= R;
  const float dz = q.z - P.z;
  return (dx * dx + dy * dy) + dz * dz <= R;
}

struct RadiusArgs {
  Waves W;
  Grid g0;  // the grid of a single-tile index
  const float4* __restrict__ pts;
  Voxels vx;
  float r;
  int32_t* __restrict__ counts;         // count pass: [nq] caller order
  const int64_t* __restrict__ offsets;  // fill pass: [nq+1]
  int32_t* __restrict__ nbr;            // fill pass: [total]
  int64_t total;                        // fill pass: entries of nbr
  // tiles, one wave per item (not persistent): [0] a count, then the items
  // whose queries are not compact, left by the first launch to the second
  int32_t* split = nullptr;
};

struct KnnArgs {
  Waves W;
  Grid g0;  // the grid of a single-tile index
  const float4* __restrict__ pts;
  Voxels vx;
  int32_t k;
  float rmax2;  // fl32(r_max^2), +inf without a radius cap
  int32_t* __restrict__ idx;
  float* __restrict__ d2;
  int64_t* __restrict__ visited;  // optional: [nq][2] voxels visited per query
  int32_t monotonic;  // growth schedule: radius + smallest voxel edge per step
  // one wave per item (not persistent): [0] a count, then the items whose
  // queries are not compact, left by the first launch to the second
  int32_t* split = nullptr;
};

// per-item tile lookups and persistent waves are needed by batched indexes
// and by the persistent option; a plain index uses the lighter kernels
inline bool multi(chs_index ix) { return ix->ntiles > 1 || ix->persistent; }

// Radius schedules (CHS_OPT_RADIUS_SCHEDULE): 64-query tiles streaming their
// union box, or 8-query groups packing their own candidate lists.
constexpr int kSchedAuto = 0, kSchedTiles = 1, kSchedGroups = 2;

// Kernel launches (radius.hip, knn.hip).  mean_rows: the fill's mean row
// length (neighbours per query).
void launch_radius(bool fill, chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A,
                   int32_t kernel, int64_t mean_rows);
void launch_knn(chs_index ix, unsigned nb, hipStream_t st, const KnnArgs& A);

}  // namespace chs
