// Neighbour search on the GPU: the kernel-based search of Section 3.4.1
// (Alg. 1) with a sphere, a cube or a cylinder, and k-NN (Section 3.4.2,
// Alg. 2, with the taboo box of Section 3.5), either as a ring expansion
// over voxels or with Alg. 2's density-growth radius.
//
// Work decomposition: a wavefront owns a tile of 64 consecutive queries in
// a Hilbert order over the (i, j) voxel columns, so its queries are spatial
// neighbours.  The tile's voxel box (the union of its queries' kernel boxes)
// is enumerated column by column, one column per lane; every column's voxels
// k0..k1 are contiguous in the stored order (the global index is z-fastest,
// Eq. 7), so each column yields one run of candidate points.  The wave then
// walks the runs with wave-uniform indices, so every candidate point is
// fetched once per wave through the scalar unit and compared against the 64
// queries held in the lanes (no per-lane gathers), with the unfused FP32
// arithmetic of the definitions.  LDS holds only per-lane output: the fill's
// staged matches and the k-NN's buffered keys.
#include <algorithm>
#include <cmath>

#include "common.h"

#pragma clang fp contract(off)

namespace chs {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;
constexpr uint32_t kInactive = 0x80000000u;
constexpr double kPadRel = 1.0 / 262144.0;              // 2^-18
constexpr double kPadAbs = 8.673617379884035e-19;       // 2^-60

static unsigned grid_for(int64_t n, int per_block = kThreads) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// ---------------------------------------------------------------- query planning
// Per tile: Hilbert order m (bits per axis), bits of the z voxel index, and
// the tile's processing rank (largest tiles first).
struct TilePlan {
  int32_t m, kbits, rank, pad_;
};

__device__ __forceinline__ int tile_of_point(const int64_t* __restrict__ toff, int ntiles, int64_t p) {
  int lo = 0, hi = ntiles - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (toff[mid] <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Per query: recentred FP32 centre (invalid queries are flagged) and the
// ordering key rank << lshift | hilbert(i, j) << kbits | k.
template <class K>
__global__ __launch_bounds__(kThreads) void k_plan_keys(
    int mode, const double* __restrict__ xyz, const int32_t* __restrict__ pidx, int64_t nq,
    const float4* __restrict__ pts, const int32_t* __restrict__ inv_perm,
    const int32_t* __restrict__ perm, int64_t npts, const Grid* __restrict__ tiles,
    TilePlan tp0, const TilePlan* __restrict__ tplan, const int64_t* __restrict__ toff,
    int ntiles, double ox, double oy, double oz, int lshift, int total_bits, K* __restrict__ keys,
    uint32_t* __restrict__ vals, float4* __restrict__ tmp) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= nq) return;
  float4 c;
  bool ok = true;
  uint32_t caller = (uint32_t)q;
  int t = 0;
  if (mode == 0) {  // every point, walked in stored order
    c = pts[q];
    caller = (uint32_t)perm[q];
    if (ntiles > 1) t = tile_of_point(toff, ntiles, (int64_t)caller);
  } else if (mode == 1) {  // point indices (single tile)
    const int32_t p = pidx[q];
    ok = p >= 0 && (int64_t)p < npts;
    c = ok ? pts[inv_perm[p]] : make_float4(0.f, 0.f, 0.f, 0.f);
  } else {  // FP64 coordinates (single tile)
    const double o[3] = {ox, oy, oz};
    float v[3];
    for (int a = 0; a < 3; ++a) {
      const double x = xyz[q * 3 + a];
      ok = ok && isfinite(x);
      v[a] = (float)(x - o[a]);
    }
    if (!ok) v[0] = v[1] = v[2] = 0.f;
    c = make_float4(v[0], v[1], v[2], 0.f);
  }
  const Grid g = tiles[t];
  const TilePlan tp = ntiles > 1 ? tplan[t] : tp0;
  int64_t cell[3] = {0, 0, 0};
  const float cc[3] = {c.x, c.y, c.z};
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a < g.dims) cell[a] = voxel_clamped((double)cc[a], g.s[a], g.n[a]);
  K key;
  if (ok) {
    const uint64_t local =
        (hilbert2((uint32_t)cell[0], (uint32_t)cell[1], tp.m) << tp.kbits) | (uint64_t)cell[2];
    key = (K)(((uint64_t)tp.rank << lshift) | local);
  } else {
    key = (K)(total_bits >= 64 ? ~0ull : ((1ull << total_bits) - 1));
  }
  keys[q] = key;
  vals[q] = (uint32_t)q;
  c.w = __uint_as_float(ok ? caller : (caller | kInactive));
  tmp[q] = c;
}

__global__ __launch_bounds__(kThreads) void k_plan_gather(const uint32_t* __restrict__ order,
                                                          const float4* __restrict__ tmp,
                                                          int64_t nq, float4* __restrict__ q4) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= nq) return;
  q4[t] = tmp[order[t]];
}

static chs_status plan_impl(chs_index ix, int mode, const double* xyz, const int32_t* pidx,
                            int64_t nq, const std::vector<int32_t>& rank, float4* q4,
                            hipStream_t st) {
  Alloc al = ix->al;
  al.stream = st;
  const int T = ix->ntiles;
  std::vector<TilePlan> tp(T);
  int lshift = 0;
  for (int t = 0; t < T; ++t) {
    const Grid& g = ix->tiles[t];
    tp[t].m = ceil_log2((uint64_t)(g.n[0] > g.n[1] ? g.n[0] : g.n[1]));
    tp[t].kbits = ceil_log2((uint64_t)g.n[2]);
    tp[t].rank = rank[t];
    tp[t].pad_ = 0;
    const int lb = 2 * tp[t].m + tp[t].kbits;
    lshift = lb > lshift ? lb : lshift;
  }
  const int bits = lshift + (T > 1 ? ceil_log2((uint64_t)T) : 0);
  if (bits > 64) {
    set_error("query ordering key would need %d bits", bits);
    return CHS_E_CAPACITY;
  }
  Buf keys(&al), vals(&al), tk(&al), tv(&al), tmp(&al), tp_d(&al), toff_d(&al);
  const bool wide = bits > 32;
  const size_t ks = wide ? 8 : 4;
  CHS_TRY(keys.alloc(ks * nq));
  CHS_TRY(tk.alloc(ks * nq));
  CHS_TRY(vals.alloc(4 * nq));
  CHS_TRY(tv.alloc(4 * nq));
  CHS_TRY(tmp.alloc(sizeof(float4) * nq));
  if (T > 1) {
    // (only the build plans several tiles; it waits for the stream before
    // these host vectors go out of scope)
    CHS_TRY(tp_d.alloc(sizeof(TilePlan) * T));
    CHS_TRY(toff_d.alloc(sizeof(int64_t) * (T + 1)));
    CHS_HIP(hipMemcpyAsync(tp_d.p, tp.data(), sizeof(TilePlan) * T, hipMemcpyHostToDevice, st));
    CHS_HIP(hipMemcpyAsync(toff_d.p, ix->tile_off.data(), sizeof(int64_t) * (T + 1),
                           hipMemcpyHostToDevice, st));
  }
  const double* o = ix->origin.data();
  if (wide) {
    k_plan_keys<uint64_t><<<grid_for(nq), kThreads, 0, st>>>(
        mode, xyz, pidx, nq, ix->pts, ix->inv_perm, ix->perm, ix->n, ix->tiles_d, tp[0],
        tp_d.as<TilePlan>(), toff_d.as<int64_t>(), T, o[0], o[1], o[2], lshift, bits,
        keys.as<uint64_t>(), vals.as<uint32_t>(), tmp.as<float4>());
    CHS_LAUNCH_CHECK();
    CHS_TRY(radix_sort_u64(al, keys.as<uint64_t>(), vals.as<uint32_t>(), tk.as<uint64_t>(),
                           tv.as<uint32_t>(), nq, bits));
  } else {
    k_plan_keys<uint32_t><<<grid_for(nq), kThreads, 0, st>>>(
        mode, xyz, pidx, nq, ix->pts, ix->inv_perm, ix->perm, ix->n, ix->tiles_d, tp[0],
        tp_d.as<TilePlan>(), toff_d.as<int64_t>(), T, o[0], o[1], o[2], lshift, bits,
        keys.as<uint32_t>(), vals.as<uint32_t>(), tmp.as<float4>());
    CHS_LAUNCH_CHECK();
    CHS_TRY(radix_sort_u32(al, keys.as<uint32_t>(), vals.as<uint32_t>(), tk.as<uint32_t>(),
                           tv.as<uint32_t>(), nq, bits));
  }
  k_plan_gather<<<grid_for(nq), kThreads, 0, st>>>(vals.as<uint32_t>(), tmp.as<float4>(), nq, q4);
  CHS_LAUNCH_CHECK();
  if (T > 1) CHS_HIP(hipStreamSynchronize(st));  // tp, toff copies read host vectors
  return CHS_OK;
}

chs_status check_queries(chs_index ix, const chs_queries* qs) {
  if (!ix || !qs) {
    set_error("index or queries is NULL");
    return CHS_E_INVALID;
  }
  if (qs->xyz && qs->point_idx) {
    set_error("queries: give xyz or point_idx, not both");
    return CHS_E_INVALID;
  }
  if (qs->nq < 0 || qs->nq > (int64_t)INT32_MAX) {
    set_error("queries: nq = %lld outside [0, 2^31 - 1]", (long long)qs->nq);
    return CHS_E_INVALID;
  }
  if (!qs->xyz && !qs->point_idx && qs->nq != 0 && qs->nq != ix->n) {
    set_error("queries: with neither xyz nor point_idx, nq must equal the cloud size %lld",
              (long long)ix->n);
    return CHS_E_INVALID;
  }
  if (ix->ntiles > 1 && qs->nq != 0 && (qs->xyz || qs->point_idx)) {
    set_error("a batched index answers \"every point\" queries only");
    return CHS_E_UNSUPPORTED;
  }
  return CHS_OK;
}

// Processing order of "every point" queries, computed once by the build and
// kept on the index: centres in Hilbert order, in waves of at most 64 that
// never straddle two tiles (largest tiles first).
chs_status plan_every_point(chs_index ix, hipStream_t st) {
  const int T = ix->ntiles;
  std::vector<int64_t> order(T);
  for (int t = 0; t < T; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return ix->tile_off[a + 1] - ix->tile_off[a] > ix->tile_off[b + 1] - ix->tile_off[b];
  });
  std::vector<int32_t> rank(T);
  for (int r = 0; r < T; ++r) rank[order[r]] = r;
  float4* a = nullptr;
  CHS_TRY(ix->own(&a, (size_t)ix->n));
  CHS_TRY(plan_impl(ix, 0, nullptr, nullptr, ix->n, rank, a, st));
  if (T > 1) {
    std::vector<int32_t> wtile, wstart, qend(T);
    int64_t pos = 0;
    for (int r = 0; r < T; ++r) {
      const int t = (int)order[r];
      const int64_t nt = ix->tile_off[t + 1] - ix->tile_off[t];
      for (int64_t b = 0; b < nt; b += kWave) {
        wtile.push_back(t);
        wstart.push_back((int32_t)(pos + b));
      }
      pos += nt;
      qend[t] = (int32_t)pos;
    }
    CHS_TRY(ix->own(&ix->wave_tile, wtile.size()));
    CHS_TRY(ix->own(&ix->wave_start, wstart.size()));
    CHS_TRY(ix->own(&ix->tile_qend, (size_t)T));
    CHS_HIP(hipMemcpyAsync(ix->wave_tile, wtile.data(), 4 * wtile.size(), hipMemcpyHostToDevice, st));
    CHS_HIP(hipMemcpyAsync(ix->wave_start, wstart.data(), 4 * wstart.size(), hipMemcpyHostToDevice, st));
    CHS_HIP(hipMemcpyAsync(ix->tile_qend, qend.data(), 4 * (size_t)T, hipMemcpyHostToDevice, st));
    CHS_HIP(hipStreamSynchronize(st));
    ix->allq_waves = (int64_t)wtile.size();
  } else {
    ix->allq_waves = (ix->n + kWave - 1) / kWave;
  }
  ix->allq = a;
  return CHS_OK;
}

chs_status plan_queries(chs_index ix, const chs_queries* qs, QueryPlan* plan, hipStream_t st) {
  plan->nq = qs->nq;
  plan->wave_tile = nullptr;
  plan->wave_start = nullptr;
  plan->tile_qend = nullptr;
  plan->nwaves = (qs->nq + kWave - 1) / kWave;
  if (qs->nq == 0) return CHS_OK;
  if (!qs->xyz && !qs->point_idx) {
    plan->q = ix->allq;
    plan->wave_tile = ix->wave_tile;
    plan->wave_start = ix->wave_start;
    plan->tile_qend = ix->tile_qend;
    plan->nwaves = ix->allq_waves;
    return CHS_OK;
  }
  CHS_TRY(plan->q4.alloc(sizeof(float4) * qs->nq));
  const std::vector<int32_t> rank(1, 0);
  CHS_TRY(plan_impl(ix, qs->point_idx ? 1 : 2, qs->xyz, qs->point_idx, qs->nq, rank,
                    plan->q4.as<float4>(), st));
  plan->q = plan->q4.as<float4>();
  return CHS_OK;
}

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

__global__ void k_reset_counter(int32_t* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
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
};

// Fill-pass staging: each lane appends its matches to a private LDS
// segment; when some segment could overflow in the next group of
// candidates, the wave flushes the segments, writing each lane's entries to
// that lane's CSR row as one contiguous run (two rows per store
// instruction, one per half-wave) instead of 64 scattered 4-byte stores per
// candidate, which the memory system would write back as 64 partial lines.
// Every store is also checked against its row's end.
constexpr int kGroup = 8;                   // candidates loaded together in the fill
constexpr int kFlushUnroll = 4;             // lane pairs written per flush step
// Stage of ST entries per lane.  A flush writes only the lanes holding at
// least min_flush entries (the others keep theirs for the next flush), so
// that stores carry more entries.  The stage's LDS bounds the waves per
// CU: short rows take the small stage (more waves in flight), long rows
// the larger one (fewer flushes).
template <int ST>
struct Stage {
  static constexpr int size = ST;
  static constexpr int stride = ST + 1;  // odd, against LDS bank conflicts
  static constexpr int min_flush = ST <= 16 ? 6 : (ST <= 24 ? 10 : 12);
  static_assert(min_flush <= ST - kGroup, "a kept run must leave room for a group");
};
constexpr int kStageShort = 16, kStageMid = 24, kStageLong = 32;
// mean row lengths (neighbours per query) from which the fill takes the
// middle and the long stage
constexpr int64_t kMidRows = 64, kLongRows = 256;

// Where a lane's staged entries go: the row position and how many of them
// are written (published once per flush, read by the half-waves).
struct alignas(16) RowSlot {
  int64_t pos;
  int32_t cnt, pad_;
};

// FINAL: the lane's last flush, everything staged is written.
template <bool FINAL, int ST>
__device__ __forceinline__ void flush_stage(const int32_t* seg_base, RowSlot* rows, int lane,
                                            int& nb, int64_t& wpos, int64_t wend,
                                            int32_t* __restrict__ nbr) {
  const int32_t used = (FINAL || nb >= Stage<ST>::min_flush) ? nb : 0;
  const int64_t room = wend - wpos;
  RowSlot slot;
  slot.pos = wpos;
  slot.cnt = room <= 0 ? 0 : (room < used ? (int32_t)room : used);
  slot.pad_ = 0;
  rows[lane] = slot;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int half = lane >> 5, i = lane & 31;
  // pairs of lanes (2m, 2m+1) with entries to write: lanes 0-31 copy lane
  // 2m's run, lanes 32-63 lane 2m+1's, each a contiguous row segment.  A
  // step takes kFlushUnroll pairs, so that all their LDS reads are in flight
  // before the first store.
  const uint64_t pending = __ballot(slot.cnt > 0);
  uint64_t pairs = (pending | (pending >> 1)) & 0x5555555555555555ull;
  while (pairs) {
    int src[kFlushUnroll];
    bool ok[kFlushUnroll];
#pragma unroll
    for (int u = 0; u < kFlushUnroll; ++u) {
      ok[u] = pairs != 0;
      src[u] = (ok[u] ? __builtin_ctzll(pairs) : 0) + half;
      pairs &= pairs - 1;
    }
    RowSlot r[kFlushUnroll];
    int32_t v[kFlushUnroll];
#pragma unroll
    for (int u = 0; u < kFlushUnroll; ++u) {
      r[u] = rows[src[u]];
      v[u] = seg_base[src[u] * Stage<ST>::stride + i];
    }
    // keep the reads ahead of every store (the compiler would otherwise sink
    // some of them into the stores' branches, one LDS round trip each)
#pragma unroll
    for (int u = 0; u < kFlushUnroll; ++u) asm volatile("" ::"v"(v[u]), "v"(r[u].pos), "v"(r[u].cnt));
#pragma unroll
    for (int u = 0; u < kFlushUnroll; ++u)
      if (ok[u] && i < r[u].cnt) nbr[r[u].pos + i] = v[u];
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  wpos += used;
  nb -= used;
}

template <bool FILL, bool MULTI, int FL, int KS, int ST>
__device__ __forceinline__ void radius_item(const RadiusArgs& A, const Item& it, int lane,
                                            int32_t* seg_base, RowSlot* rows) {
  const Grid g = MULTI ? A.W.tiles[it.tile] : A.g0;
  const int64_t t = it.t0 + lane;
  const bool in = t < it.tend;
  const float4 q = in ? A.W.q4[t] : make_float4(0.f, 0.f, 0.f, __uint_as_float(kInactive));
  const uint32_t wq = __float_as_uint(q.w);
  const uint32_t qid = wq & ~kInactive;
  const bool active = in && !(wq & kInactive) && (int64_t)qid < A.W.nq;
  const Tile tb = tile_bounds(q, active);
  // fl32(r*r); lanes without a valid query get negative bounds so that no
  // candidate (D >= 0, |d| >= 0, or NaN) ever matches for them and they
  // write nothing
  const float R = active ? A.r * A.r : -1.0f;
  const float rr = active ? A.r : -1.0f;
  const double pad = fmax((double)A.r * (1.0 + kPadRel), kPadAbs);
  const int32_t poff = (int32_t)g.poff;
  int32_t cnt = 0;
  int64_t wpos = 0, wend = 0;
  int nb = 0;
  int32_t* my_seg = seg_base + (FILL ? lane * Stage<ST>::stride : 0);
  if (FILL && active) {
    // rows are clipped to nbr's extent: offsets that do not belong to these
    // queries and this r write nothing outside [0, total)
    wpos = A.offsets[qid];
    wend = A.offsets[qid + 1];
    if (wend > A.total) wend = A.total;
    if (wpos < 0 || wpos > wend) wpos = wend = 0;
  }
  if (tb.any) {
    const VBox bx = voxel_box<KS>(g, tb.lo, tb.hi, pad);
    if (!bx.empty) {
      const int64_t nj = bx.hi[1] - bx.lo[1] + 1;
      const int64_t ncol = (bx.hi[0] - bx.lo[0] + 1) * nj;
      for (int64_t cb = 0; cb < ncol; cb += kWave) {
        const int64_t c = cb + lane;
        int32_t b = 0, e = 0;
        if (c < ncol) {
          const int64_t ci = bx.lo[0] + c / nj, cj = bx.lo[1] + c % nj;
          // the cube's box already bounds every column it holds
          if (KS == kCube || column_near(g, tb, ci, cj, pad))
            column_run<FL>(A.vx, g, ci, cj, bx.lo[2], bx.hi[2], &b, &e);
        }
        uint64_t m = __ballot(e > b);
        while (m) {
          const int src = __builtin_ctzll(m);
          m &= m - 1;
          const int32_t rb = __builtin_amdgcn_readlane(b, src);
          const int32_t re = __builtin_amdgcn_readlane(e, src);
          if (!FILL) {
            // read through the constant address space: in the persistent
            // loop the work counter's atomic would otherwise turn these
            // wave-uniform loads into vector loads
            const_pts cp = as_const(A.pts);
#pragma unroll 4
            for (int32_t p = rb; p < re; ++p) {
              const float4 P = load_const(cp, p);
              cnt += inside<KS>(q, P, rr, R) ? 1 : 0;
            }
          } else {
            // groups of kGroup candidates: their loads are issued together,
            // and the stage is flushed whenever a lane could overflow it in
            // the next group.  Every candidate is written to the next free
            // slot and kept only if it matches (no divergent branch per
            // candidate); a stage never holds more than ST - kGroup
            // entries before a group, so the slot is always in range.
            const_pts cp = as_const(A.pts);
            int32_t p = rb;
            for (; p + kGroup <= re; p += kGroup) {
              float4 P[kGroup];
#pragma unroll
              for (int u = 0; u < kGroup; ++u) P[u] = load_const(cp, p + u);
#pragma unroll
              for (int u = 0; u < kGroup; ++u) {
                my_seg[nb] = __float_as_int(P[u].w) - poff;
                nb += inside<KS>(q, P[u], rr, R) ? 1 : 0;
              }
              if (__ballot(nb > ST - kGroup)) flush_stage<false, ST>(seg_base, rows, lane, nb, wpos, wend, A.nbr);
            }
            for (; p < re; ++p) {
              const float4 P = load_const(cp, p);
              my_seg[nb] = __float_as_int(P.w) - poff;
              nb += inside<KS>(q, P, rr, R) ? 1 : 0;
              if (__ballot(nb > ST - kGroup)) flush_stage<false, ST>(seg_base, rows, lane, nb, wpos, wend, A.nbr);
            }
          }
        }
      }
    }
  }
  if (FILL) flush_stage<true, ST>(seg_base, rows, lane, nb, wpos, wend, A.nbr);
  if (!FILL && in && (int64_t)qid < A.W.nq) A.counts[qid] = active ? cnt : 0;
}

// MULTI: per-item tile lookups and, if a counter is given, a persistent
// loop over work items; otherwise one wave per item with tile 0's grid.
// ST: entries per lane of the fill's stage (unused by the count pass)
template <bool FILL, bool MULTI, int FL, int KS, int ST>
__global__ __launch_bounds__(kThreads) void k_radius(RadiusArgs A) {
  __shared__ int32_t s_stage[FILL ? kWavesPerBlock * kWave * Stage<ST>::stride : 1];
  __shared__ RowSlot s_rows[FILL ? kWavesPerBlock * kWave : 1];
  const int w = threadIdx.x / kWave, lane = lane_id();
  int32_t* seg_base = s_stage + (FILL ? w * kWave * Stage<ST>::stride : 0);
  RowSlot* rows = s_rows + (FILL ? w * kWave : 0);
  int64_t own = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + w;
  if (!MULTI) {
    if (own < A.W.nwaves)
      radius_item<FILL, false, FL, KS, ST>(A, item_of(A.W, own), lane, seg_base, rows);
    return;
  }
  while (true) {
    const int64_t item = next_item(A.W, &own, lane);
    if (item >= A.W.nwaves) break;
    radius_item<FILL, true, FL, KS, ST>(A, item_of(A.W, item), lane, seg_base, rows);
  }
}

// ---------------------------------------------------------------- k-NN
struct KnnArgs {
  Waves W;
  Grid g0;  // the grid of a single-tile index
  const float4* __restrict__ pts;
  Voxels vx;
  int32_t k;
  float rmax2;  // fl32(r_max^2), +inf without a radius cap
  int32_t* __restrict__ idx;
  float* __restrict__ d2;
};

// The list of a lane is kept sorted in registers, best[0..KC) ascending, as
// 64-bit keys (distance bits << 32 | original index).  Candidates below the
// current k-th key are appended to a per-lane buffer in LDS; when some lane's
// buffer could overflow, and at the end of every ring, each lane sorts its
// buffer and merges it in with a bitonic network, so the wave pays for one
// merge per KB accepted candidates of its busiest lane instead of one
// insertion for every candidate that any lane accepts.
// Lists shorter than kKnnBufMin take the insertion directly: their
// insertion network is short enough that buffering does not pay.  Longer
// lists buffer kKnnBufLong keys, which keeps the merge's registers (list +
// sorted buffer) and the buffers' LDS small enough for several waves per SIMD.
constexpr int kKnnBufMin = 16;
constexpr int kKnnBufLong = 8;
template <int KC>
struct KnnBuf {
  static constexpr bool on = KC >= kKnnBufMin;
  // candidates loaded together; buffered lists take small groups so that a
  // merge is due only when some buffer is nearly full
  static constexpr int group = on ? 2 : 4;
  static constexpr int KB = KC < 16 ? KC : kKnnBufLong;   // buffered keys per lane
  static constexpr int stride = KB + 1;                   // odd, against bank conflicts
};

// Sorted insertion of key x < best[KC-1] into best[0..KC) (ascending),
// dropping the last entry.  With c[i] = x < best[i] (monotone in i, keys
// are distinct): best'[i] = best[i-1] if c[i-1], else x if c[i], else
// best[i]; one compare per slot.  The list passes through an empty asm so
// that the selects are not rewritten as min/max pairs with compares of
// their own.
template <int KC>
__device__ __forceinline__ void topk_insert(uint64_t (&best)[KC], uint64_t x) {
  bool c[KC];
#pragma unroll
  for (int i = 0; i < KC; ++i) c[i] = x < best[i];
  uint64_t v[KC];
#pragma unroll
  for (int i = 0; i < KC; ++i) {
    v[i] = best[i];
    asm("" : "+v"(v[i]));
  }
#pragma unroll
  for (int i = KC - 1; i > 0; --i) best[i] = c[i - 1] ? v[i - 1] : (c[i] ? x : v[i]);
  best[0] = c[0] ? x : v[0];
}

// One compare feeds both selects.  The operands pass through an empty asm
// first: selects over the compared values themselves would be rewritten as
// a separate min and max, each with its own 64-bit compare.
__device__ __forceinline__ void cmp_swap(uint64_t& a, uint64_t& b) {
  const bool s = b < a;
  uint64_t x = a, y = b;
  asm("" : "+v"(x), "+v"(y));
  a = s ? y : x;
  b = s ? x : y;
}

template <int N>
__device__ __forceinline__ void bitonic_sort(uint64_t (&x)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          if ((i & k) == 0) cmp_swap(x[i], x[l]);
          else cmp_swap(x[l], x[i]);
        }
      }
}

// Eight keys ascending with 19 compare-exchanges (the optimal network for
// eight inputs; bitonic sorting takes 24).
__device__ __forceinline__ void sort8(uint64_t (&x)[8]) {
  constexpr int net[19][2] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6},
                              {3, 7}, {0, 1}, {2, 3}, {4, 5}, {6, 7}, {2, 4}, {3, 5},
                              {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
  for (int c = 0; c < 19; ++c) cmp_swap(x[net[c][0]], x[net[c][1]]);
}

// x bitonic -> x ascending.  x[0..P) is known to be ascending already, so
// first-stage pairs that lie inside it are in order and skipped.
template <int N, int P>
__device__ __forceinline__ void bitonic_merge(uint64_t (&x)[N]) {
#pragma unroll
  for (int j = N >> 1; j > 0; j >>= 1)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int l = i ^ j;
      if (l > i && !(j == N / 2 && l < P)) cmp_swap(x[i], x[l]);
    }
}

// best[k-1] for the uniform k
// (masks rather than selects, which the compiler would otherwise turn into
// an indexed load from a memory copy of the list)
template <int KC>
__device__ __forceinline__ uint64_t kth_key(const uint64_t (&best)[KC], int k) {
  if (KC <= 32 && k == KC) return best[KC - 1];  // k is uniform
  uint64_t v = 0;
#pragma unroll
  for (int i = 0; i < KC; ++i) v |= best[i] & (0ull - (uint64_t)(i == k - 1));
  return v;
}

// Merge the lane's nb buffered keys into best: the buffer sorted ascending,
// min(best[KC-1-j], buf[j]) forms a bitonic sequence holding the KC smallest
// keys of both, which the merge network sorts.
template <int KC>
__device__ __forceinline__ void merge_buffer(uint64_t (&best)[KC], const uint64_t* seg, int& nb) {
  constexpr int KB = KnnBuf<KC>::KB;
  uint64_t b[KB];
#pragma unroll
  for (int i = 0; i < KB; ++i) b[i] = i < nb ? seg[i] : ~0ull;
  if constexpr (KB == 8) sort8(b);
  else bitonic_sort<KB>(b);
#pragma unroll
  for (int j = 0; j < KB; ++j) best[KC - 1 - j] = b[j] < best[KC - 1 - j] ? b[j] : best[KC - 1 - j];
  // best[0 .. KC-KB) was not touched and is still ascending
  bitonic_merge<KC, KC - KB>(best);
  nb = 0;
}

// Scan the candidates [rb, re) of one run (wave-uniform), groups of KnnBuf::group
// loaded together through the scalar unit.
template <int KC>
__device__ __forceinline__ void knn_scan(const_pts cp, int32_t rb, int32_t re, float4 q,
                                         float rmax2, int k, uint64_t (&best)[KC], uint64_t& kthk,
                                         uint64_t* seg, int& nb) {
  constexpr int KB = KnnBuf<KC>::KB;
  constexpr int kKnnGroup = KnnBuf<KC>::group;
  int32_t p = rb;
  for (; p + kKnnGroup <= re; p += kKnnGroup) {
    float4 P[kKnnGroup];
#pragma unroll
    for (int u = 0; u < kKnnGroup; ++u) P[u] = load_const(cp, p + u);
#pragma unroll
    for (int u = 0; u < kKnnGroup; ++u) {
      const float dx = q.x - P[u].x, dy = q.y - P[u].y, dz = q.z - P[u].z;
      const float D = (dx * dx + dy * dy) + dz * dz;
      // D >= 0, so its bit pattern orders like its value; ties go to the
      // lower original index in the low word
      const uint64_t key = ((uint64_t)__float_as_uint(D) << 32) | (uint64_t)__float_as_uint(P[u].w);
      if (KnnBuf<KC>::on) {
        // written to the next free slot, kept only if accepted
        seg[nb] = key;
        nb += (D <= rmax2 && key < kthk) ? 1 : 0;
      } else if (D <= rmax2 && key < best[KC - 1]) {
        topk_insert<KC>(best, key);
      }
    }
    if (KnnBuf<KC>::on && __ballot(nb > KB - kKnnGroup)) {
      merge_buffer<KC>(best, seg, nb);
      kthk = kth_key<KC>(best, k);
    }
  }
  for (; p < re; ++p) {
    const float4 P = load_const(cp, p);
    const float dx = q.x - P.x, dy = q.y - P.y, dz = q.z - P.z;
    const float D = (dx * dx + dy * dy) + dz * dz;
    const uint64_t key = ((uint64_t)__float_as_uint(D) << 32) | (uint64_t)__float_as_uint(P.w);
    if (KnnBuf<KC>::on) {
      seg[nb] = key;
      nb += (D <= rmax2 && key < kthk) ? 1 : 0;
    } else if (D <= rmax2 && key < best[KC - 1]) {
      topk_insert<KC>(best, key);
    }
    if (KnnBuf<KC>::on && __ballot(nb > KB - kKnnGroup)) {
      merge_buffer<KC>(best, seg, nb);
      kthk = kth_key<KC>(best, k);
    }
  }
}

// Box of voxels (clamped into the grid) covering the padded balls of radius
// r around the queries of the unfinished lanes, as a hull with V when V is
// not empty (uniform).
__device__ __forceinline__ IBox lane_hull(const Grid& g, const float (&qc)[3], double r, bool live,
                                          const IBox& V, bool vempty) {
  IBox B;
  const double pad = fmax(r * (1.0 + kPadRel), kPadAbs);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= g.dims) {
      B.lo[a] = B.hi[a] = 0;
      continue;
    }
    const int32_t lo = (int32_t)voxel_clamped((double)qc[a] - pad, g.s[a], g.n[a]);
    const int32_t hi = (int32_t)voxel_clamped((double)qc[a] + pad, g.s[a], g.n[a]);
    int32_t l = wave_min(live ? lo : INT32_MAX), h = wave_max(live ? hi : INT32_MIN);
    if (!vempty) {
      l = V.lo[a] < l ? V.lo[a] : l;
      h = V.hi[a] > h ? V.hi[a] : h;
    }
    B.lo[a] = l;
    B.hi[a] = h;
  }
  return B;
}

// SCHED: kRings grows the visited box by one voxel per step and stops a
// lane by the distance to the box's faces; kDensity is the schedule of
// Alg. 2: each lane starts at the distance to the nearest wall of its voxel
// (Eq. 11), grows its radius from the density of the candidates within it
// (Eq. 12) or by the smallest voxel edge, and stops once k keys lie within
// the radius.  The wave visits the hull of its unfinished lanes' kernel
// boxes.  Both give the exact k nearest.
constexpr int kRings = 0, kDensity = 1;

template <int KC, bool MULTI, int FL, int SCHED>
__device__ __forceinline__ void knn_item(const KnnArgs& A, const Item& it, int lane,
                                         uint64_t* seg) {
  const Grid g = MULTI ? A.W.tiles[it.tile] : A.g0;
  const int64_t t = it.t0 + lane;
  const bool in = t < it.tend;
  const float4 q = in ? A.W.q4[t] : make_float4(0.f, 0.f, 0.f, __uint_as_float(kInactive));
  const uint32_t wq = __float_as_uint(q.w);
  const uint32_t qid = wq & ~kInactive;
  const bool active = in && !(wq & kInactive) && (int64_t)qid < A.W.nq;
  const Tile tb = tile_bounds(q, active);
  const const_pts cp = as_const(A.pts);
  // lanes without a valid query accept nothing
  const float rmax2 = active ? A.rmax2 : -1.0f;
  uint64_t best[KC];
#pragma unroll
  for (int i = 0; i < KC; ++i) best[i] = ~0ull;
  uint64_t kthk = ~0ull;
  int nb = 0;
  if (tb.any) {
    const float qc[3] = {q.x, q.y, q.z};
    // density schedule: the lane's radius, starting at the distance from
    // the query to the nearest wall of its voxel (Eq. 11)
    double rL = 0.0, smin = INFINITY;
    bool done = !active;
    if (SCHED == kDensity) {
      rL = INFINITY;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (a >= g.dims) continue;
        smin = fmin(smin, g.s[a]);
        const double c = (double)qc[a];
        const double v = (double)voxel_clamped(c, g.s[a], g.n[a]);
        rL = fmin(rL, fmin(fabs(c - v * g.s[a]), fabs(c - (v + 1.0) * g.s[a])));
      }
      if (!(rL > 0.0)) rL = smin;  // a centre on a wall would start at 0
    }
    IBox V;  // visited voxels (the taboo box)
    bool vempty = true;
    // first box: the voxels holding the tile's queries (clamped into the
    // grid), or the unfinished lanes' kernel boxes; voxel coordinates fit
    // 32 bits (fewer than 1e9 voxels per axis)
    IBox B;
    if (SCHED == kDensity) {
      B = lane_hull(g, qc, rL, !done, V, true);
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (a >= g.dims) {
          B.lo[a] = B.hi[a] = 0;
          continue;
        }
        B.lo[a] = first_lane((int32_t)voxel_clamped((double)tb.lo[a], g.s[a], g.n[a]));
        B.hi[a] = first_lane((int32_t)voxel_clamped((double)tb.hi[a], g.s[a], g.n[a]));
      }
    }
    // Points farther from the tile's query box than every unfinished lane's
    // threshold can never enter a list (thresholds only shrink), so columns
    // and z-ranges beyond that distance are skipped; +inf until every
    // unfinished lane holds k keys.
    double tau = INFINITY;
    while (true) {
      int32_t kz0 = B.lo[2], kz1 = B.hi[2];
      double padk = INFINITY;
      // (the density schedule's radii grow, so nothing may be skipped there)
      if (SCHED == kRings && tau < INFINITY) {
        padk = fmax(sqrt(tau) * (1.0 + kPadRel), kPadAbs);
        if (g.dims == 3) {
          const double zlo = floor(((double)tb.lo[2] - padk) / g.s[2]);
          const double zhi = floor(((double)tb.hi[2] + padk) / g.s[2]);
          if (zlo > (double)kz0) kz0 = (int32_t)zlo;
          if (zhi < (double)kz1) kz1 = (int32_t)zhi;
          kz0 = first_lane(kz0);
          kz1 = first_lane(kz1);
        }
      }
      // visit B minus V, column by column (one column per lane)
      const int64_t nj = B.hi[1] - B.lo[1] + 1;
      const int64_t ncol = (int64_t)(B.hi[0] - B.lo[0] + 1) * nj;
      for (int64_t cb = 0; cb < ncol; cb += kWave) {
        const int64_t c = cb + lane;
        int32_t b0 = 0, e0 = 0, b1 = 0, e1 = 0;
        if (c < ncol && kz0 <= kz1) {
          const int64_t ci = B.lo[0] + c / nj, cj = B.lo[1] + c % nj;
          const bool inner = !vempty && ci >= V.lo[0] && ci <= V.hi[0] && cj >= V.lo[1] &&
                             cj <= V.hi[1];
          if (padk == INFINITY || column_near(g, tb, ci, cj, padk)) {
            if (!inner) {
              column_run<FL>(A.vx, g, ci, cj, kz0, kz1, &b0, &e0);
            } else {
              const int32_t a1 = V.lo[2] - 1 < kz1 ? V.lo[2] - 1 : kz1;
              const int32_t a2 = V.hi[2] + 1 > kz0 ? V.hi[2] + 1 : kz0;
              if (kz0 <= a1) column_run<FL>(A.vx, g, ci, cj, kz0, a1, &b0, &e0);
              if (a2 <= kz1) column_run<FL>(A.vx, g, ci, cj, a2, kz1, &b1, &e1);
            }
          }
        }
        uint64_t m0 = __ballot(e0 > b0);
        while (m0) {
          const int src = __builtin_ctzll(m0);
          m0 &= m0 - 1;
          knn_scan<KC>(cp, __builtin_amdgcn_readlane(b0, src), __builtin_amdgcn_readlane(e0, src),
                       q, rmax2, A.k, best, kthk, seg, nb);
        }
        uint64_t m1 = __ballot(e1 > b1);
        while (m1) {
          const int src = __builtin_ctzll(m1);
          m1 &= m1 - 1;
          knn_scan<KC>(cp, __builtin_amdgcn_readlane(b1, src), __builtin_amdgcn_readlane(e1, src),
                       q, rmax2, A.k, best, kthk, seg, nb);
        }
      }
      if (KnnBuf<KC>::on && __ballot(nb > 0)) merge_buffer<KC>(best, seg, nb);
      kthk = kth_key<KC>(best, A.k);
      V = B;
      vempty = false;
      bool whole = true;  // V is the whole grid (decided from V alone: uniform)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (a >= g.dims) continue;
        if (V.lo[a] > 0 || V.hi[a] < g.n[a] - 1) whole = false;
      }
      if (whole) break;
      if (SCHED == kDensity) {
        // k keys within fl32(rL^2): every unvisited point lies beyond the
        // padded ball of radius rL, so its D exceeds that bound; past the
        // radius cap nothing more can be returned
        const float T = (float)(rL * rL);
        const uint32_t tb32 = __float_as_uint(T);
        done = done || (kthk != ~0ull && (uint32_t)(kthk >> 32) <= tb32) ||
               (double)A.rmax2 <= rL * rL;
        if (__ballot(!done) == 0ull) break;
        if (!done) {
          // |P^|: candidates within the radius (Eq. 10); the list is sorted
          int np = 0;
#pragma unroll
          for (int i = 0; i < KC; ++i) np += (uint32_t)(best[i] >> 32) <= tb32 ? 1 : 0;
          double rn = rL + smin;  // monotonic growth
          if (np > 0) {
            const double rho = (double)np / ((4.0 / 3.0) * M_PI * rL * rL * rL);  // Eq. 12
            const double rd = cbrt((double)A.k / rho);
            if (rd > rL) rn = rd;
          }
          rL = rn;
        }
        B = lane_hull(g, qc, rL, !done, V, false);
        continue;
      }
      // termination: every point outside V lies beyond the nearest face of V
      // that is not on the grid boundary; once the k-th best (or the radius
      // cap) is strictly below that distance squared, nothing outside V can
      // enter the list (ties included).
      float thr = A.rmax2;
      if (kthk != ~0ull) {
        const float dk = __uint_as_float((uint32_t)(kthk >> 32));
        thr = dk < thr ? dk : thr;
      }
      double lb = INFINITY;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (a >= g.dims) continue;
        const double c = (double)qc[a];
        if (V.lo[a] > 0) {
          const double f = (double)V.lo[a] * g.s[a];
          lb = fmin(lb, (c - f) - 0x1p-50 * (fabs(c) + fabs(f)));
        }
        if (V.hi[a] < g.n[a] - 1) {
          const double f = (double)(V.hi[a] + 1) * g.s[a];
          lb = fmin(lb, (f - c) - 0x1p-50 * (fabs(c) + fabs(f)));
        }
      }
      lb = fmax(lb, 0.0);
      const double lb2 = lb * lb;
      done = !active || (lb2 >= 0x1p-100 && (double)thr < lb2 * (1.0 - kPadRel));
      if (__ballot(!done) == 0ull) break;
      tau = wave_max(done ? -INFINITY : (double)thr);
      // next ring: grow the box by one voxel on every side
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (a >= g.dims) continue;
        B.lo[a] = V.lo[a] > 0 ? V.lo[a] - 1 : 0;
        B.hi[a] = V.hi[a] < g.n[a] - 1 ? V.hi[a] + 1 : g.n[a] - 1;
      }
    }
  }
  if (in && (int64_t)qid < A.W.nq) {
    int32_t* ro = A.idx + (int64_t)qid * A.k;
    float* rd = A.d2 + (int64_t)qid * A.k;
    const int32_t poff = (int32_t)g.poff;
#pragma unroll
    for (int i = 0; i < KC; ++i) {
      if (i < A.k) {
        const uint64_t key = active ? best[i] : ~0ull;
        const bool ok = key != ~0ull;
        ro[i] = ok ? (int32_t)(uint32_t)key - poff : -1;
        rd[i] = ok ? __uint_as_float((uint32_t)(key >> 32)) : INFINITY;
      }
    }
  }
}

// Lists of 32 run at four waves per SIMD, of 16 at six and of 8 at eight:
// the few registers spilled cost less than the latency hiding gained
// (measured on the 10 M-point tile).
template <int KC, bool MULTI, int FL, int SCHED>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(KC == 32 ? 4 : (KC == 16 ? 6 : (KC == 8 ? 8 : 1)))))
void k_knn(KnnArgs A) {
  constexpr int kSeg = KnnBuf<KC>::on ? kWave * KnnBuf<KC>::stride : 1;
  __shared__ uint64_t s_buf[kWavesPerBlock * kSeg];
  const int w = threadIdx.x / kWave, lane = lane_id();
  uint64_t* seg = s_buf + w * kSeg + (KnnBuf<KC>::on ? lane * KnnBuf<KC>::stride : 0);
  int64_t own = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + w;
  if (!MULTI) {
    if (own < A.W.nwaves) knn_item<KC, false, FL, SCHED>(A, item_of(A.W, own), lane, seg);
    return;
  }
  while (true) {
    const int64_t item = next_item(A.W, &own, lane);
    if (item >= A.W.nwaves) break;
    knn_item<KC, true, FL, SCHED>(A, item_of(A.W, item), lane, seg);
  }
}

// ---------------------------------------------------------------- host side
// Launch geometry: one wave per work item, or for persistent launches one
// block per 4 waves up to 32 waves per CU of a 256-CU part.
static Waves make_waves(chs_index ix, const QueryPlan& plan, int32_t* counter) {
  Waves W;
  W.q4 = plan.q;
  W.nq = plan.nq;
  W.nwaves = plan.nwaves;
  W.wave_tile = plan.wave_tile;
  W.wave_start = plan.wave_start;
  W.tile_qend = plan.tile_qend;
  W.tiles = ix->tiles_d;
  W.counter = counter;
  return W;
}

// per-item tile lookups and persistent waves are needed by batched indexes
// and by the persistent option; a plain index uses the lighter kernels
static bool multi(chs_index ix) { return ix->ntiles > 1 || ix->persistent; }

// ctr: the call's own work counter (persistent launches), so that searches
// in flight on different streams never share one.
static chs_status launch_dims(chs_index ix, const QueryPlan& plan, hipStream_t st, Buf* ctr,
                              int32_t** counter, unsigned* nblocks) {
  const int64_t nb = (plan.nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
  *counter = nullptr;
  *nblocks = (unsigned)(nb > 0 ? nb : 1);
  if (ix->persistent) {
    CHS_TRY(ctr->alloc(sizeof(int32_t)));
    k_reset_counter<<<1, kWave, 0, st>>>(ctr->as<int32_t>());
    CHS_LAUNCH_CHECK();
    *counter = ctr->as<int32_t>();
    const int64_t cap = 256 * 8;
    *nblocks = (unsigned)(nb < cap ? (nb > 0 ? nb : 1) : cap);
  }
  return CHS_OK;
}

// kernel instance for the index's flavor, launch mode, search kernel and
// (fill) stage size
template <bool FILL, int KS, int ST>
static void launch_radius_ks(chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A) {
  const bool mt = multi(ix);
  switch (ix->flavor) {
    case CHS_DENSE:
      mt ? k_radius<FILL, true, CHS_DENSE, KS, ST><<<nb, kThreads, 0, st>>>(A)
         : k_radius<FILL, false, CHS_DENSE, KS, ST><<<nb, kThreads, 0, st>>>(A);
      break;
    case CHS_SPARSE:
      mt ? k_radius<FILL, true, CHS_SPARSE, KS, ST><<<nb, kThreads, 0, st>>>(A)
         : k_radius<FILL, false, CHS_SPARSE, KS, ST><<<nb, kThreads, 0, st>>>(A);
      break;
    default:
      mt ? k_radius<FILL, true, CHS_MIXED, KS, ST><<<nb, kThreads, 0, st>>>(A)
         : k_radius<FILL, false, CHS_MIXED, KS, ST><<<nb, kThreads, 0, st>>>(A);
  }
}

template <bool FILL, int ST>
static void launch_radius_st(chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A,
                             int32_t kernel) {
  if (kernel == CHS_KERNEL_CUBE) launch_radius_ks<FILL, kCube, ST>(ix, nb, st, A);
  else if (kernel == CHS_KERNEL_CYLINDER) launch_radius_ks<FILL, kCylinder, ST>(ix, nb, st, A);
  else launch_radius_ks<FILL, kSphere, ST>(ix, nb, st, A);
}

// mean_rows: the fill's mean row length (neighbours per query)
template <bool FILL>
static void launch_radius(chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A,
                          int32_t kernel, int64_t mean_rows = 0) {
  if constexpr (FILL) {
    if (ix->fill_stage == kStageShort) {
      launch_radius_st<FILL, kStageShort>(ix, nb, st, A, kernel);
      return;
    }
    if (ix->fill_stage == kStageMid) {
      launch_radius_st<FILL, kStageMid>(ix, nb, st, A, kernel);
      return;
    }
    if (mean_rows >= kLongRows || ix->fill_stage == kStageLong) {
      launch_radius_st<FILL, kStageLong>(ix, nb, st, A, kernel);
      return;
    }
    if (mean_rows >= kMidRows) {
      launch_radius_st<FILL, kStageMid>(ix, nb, st, A, kernel);
      return;
    }
  }
  launch_radius_st<FILL, kStageShort>(ix, nb, st, A, kernel);
}

template <int KC, int SCHED>
static void launch_knn_s(chs_index ix, unsigned nb, hipStream_t st, const KnnArgs& A) {
  const bool mt = multi(ix);
  switch (ix->flavor) {
    case CHS_DENSE:
      mt ? k_knn<KC, true, CHS_DENSE, SCHED><<<nb, kThreads, 0, st>>>(A)
         : k_knn<KC, false, CHS_DENSE, SCHED><<<nb, kThreads, 0, st>>>(A);
      break;
    case CHS_SPARSE:
      mt ? k_knn<KC, true, CHS_SPARSE, SCHED><<<nb, kThreads, 0, st>>>(A)
         : k_knn<KC, false, CHS_SPARSE, SCHED><<<nb, kThreads, 0, st>>>(A);
      break;
    default:
      mt ? k_knn<KC, true, CHS_MIXED, SCHED><<<nb, kThreads, 0, st>>>(A)
         : k_knn<KC, false, CHS_MIXED, SCHED><<<nb, kThreads, 0, st>>>(A);
  }
}

template <int KC>
static void launch_knn(chs_index ix, unsigned nb, hipStream_t st, const KnnArgs& A) {
  if (ix->knn_density) launch_knn_s<KC, kDensity>(ix, nb, st, A);
  else launch_knn_s<KC, kRings>(ix, nb, st, A);
}

static chs_status radius_count_impl(chs_index ix, const QueryPlan& plan, int32_t kernel, float r,
                                    int64_t* offsets, hipStream_t st) {
  Alloc al = ix->al;
  al.stream = st;
  const int64_t nq = plan.nq;
  Buf counts(&al);
  CHS_TRY(counts.alloc(sizeof(int32_t) * (nq > 0 ? nq : 1)));
  if (nq > 0) {
    Buf cbuf(&al);
    int32_t* ctr;
    unsigned nb;
    CHS_TRY(launch_dims(ix, plan, st, &cbuf, &ctr, &nb));
    RadiusArgs A{make_waves(ix, plan, ctr), ix->grid(), ix->pts, ix->voxels(), r,
                 counts.as<int32_t>(), nullptr, nullptr, 0};
    launch_radius<false>(ix, nb, st, A, kernel);
    CHS_LAUNCH_CHECK();
  }
  CHS_TRY(exclusive_scan_i32_i64(al, counts.as<int32_t>(), offsets, nq));
  return CHS_OK;
}

static chs_status radius_fill_impl(chs_index ix, const QueryPlan& plan, int32_t kernel, float r,
                                   const int64_t* offsets, int32_t* nbr, int64_t total,
                                   hipStream_t st) {
  if (plan.nq == 0) return CHS_OK;
  Alloc al = ix->al;
  al.stream = st;
  Buf cbuf(&al);
  int32_t* ctr;
  unsigned nb;
  CHS_TRY(launch_dims(ix, plan, st, &cbuf, &ctr, &nb));
  RadiusArgs A{make_waves(ix, plan, ctr), ix->grid(), ix->pts, ix->voxels(), r, nullptr,
               offsets, nbr, total};
  launch_radius<true>(ix, nb, st, A, kernel, total / plan.nq);
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}

static chs_status check_r(float r) {
  if (!(r >= 0.0f) || !std::isfinite(r)) {
    set_error("radius must be finite and >= 0");
    return CHS_E_INVALID;
  }
  return CHS_OK;
}

static chs_status check_kernel(int32_t kernel) {
  if (kernel != CHS_KERNEL_SPHERE && kernel != CHS_KERNEL_CUBE && kernel != CHS_KERNEL_CYLINDER) {
    set_error("unknown search kernel %d", kernel);
    return CHS_E_INVALID;
  }
  return CHS_OK;
}

chs_status knn_impl(chs_index ix, const chs_queries* qs, int32_t k, float r_max,
                           int32_t* idx, float* d2, const Alloc& al, hipStream_t st) {
  CHS_TRY(check_queries(ix, qs));
  if (k < 1 || k > 64) {
    set_error("k = %d outside [1, 64]", k);
    return CHS_E_INVALID;
  }
  if (std::isnan(r_max) || r_max < 0.0f) {
    set_error("r_max must be >= 0 or +inf");
    return CHS_E_INVALID;
  }
  if (qs->nq > 0 && (!idx || !d2)) {
    set_error("idx or d2 is NULL");
    return CHS_E_INVALID;
  }
  if (qs->nq == 0) return CHS_OK;
  QueryPlan plan(&al);
  CHS_TRY(plan_queries(ix, qs, &plan, st));
  const float rmax2 = std::isinf(r_max) ? INFINITY : r_max * r_max;
  Buf cbuf(&al);
  int32_t* ctr;
  unsigned nb;
  CHS_TRY(launch_dims(ix, plan, st, &cbuf, &ctr, &nb));
  KnnArgs A{make_waves(ix, plan, ctr), ix->grid(), ix->pts, ix->voxels(), k, rmax2, idx, d2};
  if (k <= 8)
    launch_knn<8>(ix, nb, st, A);
  else if (k <= 16)
    launch_knn<16>(ix, nb, st, A);
  else if (k <= 32)
    launch_knn<32>(ix, nb, st, A);
  else
    launch_knn<64>(ix, nb, st, A);
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}

}  // namespace chs

using namespace chs;


extern "C" chs_status chs_kernel_count(chs_index ix, const chs_queries* qs, int32_t kernel,
                                       float r, int64_t* offsets, int64_t* total, hipStream_t st) {
  clear_error();
  CHS_TRY(check_queries(ix, qs));
  CHS_TRY(check_kernel(kernel));
  CHS_TRY(check_r(r));
  if (!offsets || !total) {
    set_error("offsets or total is NULL");
    return CHS_E_INVALID;
  }
  Alloc al = ix->al;
  al.stream = st;
  QueryPlan plan(&al);
  CHS_TRY(plan_queries(ix, qs, &plan, st));
  CHS_TRY(radius_count_impl(ix, plan, kernel, r, offsets, st));
  int64_t tot = 0;
  CHS_HIP(hipMemcpyAsync(&tot, offsets + qs->nq, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  CHS_HIP(hipStreamSynchronize(st));
  *total = tot;
  return CHS_OK;
}

extern "C" chs_status chs_kernel_fill(chs_index ix, const chs_queries* qs, int32_t kernel,
                                      float r, const int64_t* offsets, int32_t* nbr, int64_t total,
                                      hipStream_t st) {
  clear_error();
  CHS_TRY(check_queries(ix, qs));
  CHS_TRY(check_kernel(kernel));
  CHS_TRY(check_r(r));
  if (!offsets || (total > 0 && !nbr) || total < 0) {
    set_error("offsets or nbr is NULL, or total < 0");
    return CHS_E_INVALID;
  }
  Alloc al = ix->al;
  al.stream = st;
  QueryPlan plan(&al);
  CHS_TRY(plan_queries(ix, qs, &plan, st));
  CHS_TRY(radius_fill_impl(ix, plan, kernel, r, offsets, nbr, total, st));
  return CHS_OK;
}

extern "C" chs_status chs_kernel_search(chs_index ix, const chs_queries* qs, int32_t kernel,
                                        float r, const chs_allocator* alloc, int64_t* offsets,
                                        int32_t** nbr, int64_t* total, hipStream_t st) {
  clear_error();
  CHS_TRY(check_queries(ix, qs));
  CHS_TRY(check_kernel(kernel));
  CHS_TRY(check_r(r));
  if (!offsets || !nbr || !total) {
    set_error("offsets, nbr or total is NULL");
    return CHS_E_INVALID;
  }
  if (alloc && (!alloc->alloc || !alloc->free)) {
    set_error("allocator callbacks are NULL");
    return CHS_E_INVALID;
  }
  Alloc al = ix->al;
  al.stream = st;
  Alloc out_al = al;
  if (alloc) {
    out_al.a = *alloc;
    out_al.has = true;
  }
  QueryPlan plan(&al);
  CHS_TRY(plan_queries(ix, qs, &plan, st));
  CHS_TRY(radius_count_impl(ix, plan, kernel, r, offsets, st));
  int64_t tot = 0;
  CHS_HIP(hipMemcpyAsync(&tot, offsets + qs->nq, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  CHS_HIP(hipStreamSynchronize(st));
  int32_t* out = nullptr;
  if (tot > 0) {
    out = static_cast<int32_t*>(out_al.get(sizeof(int32_t) * (size_t)tot));
    if (!out) {
      set_error("allocator returned NULL for %lld neighbour indices", (long long)tot);
      return CHS_E_NOMEM;
    }
    chs_status s = radius_fill_impl(ix, plan, kernel, r, offsets, out, tot, st);
    if (s != CHS_OK) {
      out_al.put(out);
      return s;
    }
  }
  *nbr = out;
  *total = tot;
  return CHS_OK;
}

// The sphere entry points of Alg. 1 (Section 3.4.1).
extern "C" chs_status chs_radius_count(chs_index ix, const chs_queries* qs, float r,
                                       int64_t* offsets, int64_t* total, hipStream_t st) {
  return chs_kernel_count(ix, qs, CHS_KERNEL_SPHERE, r, offsets, total, st);
}

extern "C" chs_status chs_radius_fill(chs_index ix, const chs_queries* qs, float r,
                                      const int64_t* offsets, int32_t* nbr, int64_t total,
                                      hipStream_t st) {
  return chs_kernel_fill(ix, qs, CHS_KERNEL_SPHERE, r, offsets, nbr, total, st);
}

extern "C" chs_status chs_radius_search(chs_index ix, const chs_queries* qs, float r,
                                        const chs_allocator* alloc, int64_t* offsets,
                                        int32_t** nbr, int64_t* total, hipStream_t st) {
  return chs_kernel_search(ix, qs, CHS_KERNEL_SPHERE, r, alloc, offsets, nbr, total, st);
}

extern "C" chs_status chs_knn(chs_index ix, const chs_queries* qs, int32_t k, float r_max,
                              int32_t* idx, float* d2, hipStream_t st) {
  clear_error();
  if (!ix) {
    set_error("index is NULL");
    return CHS_E_INVALID;
  }
  Alloc al = ix->al;
  al.stream = st;
  return knn_impl(ix, qs, k, r_max, idx, d2, al, st);
}
