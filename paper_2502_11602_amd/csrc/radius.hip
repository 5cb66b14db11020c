// The kernel-based search of Section 3.4.1 (Alg. 1) on the GPU, with the
// sphere, the cube and the cylinder of Section 2, in two schedules:
//
// tiles   a wave owns 64 queries consecutive in the Hilbert order and streams
//         the points of its union voxel box column by column through the
//         scalar unit, every candidate tested against the 64 queries held in
//         the lanes; the fill stages each lane's matches in LDS and writes
//         them as contiguous row pieces;
// groups  the wave takes its 64 queries 8 at a time, packs the candidate runs
//         of the group's own voxel box into one list, loads 64 candidates per
//         step (one per lane) and tests them against each query of the group
//         (wave-uniform), compacting matches with a ballot.
//
// Both test the unfused FP32 distance of the definitions; the host picks the
// schedule from the radius in voxel edges (groups pay off once a query's
// kernel box spans several columns per axis).
#include "search_common.h"

#pragma clang fp contract(off)

namespace chs {

// ---------------------------------------------------------------- 64-query tiles
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
  static constexpr int min_flush = ST <= 16 ? 6 : (ST <= 24 ? 10 : (ST <= 32 ? 12 : 32));
  static constexpr int pieces = (ST + 31) / 32;  // 32-entry pieces of a run (half-wave stores)
  static_assert(min_flush <= ST - kGroup, "a kept run must leave room for a group");
};
constexpr int kStageShort = 16, kStageMid = 24, kStageLong = 32, kStageHuge = 64;
// mean row lengths (neighbours per query) from which the fill takes the
// middle, the long and the huge stage (the huge one leaves two waves per
// SIMD, which pays only for rows of thousands of entries: TLS scan at
// 0.5 m, 76 k per row, 2.05 -> 1.89 s)
constexpr int64_t kMidRows = 64, kLongRows = 256, kHugeRows = 8192;
// Mean row length from which the flushes use non-temporal stores: with rows
// of thousands of entries the output streams through L2 and, stored
// normally, evicts the candidates the tiles re-read (TLS scan: 0.1 m fill
// 147 -> 132 ms, 0.25 m 379 -> 315 ms, 0.5 m 1888 -> 1568 ms); with short
// rows it is slower (ALS tile: r = 1 m 1.58 -> 1.67 ms).
constexpr int64_t kStreamRows = 2048;

// Where a lane's staged entries go: the row position and how many of them
// are written (published once per flush, read by the half-waves).
struct alignas(16) RowSlot {
  int64_t pos;
  int32_t cnt, pad_;
};

// FINAL: the lane's last flush, everything staged is written.
template <bool FINAL, int ST, bool NT>
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
    constexpr int PC = Stage<ST>::pieces;
    RowSlot r[kFlushUnroll];
    int32_t v[kFlushUnroll][PC];
#pragma unroll
    for (int u = 0; u < kFlushUnroll; ++u) {
      r[u] = rows[src[u]];
#pragma unroll
      for (int p = 0; p < PC; ++p)
        v[u][p] = seg_base[src[u] * Stage<ST>::stride + (32 * p + i < ST ? 32 * p + i : 0)];
    }
    // keep the reads ahead of every store (the compiler would otherwise sink
    // some of them into the stores' branches, one LDS round trip each)
#pragma unroll
    for (int u = 0; u < kFlushUnroll; ++u) {
      asm volatile("" ::"v"(r[u].pos), "v"(r[u].cnt));
#pragma unroll
      for (int p = 0; p < PC; ++p) asm volatile("" ::"v"(v[u][p]));
    }
#pragma unroll
    for (int u = 0; u < kFlushUnroll; ++u)
#pragma unroll
      for (int p = 0; p < PC; ++p)
        if (ok[u] && 32 * p + i < r[u].cnt) {
          if (NT) __builtin_nontemporal_store(v[u][p], &nbr[r[u].pos + 32 * p + i]);
          else nbr[r[u].pos + 32 * p + i] = v[u][p];
        }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  wpos += used;
  nb -= used;
}

template <bool FILL, bool MULTI, int FL, int KS, int ST, bool NT, int CL>
__device__ __forceinline__ void radius_tile_item(const RadiusArgs& A, const Item& it, int lane,
                                            int32_t* seg_base, RowSlot* rows, int64_t wid) {
  const Grid g = MULTI ? A.W.tiles[it.tile] : A.g0;
  const int64_t t = it.t0 + lane;
  const bool in = t < it.tend;
  const float4 q = in ? A.W.q4[t] : make_float4(0.f, 0.f, 0.f, __uint_as_float(kInactive));
  const uint32_t wq = __float_as_uint(q.w);
  const uint32_t qid = wq & ~kInactive;
  const bool active = in && !(wq & kInactive) && (int64_t)qid < A.W.nq;
  const double pad = fmax((double)A.r * (1.0 + kPadRel), kPadAbs);
  const int32_t poff = (int32_t)g.poff;
  int32_t cnt = 0;
  int64_t wpos = 0, wend = 0;
  int nb = 0;
  int32_t* my_seg = seg_base + (FILL ? lane * Stage<ST>::stride : 0);
  if (FILL && active) {
    // rows start at offsets[q] - offsets[0] (a range of a larger counted
    // set fills its own buffer) and are clipped to nbr's extent: offsets
    // that do not belong to these queries and this r write nothing outside
    // [0, total)
    const int64_t base = A.offsets[0];
    wpos = A.offsets[qid] - base;
    wend = A.offsets[qid + 1] - base;
    if (wend > A.total) wend = A.total;
    if (wpos < 0 || wpos > wend) wpos = wend = 0;
  }
  // one search over the lanes with act set: fl32(r*r); the other lanes, and
  // lanes without a valid query, get negative bounds so that no candidate
  // (D >= 0, |d| >= 0, or NaN) ever matches for them and they write nothing
  auto pass = [&](const bool act) __attribute__((always_inline)) {
  const Tile tb = tile_bounds(q, act);
  const float R = act ? A.r * A.r : -1.0f;
  const float rr = act ? A.r : -1.0f;
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
              if (__ballot(nb > ST - kGroup)) flush_stage<false, ST, NT>(seg_base, rows, lane, nb, wpos, wend, A.nbr);
            }
            for (; p < re; ++p) {
              const float4 P = load_const(cp, p);
              my_seg[nb] = __float_as_int(P.w) - poff;
              nb += inside<KS>(q, P, rr, R) ? 1 : 0;
              if (__ballot(nb > ST - kGroup)) flush_stage<false, ST, NT>(seg_base, rows, lane, nb, wpos, wend, A.nbr);
            }
          }
        }
      }
    }
  }
  };
  const uint64_t all = __ballot(active);
  if (CL == kClAll) {
    pass(active);
  } else if (CL == kClCompact) {
    const float qc[3] = {q.x, q.y, q.z};
    if (all && !lanes_compact(all, g, qc, lane) && lane_cluster(all, g, qc, lane) != all) {
      // left to the second launch, which writes this item's counts or rows
      if (lane == 0) {
        const int32_t at = atomicAdd(A.split, 1);
        A.split[1 + at] = (int32_t)wid;
      }
      return;
    }
    pass(active);
  } else {
    const float qc[3] = {q.x, q.y, q.z};
    uint64_t todo = all;
    while (todo) {
      const uint64_t cm = lane_cluster(todo, g, qc, lane);
      todo &= ~cm;
      pass(active && ((cm >> lane) & 1ull));
    }
  }
  if (FILL) flush_stage<true, ST, NT>(seg_base, rows, lane, nb, wpos, wend, A.nbr);
  if (!FILL && in && (int64_t)qid < A.W.nq) A.counts[qid] = active ? cnt : 0;
}

// MULTI: per-item tile lookups and, if a counter is given, a persistent
// loop over work items; otherwise one wave per item with tile 0's grid.
// ST: entries per lane of the fill's stage (unused by the count pass)
template <bool FILL, bool MULTI, int FL, int KS, int ST, bool NT, int CL>
__global__ __launch_bounds__(kThreads) void k_radius_tile(RadiusArgs A) {
  static_assert(!MULTI || CL == kClAll, "persistent waves search every item with one box");
  __shared__ int32_t s_stage[FILL ? kWavesPerBlock * kWave * Stage<ST>::stride : 1];
  __shared__ RowSlot s_rows[FILL ? kWavesPerBlock * kWave : 1];
  const int w = threadIdx.x / kWave, lane = lane_id();
  int32_t* seg_base = s_stage + (FILL ? w * kWave * Stage<ST>::stride : 0);
  RowSlot* rows = s_rows + (FILL ? w * kWave : 0);
  int64_t own = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + w;
  if (!MULTI) {
    if (CL == kClSplit) {
      // the listed items (written by the previous launch on this stream)
      const int64_t cnt = uniform(A.split[0]);
      const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
      for (int64_t i = own; i < cnt; i += stride) {
        const int64_t wv = uniform(A.split[1 + i]);
        radius_tile_item<FILL, false, FL, KS, ST, NT, CL>(A, item_of(A.W, wv), lane, seg_base,
                                                          rows, wv);
      }
      return;
    }
    if (own < A.W.nwaves)
      radius_tile_item<FILL, false, FL, KS, ST, NT, CL>(A, item_of(A.W, own), lane, seg_base, rows,
                                                        own);
    return;
  }
  while (true) {
    const int64_t item = next_item(A.W, &own, lane);
    if (item >= A.W.nwaves) break;
    radius_tile_item<FILL, true, FL, KS, ST, NT, kClAll>(A, item_of(A.W, item), lane, seg_base,
                                                         rows, item);
  }
}

// ---------------------------------------------------------------- 8-query groups
// Query groups.  A work item (at most 64 queries, consecutive in the
// Hilbert order) is taken kQGroup queries at a time.  The candidates of a
// group are the points of the columns of its voxel box (the union of the
// group's kernel boxes), each column cut to the z voxels that can hold a
// point within r of the group's bounding box.  The wave packs the runs of
// up to 64 columns (one per lane) into one list in LDS (a lane prefix sum
// gives each run its place) and walks the list 64 candidates at a time, one
// per lane (vector loads of nearby points).  Every candidate is then tested
// against each query of the group, whose centre is wave-uniform, so one test
// instruction covers 64 (query, candidate) pairs of nearby points.  The
// count pass adds up the ballot of each test; the fill pass compacts each
// test's matches with a lane prefix count of the ballot and writes them as
// one contiguous piece of the query's row.
constexpr int kQGroup = 8;
constexpr int kCandCap = 1024;       // packed candidates per wave in LDS

// Lane's rank among the set lanes of m below it.
__device__ __forceinline__ int32_t lane_rank(uint64_t m) {
  return (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Voxel bounds of query boxes from a precomputed inverse edge: never above
// (lo) or below (hi) the voxel floor(v / s) of any value v in the box (the
// margin dwarfs the rounding of v * (1/s) against an IEEE v / s), so a box
// may take one voxel more than needed, never one less.
__device__ __forceinline__ double vfloor_lo(double v, double inv) {
  const double t = v * inv;
  return floor(t - (fabs(t) * 0x1p-40 + 0x1p-40));
}
__device__ __forceinline__ double vfloor_hi(double v, double inv) {
  const double t = v * inv;
  return floor(t + (fabs(t) * 0x1p-40 + 0x1p-40));
}

typedef const int64_t __attribute__((address_space(4)))* const_i64;
typedef int32_t __attribute__((address_space(1)))* global_i32;

// The column test of a query group in FP32.  The column's footprint is
// widened by 2^-20 of its coordinates plus 2^-20 of an edge, far above the
// FP32 rounding of its bounds, so the horizontal distance d to the group's
// box is never overestimated; the padded radius (2^-18 above r) leaves room
// for the rounding of d*d, so a column is dropped only when no point of it
// can pass the FP32 test.  hz bounds the height difference between such a
// point and the box's z range (sqrt(pad^2 - d^2), widened by 2^-16 of itself
// and of the padded radius for the FP32 square root and the z bounds).
__device__ __forceinline__ bool column_near32(float s0, float s1, const Tile& t, int32_t i,
                                              int32_t j, float pad, float* hz) {
  const float x0 = (float)i * s0, x1 = (float)(i + 1) * s0;
  const float y0 = (float)j * s1, y1 = (float)(j + 1) * s1;
  const float ex = (fabsf(x1) + s0) * 0x1p-20f, ey = (fabsf(y1) + s1) * 0x1p-20f;
  const float dx = fmaxf(0.f, fmaxf((x0 - ex) - t.hi[0], t.lo[0] - (x1 + ex)));
  const float dy = fmaxf(0.f, fmaxf((y0 - ey) - t.hi[1], t.lo[1] - (y1 + ey)));
  const float h2 = pad * pad - (dx * dx + dy * dy);
  *hz = (h2 > 0.f ? __builtin_sqrtf(h2) * (1.f + 0x1p-16f) : 0.f) + pad * 0x1p-16f;
  return h2 >= 0.f;
}

// Voxel bounds in FP32 from the inverse edge, widened by 2^-20 (relative and
// absolute) against the FP32 rounding: never above (lo) or below (hi) the
// voxel floor(v / s) of a value in range.
__device__ __forceinline__ float vfloor32_lo(float v, float inv) {
  const float t = v * inv;
  return floorf(t - (fabsf(t) * 0x1p-20f + 0x1p-20f));
}
__device__ __forceinline__ float vfloor32_hi(float v, float inv) {
  const float t = v * inv;
  return floorf(t + (fabsf(t) * 0x1p-20f + 0x1p-20f));
}

template <bool FILL, bool MULTI, int FL, int KS>
__device__ __forceinline__ void radius_group_item(const RadiusArgs& A, const Item& it, int lane,
                                                  int32_t* s_cand) {
  const Grid g = MULTI ? A.W.tiles[it.tile] : A.g0;
  const const_pts cq = as_const(A.W.q4);
  const float R = A.r * A.r;  // fl32(r*r)
  const float rr = A.r;
  const double pad = fmax((double)A.r * (1.0 + kPadRel), kPadAbs);
  const float padf = (float)pad;
  const int32_t poff = (int32_t)g.poff;
  const double inv[3] = {1.0 / g.s[0], 1.0 / g.s[1], 1.0 / g.s[2]};
  const float s0f = (float)g.s[0], s1f = (float)g.s[1], inv2f = (float)inv[2];
  // the item's queries, one per lane; lanes 8j .. 8j+7 form group j
  const int64_t t = it.t0 + lane;
  const bool in = t < it.tend;
  const float4 q = in ? A.W.q4[t] : make_float4(0.f, 0.f, 0.f, __uint_as_float(kInactive));
  const uint32_t wq = __float_as_uint(q.w);
  const bool active = in && !(wq & kInactive) && (int64_t)wq < A.W.nq;
  // each group's bounding box and voxel box, computed by all its lanes
  float lo[3] = {active ? q.x : INFINITY, active ? q.y : INFINITY, active ? q.z : INFINITY};
  float hi[3] = {active ? q.x : -INFINITY, active ? q.y : -INFINITY, active ? q.z : -INFINITY};
#pragma unroll
  for (int m = 1; m < kQGroup; m <<= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], m, kWave));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], m, kWave));
    }
  int32_t blo[3], bhi[3];
  bool bempty = !(lo[0] <= hi[0]);  // no active query in the group
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    blo[a] = bhi[a] = 0;
    if (a >= g.dims) continue;
    if (KS == kCylinder && a == 2) {
      bhi[2] = (int32_t)(g.n[2] - 1);
      continue;
    }
    const double clo = vfloor_lo((double)lo[a] - pad, inv[a]);
    const double chi = vfloor_hi((double)hi[a] + pad, inv[a]);
    if (!(chi >= 0.0 && clo <= (double)(g.n[a] - 1))) bempty = true;
    blo[a] = clo < 0.0 ? 0 : (int32_t)clo;
    bhi[a] = chi > (double)(g.n[a] - 1) ? (int32_t)(g.n[a] - 1) : (int32_t)chi;
  }
  int32_t mycnt = 0;
  const int ngroups = (int)((it.tend - it.t0 + kQGroup - 1) / kQGroup);
  for (int gi = 0; gi < ngroups; ++gi) {
    const int src = gi * kQGroup;
    if (__builtin_amdgcn_readlane((int32_t)bempty, src)) continue;
    Tile tb;
    int32_t glo[3], ghi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      tb.lo[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lo[a]), src));
      tb.hi[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hi[a]), src));
      glo[a] = __builtin_amdgcn_readlane(blo[a], src);
      ghi[a] = __builtin_amdgcn_readlane(bhi[a], src);
    }
    // the group's queries, wave-uniform (scalar registers); the fill keeps
    // each query's next row slot and the room left in its row
    const int64_t g0 = it.t0 + src;
    const int ng = (int)(it.tend - g0 < kQGroup ? it.tend - g0 : kQGroup);
    float qx[kQGroup], qy[kQGroup], qz[kQGroup];
    bool qa[kQGroup];
    int32_t cnt[kQGroup];
    global_i32 row[kQGroup];   // fill: the query's row
    int32_t rlen[kQGroup];     //   its length (clipped to nbr)
    int32_t wcnt[kQGroup];     //   entries found so far
#pragma unroll
    for (int j = 0; j < kQGroup; ++j) {
      qa[j] = false;
      // a query without a valid centre gets NaN coordinates: every test
      // fails and it takes no further work
      qx[j] = qy[j] = qz[j] = __builtin_nanf("");
      cnt[j] = 0;
      row[j] = (global_i32)A.nbr;
      rlen[j] = 0;
      wcnt[j] = 0;
      if (j < ng) {
        const float4 c = load_const(cq, (int32_t)(g0 + j));
        const uint32_t w = __float_as_uint(c.w);
        qa[j] = !(w & kInactive) && (int64_t)w < A.W.nq;
        if (qa[j]) {
          qx[j] = c.x;
          qy[j] = c.y;
          qz[j] = c.z;
        }
        if (FILL) {
          // the fill keeps the centres in vector registers (same value in
          // every lane), leaving the scalar registers to the row cursors
          asm volatile("v_mov_b32 %0, %1" : "=v"(qx[j]) : "s"(qx[j]));
          asm volatile("v_mov_b32 %0, %1" : "=v"(qy[j]) : "s"(qy[j]));
          asm volatile("v_mov_b32 %0, %1" : "=v"(qz[j]) : "s"(qz[j]));
        }
        if (FILL && qa[j]) {
          // rows start at offsets[q] - offsets[0] and are clipped to nbr's
          // extent: offsets that do not belong to these queries and this r
          // write nothing outside [0, total); a row holds fewer than 2^31
          // entries (the counts are int32)
          const const_i64 co = (const_i64)A.offsets;
          int64_t rb = co[w] - co[0], re = co[w + 1] - co[0];
          if (re > A.total) re = A.total;
          if (rb < 0 || rb > re) rb = re = 0;
          row[j] = (global_i32)A.nbr + rb;
          rlen[j] = re - rb > (int64_t)INT32_MAX ? INT32_MAX : (int32_t)(re - rb);
        }
      }
    }
    const int32_t nj = ghi[1] - glo[1] + 1;
    const int32_t ncol = (ghi[0] - glo[0] + 1) * nj;
    const float rnj = 1.0f / (float)nj;
    for (int32_t cb = 0; cb < ncol; cb += kWave) {
      const int32_t c = cb + lane;
      int32_t b = 0, e = 0;
      if (c < ncol) {
        // c / nj without an integer division (c < 2^31, nj < 2^16: the FP32
        // quotient is at most one too small)
        int32_t di = (int32_t)((float)c * rnj);
        int32_t dj = c - di * nj;
        if (dj >= nj) {
          di += 1;
          dj -= nj;
        }
        const int32_t ci = glo[0] + di, cj = glo[1] + dj;
        int32_t k0 = glo[2], k1 = ghi[2];
        float hz;
        // the cube's box already bounds every column it holds
        if (KS == kCube || column_near32(s0f, s1f, tb, ci, cj, padf, &hz)) {
          if (KS == kSphere && g.dims == 3) {
            // a point of this column within r of the group's box lies at
            // most hz above or below it
            const float zl = vfloor32_lo(tb.lo[2] - hz, inv2f);
            const float zh = vfloor32_hi(tb.hi[2] + hz, inv2f);
            if (zl > (float)k0) k0 = (int32_t)zl;
            if (zh < (float)k1) k1 = (int32_t)zh;
          }
          if (k0 <= k1) column_run<FL>(A.vx, g, ci, cj, k0, k1, &b, &e);
        }
      }
      const int32_t len = e - b;
      const int32_t incl = wave_incl_scan(len, lane);
      const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
      for (int32_t p0 = 0; p0 < total; p0 += kCandCap) {
        // this piece of the packed list: every run writes the positions of
        // its candidates that fall in [p0, p0 + kCandCap)
        const int32_t pend = total - p0 < kCandCap ? total : p0 + kCandCap;
        const int32_t at = incl - len;
        const int32_t lo_t = p0 - at > 0 ? p0 - at : 0;
        const int32_t hi_t = pend - at < len ? pend - at : len;
        for (int32_t k = lo_t; k < hi_t; ++k) s_cand[at + k - p0] = b + k;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // two candidates per lane per step (independent loads and tests
        // in flight: r = 3 m count 2.03 -> 1.96 ms, fill 4.34 -> 4.20 ms);
        // per query the first set's matches take their row slots first
        for (int32_t c0 = p0; c0 < pend; c0 += 2 * kWave) {
          const int32_t va = c0 + lane, vb = c0 + kWave + lane;
          const bool valida = va < pend, validb = vb < pend;
          const int32_t posa = valida ? s_cand[va - p0] : 0;
          const int32_t posb = validb ? s_cand[vb - p0] : 0;
          const float4 Pa = A.pts[posa];
          const float4 Pb = A.pts[posb];
          const uint64_t vmaska = __ballot(valida), vmaskb = __ballot(validb);
          const int32_t pida = __float_as_int(Pa.w) - poff, pidb = __float_as_int(Pb.w) - poff;
#pragma unroll
          for (int j = 0; j < kQGroup; ++j) {
            if (j >= ng) break;
            const float4 qj = make_float4(qx[j], qy[j], qz[j], 0.f);
            const bool hita = inside<KS>(qj, Pa, rr, R);
            const bool hitb = inside<KS>(qj, Pb, rr, R);
            const uint64_t ma = __ballot(hita) & vmaska;
            const uint64_t mb = __ballot(hitb) & vmaskb;
            if (!FILL) {
              cnt[j] += __popcll(ma) + __popcll(mb);
            } else {
              if (ma) {
                const int32_t w0 = wcnt[j];
                wcnt[j] = w0 + __popcll(ma);
                const int32_t at = (int32_t)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(ma >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ma, (uint32_t)w0));
                if (hita && valida && at < rlen[j]) row[j][(uint32_t)at] = pida;
              }
              if (mb) {
                const int32_t w0 = wcnt[j];
                wcnt[j] = w0 + __popcll(mb);
                const int32_t at = (int32_t)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, (uint32_t)w0));
                if (hitb && validb && at < rlen[j]) row[j][(uint32_t)at] = pidb;
              }
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    if (!FILL) {
#pragma unroll
      for (int j = 0; j < kQGroup; ++j)
        if (lane == src + j) mycnt = cnt[j];
    }
  }
  // each lane writes its query's count (0 for a query without a valid centre)
  if (!FILL && in && (int64_t)(wq & ~kInactive) < A.W.nq) A.counts[wq & ~kInactive] = active ? mycnt : 0;
}

// MULTI: per-item tile lookups and, if a counter is given, a persistent
// loop over work items; otherwise one wave per item with tile 0's grid.
// Register budgets for more waves per SIMD (measured on the 10 M-point
// tile): the count in 64 VGPRs, eight waves (r = 3 m 2.28 -> 2.02 ms); the
// fill in 72, seven waves (4.56 -> 4.35 ms; held to 64 it spilled 24 bytes
// per lane and read 80 % more from HBM; with two candidates per lane it
// spills 12, and six waves without spilling are slower).
template <bool FILL, bool MULTI, int FL, int KS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(FILL ? 7 : 8))) void k_radius_group(RadiusArgs A) {
  __shared__ int32_t s_cand[kWavesPerBlock * kCandCap];
  const int w = threadIdx.x / kWave, lane = lane_id();
  // (the wave index is uniform: keep the item and its queries in scalar
  // registers)
  int64_t own = first_lane((int64_t)xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + w);
  if (!MULTI) {
    if (own < A.W.nwaves)
      radius_group_item<FILL, false, FL, KS>(A, item_of(A.W, own), lane, s_cand + w * kCandCap);
    return;
  }
  while (true) {
    const int64_t item = next_item(A.W, &own, lane);
    if (item >= A.W.nwaves) break;
    radius_group_item<FILL, true, FL, KS>(A, item_of(A.W, item), lane, s_cand + w * kCandCap);
  }
}

// ---------------------------------------------------------------- launches
template <bool FILL, int FL, int KS, int ST, bool NT>
static void launch_tile_fl(chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A) {
  // one wave per item: the compact items, then the listed others;
  // persistent waves take every item
  if (multi(ix)) {
    k_radius_tile<FILL, true, FL, KS, ST, NT, kClAll><<<nb, kThreads, 0, st>>>(A);
  } else {
    const unsigned nb2 = nb < kSplitBlocks ? nb : kSplitBlocks;
    k_radius_tile<FILL, false, FL, KS, ST, NT, kClCompact><<<nb, kThreads, 0, st>>>(A);
    k_radius_tile<FILL, false, FL, KS, ST, NT, kClSplit><<<nb2, kThreads, 0, st>>>(A);
  }
}

template <bool FILL, int KS, int ST, bool NT>
static void launch_tile_ks(chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A) {
  switch (ix->flavor) {
    case CHS_DENSE: launch_tile_fl<FILL, CHS_DENSE, KS, ST, NT>(ix, nb, st, A); break;
    case CHS_SPARSE: launch_tile_fl<FILL, CHS_SPARSE, KS, ST, NT>(ix, nb, st, A); break;
    default: launch_tile_fl<FILL, CHS_MIXED, KS, ST, NT>(ix, nb, st, A);
  }
}

template <bool FILL, int ST, bool NT = false>
static void launch_tile_st(chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A,
                           int32_t kernel) {
  if (kernel == CHS_KERNEL_CUBE) launch_tile_ks<FILL, kCube, ST, NT>(ix, nb, st, A);
  else if (kernel == CHS_KERNEL_CYLINDER) launch_tile_ks<FILL, kCylinder, ST, NT>(ix, nb, st, A);
  else launch_tile_ks<FILL, kSphere, ST, NT>(ix, nb, st, A);
}

template <bool FILL>
static void launch_tiles(chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A,
                         int32_t kernel, int64_t mean_rows) {
  if constexpr (FILL) {
    if (ix->fill_stage == kStageShort) {
      launch_tile_st<FILL, kStageShort>(ix, nb, st, A, kernel);
      return;
    }
    if (ix->fill_stage == kStageMid) {
      launch_tile_st<FILL, kStageMid>(ix, nb, st, A, kernel);
      return;
    }
    if (ix->fill_stage == kStageHuge || (ix->fill_stage == 0 && mean_rows >= kHugeRows)) {
      launch_tile_st<FILL, kStageHuge, true>(ix, nb, st, A, kernel);
      return;
    }
    if (ix->fill_stage == 0 && mean_rows >= kStreamRows) {
      launch_tile_st<FILL, kStageLong, true>(ix, nb, st, A, kernel);
      return;
    }
    if (mean_rows >= kLongRows || ix->fill_stage == kStageLong) {
      launch_tile_st<FILL, kStageLong>(ix, nb, st, A, kernel);
      return;
    }
    if (mean_rows >= kMidRows) {
      launch_tile_st<FILL, kStageMid>(ix, nb, st, A, kernel);
      return;
    }
  }
  launch_tile_st<FILL, kStageShort>(ix, nb, st, A, kernel);
}

template <bool FILL, int KS>
static void launch_group_ks(chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A) {
  const bool mt = multi(ix);
  switch (ix->flavor) {
    case CHS_DENSE:
      mt ? k_radius_group<FILL, true, CHS_DENSE, KS><<<nb, kThreads, 0, st>>>(A)
         : k_radius_group<FILL, false, CHS_DENSE, KS><<<nb, kThreads, 0, st>>>(A);
      break;
    case CHS_SPARSE:
      mt ? k_radius_group<FILL, true, CHS_SPARSE, KS><<<nb, kThreads, 0, st>>>(A)
         : k_radius_group<FILL, false, CHS_SPARSE, KS><<<nb, kThreads, 0, st>>>(A);
      break;
    default:
      mt ? k_radius_group<FILL, true, CHS_MIXED, KS><<<nb, kThreads, 0, st>>>(A)
         : k_radius_group<FILL, false, CHS_MIXED, KS><<<nb, kThreads, 0, st>>>(A);
  }
}

template <bool FILL>
static void launch_groups(chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A,
                          int32_t kernel) {
  if (kernel == CHS_KERNEL_CUBE) launch_group_ks<FILL, kCube>(ix, nb, st, A);
  else if (kernel == CHS_KERNEL_CYLINDER) launch_group_ks<FILL, kCylinder>(ix, nb, st, A);
  else launch_group_ks<FILL, kSphere>(ix, nb, st, A);
}

// The schedule of a search: query groups for spheres and cubes whose radius
// spans at least kGroupMinSpan voxel edges (measured on the 10 M-point ALS
// tile: below that the tiles' shared setup wins, above it the groups' tighter
// candidate lists), and for the cylinder, whose full-height columns give the
// groups no cut, tiles.
constexpr double kGroupMinSpan = 1.5;

static int radius_schedule(chs_index ix, int32_t kernel, float r) {
  if (ix->radius_sched != kSchedAuto) return ix->radius_sched;
  if (kernel == CHS_KERNEL_CYLINDER) return kSchedTiles;
  return (double)r >= kGroupMinSpan * ix->cell_xy ? kSchedGroups : kSchedTiles;
}

void launch_radius(bool fill, chs_index ix, unsigned nb, hipStream_t st, const RadiusArgs& A,
                   int32_t kernel, int64_t mean_rows) {
  const bool groups = radius_schedule(ix, kernel, A.r) == kSchedGroups;
  if (fill) {
    if (groups) launch_groups<true>(ix, nb, st, A, kernel);
    else launch_tiles<true>(ix, nb, st, A, kernel, mean_rows);
  } else {
    if (groups) launch_groups<false>(ix, nb, st, A, kernel);
    else launch_tiles<false>(ix, nb, st, A, kernel, mean_rows);
  }
}

}  // namespace chs
