// k-nearest-neighbour search on the GPU (Section 3.4.2, Alg. 2, with the
// taboo box of Section 3.5): a wave owns 64 queries consecutive in the
// Hilbert order, one per lane, and grows a visited voxel box around them,
// either ring by ring or with Alg. 2's density-growth radius; each lane keeps
// its sorted candidate list in registers (Section 3.5, "Candidate list").
#include "search_common.h"

#pragma clang fp contract(off)

namespace chs {

// ---------------------------------------------------------------- k-NN


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
// the radius (with A.monotonic the radius always grows by that edge, the
// baseline Section 3.5 compares density growth with).  The wave visits the
// hull of its unfinished lanes' kernel boxes.  All give the exact k nearest.
constexpr int kRings = 0, kDensity = 1;

__device__ __forceinline__ int64_t box_voxels(const IBox& V, const Grid& g) {
  int64_t c = 1;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a < g.dims) c *= (int64_t)(V.hi[a] - V.lo[a] + 1);
  return c;
}

// One query's own voxels under a growing radius (Alg. 2 run for that query
// alone): the voxels of the padded box of B(c, r), clamped to the grid,
// at the first radius of the schedule, from r on, that holds k keys of
// the (final) sorted list or whose box is the whole grid.
template <int KC>
__device__ int64_t own_voxels(const Grid& g, const float (&qc)[3], double r, double smin,
                              const uint64_t (&best)[KC], int k, bool monotonic) {
  int64_t grid = 1;
  for (int a = 0; a < g.dims; ++a) grid *= g.n[a];
  while (true) {
    const double pad = fmax(r * (1.0 + kPadRel), kPadAbs);
    int64_t c = 1;
    for (int a = 0; a < g.dims; ++a)
      c *= voxel_clamped((double)qc[a] + pad, g.s[a], g.n[a]) -
           voxel_clamped((double)qc[a] - pad, g.s[a], g.n[a]) + 1;
    const uint32_t tb32 = __float_as_uint((float)(r * r));
    int np = 0;
#pragma unroll
    for (int i = 0; i < KC; ++i) np += (uint32_t)(best[i] >> 32) <= tb32 ? 1 : 0;
    if (np >= k || c == grid) return c;
    double rn = r + smin;
    if (np > 0 && !monotonic) {
      const double rd = cbrt((double)k / ((double)np / ((4.0 / 3.0) * M_PI * r * r * r)));
      if (rd > r) rn = rd;
    }
    r = rn;
  }
}


template <int KC, bool MULTI, int FL, int SCHED, bool VIS, int CL>
__device__ __forceinline__ void knn_item(const KnnArgs& A, const Item& it, int lane,
                                         uint64_t* seg, int64_t wid) {
  const Grid g = MULTI ? A.W.tiles[it.tile] : A.g0;
  const int64_t t = it.t0 + lane;
  const bool in = t < it.tend;
  const float4 q = in ? A.W.q4[t] : make_float4(0.f, 0.f, 0.f, __uint_as_float(kInactive));
  const uint32_t wq = __float_as_uint(q.w);
  const uint32_t qid = wq & ~kInactive;
  const bool active = in && !(wq & kInactive) && (int64_t)qid < A.W.nq;
  const const_pts cp = as_const(A.pts);
  uint64_t best[KC];
#pragma unroll
  for (int i = 0; i < KC; ++i) best[i] = ~0ull;
  uint64_t kthk = ~0ull;
  int nb = 0;
  // voxels of the wave's visited box when this lane's list became final,
  // and of the lane's own box (written only when the caller asks for them)
  int64_t vis = -1, own_vis = -1;
  const float qc[3] = {q.x, q.y, q.z};
  // one search over the lanes with act set; the others accept nothing
  auto pass = [&](const bool act) __attribute__((always_inline)) {
    const Tile tb = tile_bounds(q, act);
    const float rmax2 = act ? A.rmax2 : -1.0f;
    // density schedule: the lane's radius, starting at the distance from
    // the query to the nearest wall of its voxel (Eq. 11)
    double rL = 0.0, smin = INFINITY;
    bool done = !act;
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
      if (whole) {
        if (VIS && vis < 0 && act) {
          vis = box_voxels(V, g);
          own_vis = SCHED == kDensity ? own_voxels<KC>(g, qc, rL, smin, best, A.k, A.monotonic)
                                      : vis;
        }
        break;
      }
      if (SCHED == kDensity) {
        // k keys within fl32(rL^2): every unvisited point lies beyond the
        // padded ball of radius rL, so its D exceeds that bound; past the
        // radius cap nothing more can be returned
        const float T = (float)(rL * rL);
        const uint32_t tb32 = __float_as_uint(T);
        done = done || (kthk != ~0ull && (uint32_t)(kthk >> 32) <= tb32) ||
               (double)A.rmax2 <= rL * rL;
        if (VIS && done && vis < 0 && act) {
          vis = box_voxels(V, g);
          own_vis = (double)A.rmax2 <= rL * rL
                        ? own_voxels<KC>(g, qc, rL, smin, best, 0, A.monotonic)
                        : own_voxels<KC>(g, qc, rL, smin, best, A.k, A.monotonic);
        }
        if (__ballot(!done) == 0ull) break;
        if (!done) {
          // |P^|: candidates within the radius (Eq. 10); the list is sorted
          int np = 0;
#pragma unroll
          for (int i = 0; i < KC; ++i) np += (uint32_t)(best[i] >> 32) <= tb32 ? 1 : 0;
          double rn = rL + smin;  // monotonic growth
          if (np > 0 && !A.monotonic) {
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
      done = !act || (lb2 >= 0x1p-100 && (double)thr < lb2 * (1.0 - kPadRel));
      if (VIS && done && vis < 0 && act) vis = own_vis = box_voxels(V, g);
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
  };
  const uint64_t all = __ballot(active);
  if (CL == kClAll) {
    if (all) pass(active);
  } else if (CL == kClCompact) {
    // a wave whose lanes form one cluster searches here with one box
    if (all && !lanes_compact(all, g, qc, lane) && lane_cluster(all, g, qc, lane) != all) {
      // left to the second launch, which writes this item's rows
      if (lane == 0) {
        const int32_t at = atomicAdd(A.split, 1);
        A.split[1 + at] = (int32_t)wid;
      }
      return;
    }
    if (all) pass(active);
  } else {
    uint64_t todo = all;
    while (todo) {
      const uint64_t cm = lane_cluster(todo, g, qc, lane);
      todo &= ~cm;
      pass(active && ((cm >> lane) & 1ull));
    }
  }
  if (VIS && active) {
    A.visited[2 * (int64_t)qid] = own_vis;
    A.visited[2 * (int64_t)qid + 1] = vis;
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
// (measured on the 10 M-point tile).  MODE: 0 = one wave per work item,
// 1 = persistent waves over a batched or persistent index, 2 = as 0 and
// reporting the visited voxels (kept out of the other two, whose registers
// it would cost).
template <int KC, int MODE, int FL, int SCHED, int CL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(KC == 32 ? 4 : (KC == 16 ? 6 : (KC == 8 ? 8 : 1)))))
void k_knn(KnnArgs A) {
  constexpr bool MULTI = MODE == 1, VIS = MODE == 2;
  static_assert(!MULTI || CL == kClAll, "persistent waves search every item with one box");
  constexpr int kSeg = KnnBuf<KC>::on ? kWave * KnnBuf<KC>::stride : 1;
  __shared__ uint64_t s_buf[kWavesPerBlock * kSeg];
  const int w = threadIdx.x / kWave, lane = lane_id();
  uint64_t* seg = s_buf + w * kSeg + (KnnBuf<KC>::on ? lane * KnnBuf<KC>::stride : 0);
  int64_t own = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + w;
  if (!MULTI) {
    if (CL == kClSplit) {
      // the listed items (written by the previous launch on this stream)
      const int64_t cnt = uniform(A.split[0]);
      const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
      for (int64_t i = own; i < cnt; i += stride) {
        const int64_t wv = uniform(A.split[1 + i]);
        knn_item<KC, false, FL, SCHED, VIS, CL>(A, item_of(A.W, wv), lane, seg, wv);
      }
      return;
    }
    if (own < A.W.nwaves)
      knn_item<KC, false, FL, SCHED, VIS, CL>(A, item_of(A.W, own), lane, seg, own);
    return;
  }
  while (true) {
    const int64_t item = next_item(A.W, &own, lane);
    if (item >= A.W.nwaves) break;
    knn_item<KC, true, FL, SCHED, false, kClAll>(A, item_of(A.W, item), lane, seg, item);
  }
}

// ---------------------------------------------------------------- one query at a time
// The solo schedule, for query sets that sample the cloud sparsely: a wave's
// 64 queries are far apart, so the box holding all of them (which the ring
// schedule streams) is mostly empty space between them.  Here the wave takes
// its queries one at a time (centre in scalar registers), grows that query's
// own visited box ring by ring (Alg. 2's taboo box, Section 3.5), packs the
// new shell's column runs into an LDS list and tests 64 candidates per step,
// one per lane.  The query's sorted list lives across the lanes (lane l
// holds its l-th key); accepted candidates enter it by a bitonic sort and
// merge across the lanes, or, when at most 12 are accepted, one by one.
constexpr int kSoloCap = 1024;  // packed candidate positions per wave in LDS

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  const int lo = __shfl((int)(uint32_t)v, src, kWave);
  const int hi = __shfl((int)(uint32_t)(v >> 32), src, kWave);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  const int lo = __shfl_xor((int)(uint32_t)v, m, kWave);
  const int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, kWave);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// The 64 lanes' keys sorted ascending across the lanes (bitonic network).
__device__ __forceinline__ uint64_t lane_sort(uint64_t x, int lane) {
#pragma unroll
  for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
    for (int j = size >> 1; j > 0; j >>= 1) {
      const uint64_t y = shfl_xor64(x, j);
      const bool keep_min = ((lane & j) == 0) == ((lane & size) == 0);
      x = keep_min ? (x < y ? x : y) : (x < y ? y : x);
    }
  }
  return x;
}

// The 64 smallest of two ascending lane lists, ascending: min(L[l], C[63-l])
// is bitonic and holds them; a bitonic merge sorts it.
__device__ __forceinline__ uint64_t lane_merge(uint64_t L, uint64_t C, int lane) {
  const uint64_t cr = shfl64(C, kWave - 1 - lane);
  uint64_t x = L < cr ? L : cr;
#pragma unroll
  for (int j = kWave / 2; j > 0; j >>= 1) {
    const uint64_t y = shfl_xor64(x, j);
    x = (lane & j) == 0 ? (x < y ? x : y) : (x < y ? y : x);
  }
  return x;
}

// Inserts key c (not in L, below L[63]) into the ascending lane list L.
__device__ __forceinline__ uint64_t lane_insert(uint64_t L, uint64_t c, int lane) {
  const int pos = __popcll(__ballot(L < c));
  const uint64_t up = shfl64(L, lane > 0 ? lane - 1 : 0);
  return lane < pos ? L : (lane == pos ? c : up);
}

template <bool MULTI, int FL>
__device__ void knn_solo_item(const KnnArgs& A, const Item& it, int lane, int32_t* s_cand) {
  const Grid g = MULTI ? A.W.tiles[it.tile] : A.g0;
  const int32_t poff = (int32_t)g.poff;
  const const_pts cq = as_const(A.W.q4);
  for (int64_t t = it.t0; t < it.tend; ++t) {
    const float4 q = load_const(cq, (int32_t)t);
    const uint32_t wq = __float_as_uint(q.w);
    const uint32_t qid = wq & ~kInactive;
    if ((int64_t)qid >= A.W.nq) continue;
    const bool active = !(wq & kInactive);
    uint64_t L = ~0ull;  // lane l: the l-th key of the list
    if (active) {
      const float qc[3] = {q.x, q.y, q.z};
      int32_t v[3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        v[a] = a < g.dims ? (int32_t)voxel_clamped((double)qc[a], g.s[a], g.n[a]) : 0;
      IBox V;
      bool vempty = true;
      uint64_t kthk = ~0ull;  // the k-th key (uniform)
      for (int32_t d = 0;; ++d) {
        IBox B;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (a >= g.dims) {
            B.lo[a] = B.hi[a] = 0;
            continue;
          }
          B.lo[a] = v[a] - d > 0 ? v[a] - d : 0;
          B.hi[a] = v[a] + d < g.n[a] - 1 ? v[a] + d : (int32_t)(g.n[a] - 1);
        }
        // the shell B minus V: one column per lane, up to two runs each
        const int32_t nj = B.hi[1] - B.lo[1] + 1;
        const int32_t ncol = (B.hi[0] - B.lo[0] + 1) * nj;
        for (int32_t cb = 0; cb < ncol; cb += kWave) {
          const int32_t c = cb + lane;
          int32_t b0 = 0, e0 = 0, b1 = 0, e1 = 0;
          if (c < ncol) {
            const int32_t ci = B.lo[0] + c / nj, cj = B.lo[1] + c % nj;
            const bool inner = !vempty && ci >= V.lo[0] && ci <= V.hi[0] && cj >= V.lo[1] &&
                               cj <= V.hi[1];
            if (!inner) {
              column_run<FL>(A.vx, g, ci, cj, B.lo[2], B.hi[2], &b0, &e0);
            } else {
              if (B.lo[2] < V.lo[2]) column_run<FL>(A.vx, g, ci, cj, B.lo[2], V.lo[2] - 1, &b0, &e0);
              if (V.hi[2] < B.hi[2]) column_run<FL>(A.vx, g, ci, cj, V.hi[2] + 1, B.hi[2], &b1, &e1);
            }
          }
          const int32_t l0 = e0 - b0, l1 = e1 - b1;
          const int32_t incl = wave_incl_scan(l0 + l1, lane);
          const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
          for (int32_t p0 = 0; p0 < total; p0 += kSoloCap) {
            const int32_t pend = total - p0 < kSoloCap ? total : p0 + kSoloCap;
            const int32_t at = incl - l0 - l1;
            for (int32_t k = 0; k < l0 + l1; ++k) {
              const int32_t x = at + k - p0;
              if (x >= 0 && x < pend - p0) s_cand[x] = k < l0 ? b0 + k : b1 + (k - l0);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int32_t c0 = p0; c0 < pend; c0 += kWave) {
              const int32_t vv = c0 + lane;
              const bool valid = vv < pend;
              const float4 P = A.pts[valid ? s_cand[vv - p0] : 0];
              const float dx = q.x - P.x, dy = q.y - P.y, dz = q.z - P.z;
              const float D = (dx * dx + dy * dy) + dz * dz;
              const uint64_t key =
                  ((uint64_t)__float_as_uint(D) << 32) | (uint64_t)__float_as_uint(P.w);
              const bool acc = valid && D <= A.rmax2 && key < kthk;
              const uint64_t m = __ballot(acc);
              if (m == 0) continue;
              // a few keys one by one (each a dependent shuffle), more by
              // one sort and merge (27 dependent shuffle stages)
              if (__popcll(m) <= 12) {
                uint64_t mm = m;
                while (mm) {
                  const int src = __builtin_ctzll(mm);
                  mm &= mm - 1;
                  const uint64_t ck = readlane64(key, src);
                  if (ck < readlane64(L, kWave - 1)) L = lane_insert(L, ck, lane);
                }
              } else {
                L = lane_merge(L, lane_sort(acc ? key : ~0ull, lane), lane);
              }
              kthk = readlane64(L, A.k - 1);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          }
        }
        V = B;
        vempty = false;
        bool whole = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (a >= g.dims) continue;
          if (V.lo[a] > 0 || V.hi[a] < g.n[a] - 1) whole = false;
        }
        if (whole) break;
        // every point outside V lies beyond the nearest face of V that is
        // not on the grid boundary (as the ring schedule)
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
        if (lb2 >= 0x1p-100 && (double)thr < lb2 * (1.0 - kPadRel)) break;
      }
    }
    if (lane < A.k) {
      const bool ok = L != ~0ull;
      A.idx[(int64_t)qid * A.k + lane] = ok ? (int32_t)(uint32_t)L - poff : -1;
      A.d2[(int64_t)qid * A.k + lane] = ok ? __uint_as_float((uint32_t)(L >> 32)) : INFINITY;
    }
  }
}

template <bool MULTI, int FL>
__global__ __launch_bounds__(kThreads) void k_knn_solo(KnnArgs A) {
  __shared__ int32_t s_cand[kWavesPerBlock * kSoloCap];
  const int w = threadIdx.x / kWave, lane = lane_id();
  int64_t own = first_lane((int64_t)xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + w);
  if (!MULTI) {
    if (own < A.W.nwaves) knn_solo_item<false, FL>(A, item_of(A.W, own), lane, s_cand + w * kSoloCap);
    return;
  }
  while (true) {
    const int64_t item = next_item(A.W, &own, lane);
    if (item >= A.W.nwaves) break;
    knn_solo_item<true, FL>(A, item_of(A.W, item), lane, s_cand + w * kSoloCap);
  }
}

// ---------------------------------------------------------------- launches
template <int KC, int SCHED, int FL>
static void launch_knn_f(chs_index ix, unsigned nb, hipStream_t st, const KnnArgs& A) {
  // one wave per item: the compact items, then the listed others;
  // persistent waves take every item
  const unsigned nb2 = nb < kSplitBlocks ? nb : kSplitBlocks;
  if (multi(ix)) {
    k_knn<KC, 1, FL, SCHED, kClAll><<<nb, kThreads, 0, st>>>(A);
  } else if (A.visited) {
    k_knn<KC, 2, FL, SCHED, kClCompact><<<nb, kThreads, 0, st>>>(A);
    k_knn<KC, 2, FL, SCHED, kClSplit><<<nb2, kThreads, 0, st>>>(A);
  } else {
    k_knn<KC, 0, FL, SCHED, kClCompact><<<nb, kThreads, 0, st>>>(A);
    k_knn<KC, 0, FL, SCHED, kClSplit><<<nb2, kThreads, 0, st>>>(A);
  }
}

template <int KC, int SCHED>
static void launch_knn_s(chs_index ix, unsigned nb, hipStream_t st, const KnnArgs& A) {
  switch (ix->flavor) {
    case CHS_DENSE: launch_knn_f<KC, SCHED, CHS_DENSE>(ix, nb, st, A); break;
    case CHS_SPARSE: launch_knn_f<KC, SCHED, CHS_SPARSE>(ix, nb, st, A); break;
    default: launch_knn_f<KC, SCHED, CHS_MIXED>(ix, nb, st, A);
  }
}

template <int KC>
static void launch_knn_kc(chs_index ix, unsigned nb, hipStream_t st, const KnnArgs& A) {
  if (ix->knn_sched == 0) {
    launch_knn_s<KC, kRings>(ix, nb, st, A);
  } else {
    KnnArgs B = A;
    B.monotonic = ix->knn_sched == 2;
    launch_knn_s<KC, kDensity>(ix, nb, st, B);
  }
}

template <int FL>
static void launch_knn_solo(chs_index ix, unsigned nb, hipStream_t st, const KnnArgs& A) {
  if (multi(ix))
    k_knn_solo<true, FL><<<nb, kThreads, 0, st>>>(A);
  else
    k_knn_solo<false, FL><<<nb, kThreads, 0, st>>>(A);
}

void launch_knn(chs_index ix, unsigned nb, hipStream_t st, const KnnArgs& A) {
  if (ix->knn_sched == 3) {
    switch (ix->flavor) {
      case CHS_DENSE: launch_knn_solo<CHS_DENSE>(ix, nb, st, A); break;
      case CHS_SPARSE: launch_knn_solo<CHS_SPARSE>(ix, nb, st, A); break;
      default: launch_knn_solo<CHS_MIXED>(ix, nb, st, A);
    }
    return;
  }
  if (A.k <= 8)
    launch_knn_kc<8>(ix, nb, st, A);
  else if (A.k <= 16)
    launch_knn_kc<16>(ix, nb, st, A);
  else if (A.k <= 32)
    launch_knn_kc<32>(ix, nb, st, A);
  else
    launch_knn_kc<64>(ix, nb, st, A);
}

}  // namespace chs
