// Query planning and the search entry points of the C ABI: the kernel-based
// search of Section 3.4.1 (Alg. 1: count, offsets, fill) and k-NN (Section
// 3.4.2, Alg. 2).  Queries are put in a Hilbert order over the (i, j) voxel
// columns, then k, so that consecutive queries are spatial neighbours; the
// kernels (radius.hip, knn.hip) take them 64 at a time.
#include <algorithm>
#include <cstring>
#include <cmath>

#include "search_common.h"

#pragma clang fp contract(off)

namespace chs {

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
    const int64_t* __restrict__ qoff, const double* __restrict__ origins, int ntiles, double ox,
    double oy, double oz, int lshift, int total_bits, K* __restrict__ keys,
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
  } else if (mode == 1) {  // point indices (tile-local with per-tile query sets)
    int64_t p = pidx[q], lo = 0, hi = npts;
    if (qoff) {
      t = tile_of_point(qoff, ntiles, q);
      lo = toff[t];
      hi = toff[t + 1];
      p += lo;
    }
    ok = p >= lo && p < hi;
    c = ok ? pts[inv_perm[p]] : make_float4(0.f, 0.f, 0.f, 0.f);
  } else {  // FP64 coordinates (recentred with the query's tile's p-)
    if (qoff) {
      t = tile_of_point(qoff, ntiles, q);
      ox = origins[3 * t];
      oy = origins[3 * t + 1];
      oz = origins[3 * t + 2];
    }
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
  // (lshift reaches 64 only for one tile, rank 0)
  const uint64_t hi_part = lshift >= 64 ? 0ull : ((uint64_t)tp.rank << lshift);
  if (ok) {
    const uint64_t local =
        (hilbert2((uint32_t)cell[0], (uint32_t)cell[1], tp.m) << tp.kbits) | (uint64_t)cell[2];
    key = (K)(hi_part | local);
  } else {
    // last within its tile's range (the tile's waves must hold exactly its
    // queries)
    key = (K)(hi_part | (lshift >= 64 ? ~0ull : ((1ull << lshift) - 1)));
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

// Temporaries come from `al` (on stream st).  q_off (host, ntiles+1): the
// per-tile query sets of index or coordinate queries on a batched index.
static chs_status plan_impl(chs_index ix, int mode, const double* xyz, const int32_t* pidx,
                            int64_t nq, const std::vector<int32_t>& rank, float4* q4,
                            const Alloc& al, hipStream_t st, const int64_t* q_off = nullptr) {
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
  Buf keys(&al), vals(&al), tk(&al), tv(&al), tmp(&al), tp_d(&al), toff_d(&al), qoff_d(&al),
      org_d(&al);
  const bool wide = bits > 32;
  const size_t ks = wide ? 8 : 4;
  CHS_TRY(keys.alloc(ks * nq));
  CHS_TRY(tk.alloc(ks * nq));
  CHS_TRY(vals.alloc(4 * nq));
  CHS_TRY(tv.alloc(4 * nq));
  CHS_TRY(tmp.alloc(sizeof(float4) * nq));
  if (T > 1) {
    // (from the index's own copies, which outlive the queued copies)
    ix->tplan_h.resize(4 * (size_t)T);
    std::memcpy(ix->tplan_h.data(), tp.data(), sizeof(TilePlan) * T);
    CHS_TRY(tp_d.alloc(sizeof(TilePlan) * T));
    CHS_TRY(toff_d.alloc(sizeof(int64_t) * (T + 1)));
    CHS_HIP(hipMemcpyAsync(tp_d.p, ix->tplan_h.data(), sizeof(TilePlan) * T,
                           hipMemcpyHostToDevice, st));
    CHS_HIP(hipMemcpyAsync(toff_d.p, ix->tile_off.data(), sizeof(int64_t) * (T + 1),
                           hipMemcpyHostToDevice, st));
    if (q_off) {
      // (the calls with per-tile query sets wait for the stream before
      // returning, so the caller's array outlives this copy)
      CHS_TRY(qoff_d.alloc(sizeof(int64_t) * (T + 1)));
      CHS_TRY(org_d.alloc(sizeof(double) * 3 * T));
      CHS_HIP(hipMemcpyAsync(qoff_d.p, q_off, sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice, st));
      CHS_HIP(hipMemcpyAsync(org_d.p, ix->origin.data(), sizeof(double) * 3 * T,
                             hipMemcpyHostToDevice, st));
    }
  }
  const double* o = ix->origin.data();
  if (wide) {
    k_plan_keys<uint64_t><<<grid_for(nq), kThreads, 0, st>>>(
        mode, xyz, pidx, nq, ix->pts, ix->inv_perm, ix->perm, ix->n, ix->tiles_d, tp[0],
        tp_d.as<TilePlan>(), toff_d.as<int64_t>(), qoff_d.as<int64_t>(), org_d.as<double>(), T,
        o[0], o[1], o[2], lshift, bits,
        keys.as<uint64_t>(), vals.as<uint32_t>(), tmp.as<float4>());
    CHS_LAUNCH_CHECK();
    CHS_TRY(radix_sort_u64(al, keys.as<uint64_t>(), vals.as<uint32_t>(), tk.as<uint64_t>(),
                           tv.as<uint32_t>(), nq, bits));
  } else {
    k_plan_keys<uint32_t><<<grid_for(nq), kThreads, 0, st>>>(
        mode, xyz, pidx, nq, ix->pts, ix->inv_perm, ix->perm, ix->n, ix->tiles_d, tp[0],
        tp_d.as<TilePlan>(), toff_d.as<int64_t>(), qoff_d.as<int64_t>(), org_d.as<double>(), T,
        o[0], o[1], o[2], lshift, bits,
        keys.as<uint32_t>(), vals.as<uint32_t>(), tmp.as<float4>());
    CHS_LAUNCH_CHECK();
    CHS_TRY(radix_sort_u32(al, keys.as<uint32_t>(), vals.as<uint32_t>(), tk.as<uint32_t>(),
                           tv.as<uint32_t>(), nq, bits));
  }
  k_plan_gather<<<grid_for(nq), kThreads, 0, st>>>(vals.as<uint32_t>(), tmp.as<float4>(), nq, q4);
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}

__global__ __launch_bounds__(kThreads) void k_plan_order(const float4* __restrict__ q4, int64_t nq,
                                                         int32_t* __restrict__ order) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= nq) return;
  order[t] = (int32_t)(__float_as_uint(q4[t].w) & ~kInactive);
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
  Alloc al = ix->al;
  al.stream = st;
  CHS_TRY(plan_impl(ix, 0, nullptr, nullptr, ix->n, rank, a, al, st));
  if (T > 1) {
    // the wave tables are the index's own host arrays (the copies below read
    // them after this returns)
    std::vector<int32_t>& wtile = ix->wtile_h;
    std::vector<int32_t>& wstart = ix->wstart_h;
    std::vector<int32_t>& qend = ix->qend_h;
    wtile.clear();
    wstart.clear();
    qend.assign(T, 0);
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
  // the plan's own allocator (the caller's, or a fixed arena) serves the
  // sort's temporaries too
  CHS_TRY(plan_impl(ix, qs->point_idx ? 1 : 2, qs->xyz, qs->point_idx, qs->nq, rank,
                    plan->q4.as<float4>(), *plan->q4.al, st));
  plan->q = plan->q4.as<float4>();
  return CHS_OK;
}

// Per-tile query sets on a batched index: queries [q_off[t], q_off[t+1])
// belong to tile t.  They are planned like "every point" queries (tiles by
// decreasing query count, waves of at most 64 that never straddle a tile);
// the wave tables come from the host and the call waits for the stream
// before its host arrays go.
static chs_status plan_queries_tiles(chs_index ix, const chs_queries* qs, const int64_t* q_off,
                                     QueryPlan* plan, hipStream_t st) {
  const int T = ix->ntiles;
  plan->nq = qs->nq;
  plan->nwaves = 0;
  plan->wave_tile = plan->wave_start = plan->tile_qend = nullptr;
  if (qs->nq == 0) return CHS_OK;
  std::vector<int64_t> order(T);
  for (int t = 0; t < T; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return q_off[a + 1] - q_off[a] > q_off[b + 1] - q_off[b];
  });
  std::vector<int32_t> rank(T);
  for (int r = 0; r < T; ++r) rank[order[r]] = r;
  CHS_TRY(plan->q4.alloc(sizeof(float4) * qs->nq));
  CHS_TRY(plan_impl(ix, qs->point_idx ? 1 : 2, qs->xyz, qs->point_idx, qs->nq, rank,
                    plan->q4.as<float4>(), *plan->q4.al, st, q_off));
  plan->q = plan->q4.as<float4>();
  std::vector<int32_t> wtile, wstart, qend(T);
  int64_t pos = 0;
  for (int r = 0; r < T; ++r) {
    const int t = (int)order[r];
    const int64_t nt = q_off[t + 1] - q_off[t];
    for (int64_t b = 0; b < nt; b += kWave) {
      wtile.push_back(t);
      wstart.push_back((int32_t)(pos + b));
    }
    pos += nt;
    qend[t] = (int32_t)pos;
  }
  plan->nwaves = (int64_t)wtile.size();
  CHS_TRY(plan->wt.alloc(4 * (wtile.size() + 1)));
  CHS_TRY(plan->ws.alloc(4 * (wstart.size() + 1)));
  CHS_TRY(plan->qe.alloc(4 * (size_t)T));
  if (!wtile.empty()) {
    CHS_HIP(hipMemcpyAsync(plan->wt.p, wtile.data(), 4 * wtile.size(), hipMemcpyHostToDevice, st));
    CHS_HIP(hipMemcpyAsync(plan->ws.p, wstart.data(), 4 * wstart.size(), hipMemcpyHostToDevice, st));
  }
  CHS_HIP(hipMemcpyAsync(plan->qe.p, qend.data(), 4 * (size_t)T, hipMemcpyHostToDevice, st));
  CHS_HIP(hipStreamSynchronize(st));
  plan->wave_tile = plan->wt.as<int32_t>();
  plan->wave_start = plan->ws.as<int32_t>();
  plan->tile_qend = plan->qe.as<int32_t>();
  return CHS_OK;
}

static chs_status check_tile_queries(chs_index ix, const chs_queries* qs, const int64_t* q_off) {
  if (!ix || !qs || !q_off) {
    set_error("index, queries or q_off is NULL");
    return CHS_E_INVALID;
  }
  if (qs->nq != 0 && !!qs->xyz == !!qs->point_idx) {
    set_error("per-tile query sets: give exactly one of xyz and point_idx");
    return CHS_E_INVALID;
  }
  if (qs->nq < 0 || qs->nq > (int64_t)INT32_MAX) {
    set_error("queries: nq = %lld outside [0, 2^31 - 1]", (long long)qs->nq);
    return CHS_E_INVALID;
  }
  if (q_off[0] != 0 || q_off[ix->ntiles] != qs->nq) {
    set_error("q_off must run from 0 to nq over the index's %d tiles", ix->ntiles);
    return CHS_E_INVALID;
  }
  for (int t = 0; t < ix->ntiles; ++t)
    if (q_off[t + 1] < q_off[t]) {
      set_error("q_off decreases at tile %d", t);
      return CHS_E_INVALID;
    }
  return CHS_OK;
}

__global__ void k_reset_counter(int32_t* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
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

// The list of items a one-wave-per-item k-NN or radius-tile search leaves
// to its second launch (a count, reset here, then up to one entry per
// wave); none for persistent launches (and the k-NN's one-query-at-a-time
// schedule, which has no tiles).
static chs_status split_list(chs_index ix, const QueryPlan& plan, hipStream_t st, Buf* buf,
                             int32_t** out) {
  *out = nullptr;
  if (multi(ix)) return CHS_OK;
  CHS_TRY(buf->alloc(sizeof(int32_t) * (size_t)(plan.nwaves + 1)));
  k_reset_counter<<<1, kWave, 0, st>>>(buf->as<int32_t>());
  CHS_LAUNCH_CHECK();
  *out = buf->as<int32_t>();
  return CHS_OK;
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
    Buf sbuf(&al);
    int32_t* split;
    CHS_TRY(split_list(ix, plan, st, &sbuf, &split));
    RadiusArgs A{make_waves(ix, plan, ctr), ix->grid(), ix->pts, ix->voxels(), r,
                 counts.as<int32_t>(), nullptr, nullptr, 0};
    A.split = split;
    launch_radius(false, ix, nb, st, A, kernel, 0);
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
  Buf sbuf(&al);
  int32_t* split;
  CHS_TRY(split_list(ix, plan, st, &sbuf, &split));
  RadiusArgs A{make_waves(ix, plan, ctr), ix->grid(), ix->pts, ix->voxels(), r, nullptr,
               offsets, nbr, total};
  A.split = split;
  launch_radius(true, ix, nb, st, A, kernel, total / plan.nq);
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
                           int32_t* idx, float* d2, const Alloc& al, hipStream_t st,
                           int64_t* visited) {
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
  Buf sbuf(&al);
  int32_t* split = nullptr;
  if (ix->knn_sched != 3) {
    CHS_TRY(split_list(ix, plan, st, &sbuf, &split));
  }
  KnnArgs A{make_waves(ix, plan, ctr), ix->grid(), ix->pts, ix->voxels(), k, rmax2, idx, d2,
            visited};
  A.split = split;
  launch_knn(ix, nb, st, A);
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
  if (!offsets) {
    set_error("offsets is NULL");
    return CHS_E_INVALID;
  }
  Alloc al = ix->al;
  al.stream = st;
  QueryPlan plan(&al);
  CHS_TRY(plan_queries(ix, qs, &plan, st));
  CHS_TRY(radius_count_impl(ix, plan, kernel, r, offsets, st));
  if (!total) return CHS_OK;  // the total stays on the device, offsets[nq]
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

extern "C" chs_status chs_query_order(chs_index ix, const chs_queries* qs, int32_t* order,
                                      hipStream_t st) {
  clear_error();
  CHS_TRY(check_queries(ix, qs));
  if (qs->nq > 0 && !order) {
    set_error("order is NULL");
    return CHS_E_INVALID;
  }
  if (qs->nq == 0) return CHS_OK;
  Alloc al = ix->al;
  al.stream = st;
  QueryPlan plan(&al);
  CHS_TRY(plan_queries(ix, qs, &plan, st));
  k_plan_order<<<grid_for(plan.nq), kThreads, 0, st>>>(plan.q, plan.nq, order);
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}

extern "C" chs_status chs_fill_chunks(const int64_t* offsets, int64_t nq, int64_t max_entries,
                                      int64_t* bounds, int64_t* entry_bounds, int64_t cap,
                                      int64_t* nchunks, hipStream_t st) {
  clear_error();
  if (!offsets || !nchunks || nq < 0 || max_entries < 1 || cap < 0 ||
      (cap > 0 && (!bounds || !entry_bounds))) {
    set_error("offsets or nchunks is NULL, nq < 0, max_entries < 1, or bounds missing");
    return CHS_E_INVALID;
  }
  std::vector<int64_t> off((size_t)nq + 1);
  CHS_HIP(hipMemcpyAsync(off.data(), offsets, off.size() * sizeof(int64_t),
                         hipMemcpyDeviceToHost, st));
  CHS_HIP(hipStreamSynchronize(st));
  for (int64_t q = 0; q < nq; ++q)
    if (off[q + 1] < off[q]) {
      set_error("offsets decrease at query %lld", (long long)q);
      return CHS_E_INVALID;
    }
  // greedy: each range takes as many further queries as fit, which gives
  // the fewest ranges
  std::vector<int64_t> b{0};
  while (b.back() < nq) {
    const int64_t q = b.back();
    const int64_t room = off[(size_t)nq] - off[q];
    const int64_t lim = max_entries >= room ? off[(size_t)nq] : off[q] + max_entries;
    const int64_t e =
        (int64_t)(std::upper_bound(off.begin() + q + 1, off.end(), lim) - off.begin()) - 1;
    if (e == q) {
      set_error("query %lld alone has %lld entries > max_entries", (long long)q,
                (long long)(off[q + 1] - off[q]));
      return CHS_E_CAPACITY;
    }
    b.push_back(e);
  }
  const int64_t m = (int64_t)b.size() - 1;
  *nchunks = m;
  if (cap == 0) return CHS_OK;
  if (cap < m + 1) {
    set_error("%lld ranges need %lld bound entries, cap is %lld", (long long)m,
              (long long)(m + 1), (long long)cap);
    return CHS_E_CAPACITY;
  }
  for (int64_t i = 0; i <= m; ++i) {
    bounds[i] = b[(size_t)i];
    entry_bounds[i] = off[(size_t)b[(size_t)i]];
  }
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

extern "C" chs_status chs_knn_visited(chs_index ix, const chs_queries* qs, int32_t k,
                                      float r_max, int32_t* idx, float* d2, int64_t* visited,
                                      hipStream_t st) {
  clear_error();
  if (!ix) {
    set_error("index is NULL");
    return CHS_E_INVALID;
  }
  if (qs && qs->nq > 0 && !visited) {
    set_error("visited is NULL");
    return CHS_E_INVALID;
  }
  if (multi(ix) || ix->knn_sched == 3) {
    set_error("visited voxels are reported on a single-tile index without persistent waves, "
              "under the ring or growth schedules");
    return CHS_E_UNSUPPORTED;
  }
  Alloc al = ix->al;
  al.stream = st;
  return knn_impl(ix, qs, k, r_max, idx, d2, al, st, visited);
}

// ---- per-tile query sets on a batched index (Alg. 1 and 2 per tile)
extern "C" chs_status chs_kernel_count_tiles(chs_index ix, const chs_queries* qs,
                                             const int64_t* q_off, int32_t kernel, float r,
                                             int64_t* offsets, int64_t* total, hipStream_t st) {
  clear_error();
  CHS_TRY(check_tile_queries(ix, qs, q_off));
  CHS_TRY(check_kernel(kernel));
  CHS_TRY(check_r(r));
  if (!offsets || !total) {
    set_error("offsets or total is NULL");
    return CHS_E_INVALID;
  }
  Alloc al = ix->al;
  al.stream = st;
  QueryPlan plan(&al);
  CHS_TRY(plan_queries_tiles(ix, qs, q_off, &plan, st));
  CHS_TRY(radius_count_impl(ix, plan, kernel, r, offsets, st));
  int64_t tot = 0;
  CHS_HIP(hipMemcpyAsync(&tot, offsets + qs->nq, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  CHS_HIP(hipStreamSynchronize(st));
  *total = tot;
  return CHS_OK;
}

extern "C" chs_status chs_kernel_fill_tiles(chs_index ix, const chs_queries* qs,
                                            const int64_t* q_off, int32_t kernel, float r,
                                            const int64_t* offsets, int32_t* nbr, int64_t total,
                                            hipStream_t st) {
  clear_error();
  CHS_TRY(check_tile_queries(ix, qs, q_off));
  CHS_TRY(check_kernel(kernel));
  CHS_TRY(check_r(r));
  if (!offsets || (total > 0 && !nbr) || total < 0) {
    set_error("offsets or nbr is NULL, or total < 0");
    return CHS_E_INVALID;
  }
  Alloc al = ix->al;
  al.stream = st;
  QueryPlan plan(&al);
  CHS_TRY(plan_queries_tiles(ix, qs, q_off, &plan, st));
  CHS_TRY(radius_fill_impl(ix, plan, kernel, r, offsets, nbr, total, st));
  return CHS_OK;
}

extern "C" chs_status chs_knn_tiles(chs_index ix, const chs_queries* qs, const int64_t* q_off,
                                    int32_t k, float r_max, int32_t* idx, float* d2,
                                    hipStream_t st) {
  clear_error();
  CHS_TRY(check_tile_queries(ix, qs, q_off));
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
  Alloc al = ix->al;
  al.stream = st;
  QueryPlan plan(&al);
  CHS_TRY(plan_queries_tiles(ix, qs, q_off, &plan, st));
  const float rmax2 = std::isinf(r_max) ? INFINITY : r_max * r_max;
  Buf cbuf(&al);
  int32_t* ctr;
  unsigned nb;
  CHS_TRY(launch_dims(ix, plan, st, &cbuf, &ctr, &nb));
  Buf sbuf(&al);
  int32_t* split = nullptr;
  if (ix->knn_sched != 3) {
    CHS_TRY(split_list(ix, plan, st, &sbuf, &split));
  }
  KnnArgs A{make_waves(ix, plan, ctr), ix->grid(), ix->pts, ix->voxels(), k, rmax2, idx, d2};
  A.split = split;
  launch_knn(ix, nb, st, A);
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}
