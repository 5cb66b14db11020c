// Index construction on the GPU (Section 3.1-3.3 and the reordering remark
// of Section 3.5):
//   bounding box (Eq. 1-2) -> grid size (Eq. 3) -> per-point voxel and global
//   index (Eq. 5-7) -> stable sort by global index (LSD radix: a chain of
//   stable counting sorts on 8-bit digits, so points inside a voxel keep
//   ascending original index) -> non-empty voxels and their starts (per-voxel
//   counts and exclusive prefix sum) -> the flavor's voxel map.
#include <cmath>
#include <cstring>

#include "common.h"

#pragma clang fp contract(off)

namespace chs {

constexpr int kThreads = 256;

static unsigned grid_for(int64_t n, int per_block = kThreads) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// ---------------------------------------------------------------- bbox
// Per-tile FP64 bounding boxes (Eq. 1-2): blocks reduce chunks of one tile
// each, then one block per tile folds its chunks.  Also flags non-finite
// coordinates.
constexpr int64_t kBoxChunk = 1 << 16;

struct Chunk {
  int64_t begin, end;
};

__device__ __forceinline__ void block_fold7(double (&r)[7], double* out) {
  __shared__ double s[kThreads / kWave][7];
  const int w = threadIdx.x / kWave;
  for (int a = 0; a < 3; ++a) {
    r[a] = wave_min(r[a]);
    r[3 + a] = wave_max(r[3 + a]);
  }
  r[6] = wave_max(r[6]);
  if (lane_id() == 0)
    for (int a = 0; a < 7; ++a) s[w][a] = r[a];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kThreads / kWave; ++q) {
      for (int a = 0; a < 3; ++a) {
        r[a] = s[q][a] < r[a] ? s[q][a] : r[a];
        r[3 + a] = s[q][3 + a] > r[3 + a] ? s[q][3 + a] : r[3 + a];
      }
      r[6] = s[q][6] > r[6] ? s[q][6] : r[6];
    }
    for (int a = 0; a < 7; ++a) out[a] = r[a];
  }
}

__global__ __launch_bounds__(kThreads) void k_bbox_chunks(const double* __restrict__ xyz,
                                                          const Chunk* __restrict__ chunks,
                                                          double* __restrict__ part) {
  const Chunk c = chunks[blockIdx.x];
  double r[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
  for (int64_t p = c.begin + threadIdx.x; p < c.end; p += kThreads) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double v = xyz[p * 3 + a];
      if (!isfinite(v)) r[6] = 1.0;
      r[a] = v < r[a] ? v : r[a];
      r[3 + a] = v > r[3 + a] ? v : r[3 + a];
    }
  }
  block_fold7(r, part + (int64_t)blockIdx.x * 7);
}

// block t folds chunks [cfirst[t], cfirst[t+1])
__global__ __launch_bounds__(kThreads) void k_bbox_tiles(const double* __restrict__ part,
                                                         const int32_t* __restrict__ cfirst,
                                                         double* __restrict__ out) {
  const int t = blockIdx.x;
  double r[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
  for (int b = cfirst[t] + threadIdx.x; b < cfirst[t + 1]; b += kThreads) {
    for (int a = 0; a < 3; ++a) {
      r[a] = part[b * 7 + a] < r[a] ? part[b * 7 + a] : r[a];
      r[3 + a] = part[b * 7 + 3 + a] > r[3 + a] ? part[b * 7 + 3 + a] : r[3 + a];
    }
    r[6] = part[b * 7 + 6] > r[6] ? part[b * 7 + 6] : r[6];
  }
  block_fold7(r, out + (int64_t)t * 7);
}

// ---------------------------------------------------------------- keys
// Tile of input point p: binary search over the tile offsets.
__device__ __forceinline__ int tile_of(const int64_t* __restrict__ toff, int ntiles, int64_t p) {
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

template <class K>
__global__ __launch_bounds__(kThreads) void k_keys(const double* __restrict__ xyz, int64_t n,
                                                   const Grid* __restrict__ tiles,
                                                   const double* __restrict__ origin,
                                                   const int64_t* __restrict__ toff, int ntiles,
                                                   K* __restrict__ keys, uint32_t* __restrict__ vals,
                                                   float4* __restrict__ xyz4) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const int t = ntiles > 1 ? tile_of(toff, ntiles, p) : 0;
  const Grid g = tiles[t];
  float c[3];
  int64_t v[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c[a] = (float)(xyz[p * 3 + a] - origin[t * 3 + a]);  // FP64 recentring, then FP32
    if (a < g.dims) v[a] = voxel_clamped((double)c[a], g.s[a], g.n[a]);
  }
  const uint64_t key =
      g.koff + ((uint64_t)v[0] * (uint64_t)g.n[1] + (uint64_t)v[1]) * (uint64_t)g.n[2] + (uint64_t)v[2];
  keys[p] = (K)key;
  vals[p] = (uint32_t)p;
  xyz4[p] = make_float4(c[0], c[1], c[2], __int_as_float((int)p));
}

__global__ __launch_bounds__(kThreads) void k_gather_points(
    const uint32_t* __restrict__ perm_u, const float4* __restrict__ xyz4, int64_t n,
    float4* __restrict__ pts, float* __restrict__ sxyz, int32_t* __restrict__ perm,
    int32_t* __restrict__ inv_perm) {
  const int64_t pos = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (pos >= n) return;
  const uint32_t p = perm_u[pos];
  const float4 c = xyz4[p];
  pts[pos] = c;
  sxyz[pos] = c.x;
  sxyz[n + pos] = c.y;
  sxyz[2 * n + pos] = c.z;
  perm[pos] = (int32_t)p;
  inv_perm[p] = (int32_t)pos;
}

// FP32 coordinates in input order (each tile in its own recentred frame).
__global__ __launch_bounds__(kThreads) void k_coords(const float4* __restrict__ pts,
                                                     const int32_t* __restrict__ inv_perm,
                                                     int64_t n, float* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const float4 c = pts[inv_perm[p]];
  out[3 * p] = c.x;
  out[3 * p + 1] = c.y;
  out[3 * p + 2] = c.z;
}

// ---------------------------------------------------------------- non-empty voxels
template <class K>
__global__ __launch_bounds__(kThreads) void k_run_heads(const K* __restrict__ skeys, int64_t n,
                                                        int32_t* __restrict__ flag) {
  const int64_t pos = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (pos >= n) return;
  flag[pos] = (pos == 0 || skeys[pos] != skeys[pos - 1]) ? 1 : 0;
}

template <class K>
__global__ __launch_bounds__(kThreads) void k_compact_voxels(const K* __restrict__ skeys,
                                                             const int32_t* __restrict__ flag,
                                                             const int32_t* __restrict__ uidx,
                                                             int64_t n, uint64_t* __restrict__ ukeys,
                                                             int32_t* __restrict__ ustart,
                                                             int32_t* __restrict__ m_out) {
  const int64_t pos = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (pos > n) return;
  if (pos == n) {
    ustart[uidx[n]] = (int32_t)n;
    if (m_out) *m_out = uidx[n];
    return;
  }
  if (flag[pos]) {
    const int32_t u = uidx[pos];
    ukeys[u] = (uint64_t)skeys[pos];
    ustart[u] = (int32_t)pos;
  }
}

// ---------------------------------------------------------------- dense map
__global__ __launch_bounds__(kThreads) void k_fill_i32(int32_t* __restrict__ a, int64_t n,
                                                       int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    a[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_fill_u64(uint64_t* __restrict__ a, int64_t n,
                                                       uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    a[i] = v;
}

// M: the non-empty voxels, or (m_dev given) their capacity, the count
// itself being on the device (framed builds)
__global__ __launch_bounds__(kThreads) void k_voxel_counts(const uint64_t* __restrict__ ukeys,
                                                           const int32_t* __restrict__ ustart,
                                                           int64_t M, const int32_t* m_dev,
                                                           int32_t* __restrict__ cnt) {
  const int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (u >= (m_dev ? (int64_t)*m_dev : M)) return;
  cnt[ukeys[u]] = ustart[u + 1] - ustart[u];
}

// ---------------------------------------------------------------- sparse map
__device__ void hash_insert(uint64_t* hk, int32_t* hv, uint64_t mask, uint64_t g, int32_t u) {
  uint64_t h = mix64(g) & mask;
  while (true) {
    const unsigned long long prev =
        atomicCAS((unsigned long long*)&hk[h], (unsigned long long)kEmptyKey,
                  (unsigned long long)g);
    if (prev == kEmptyKey) {
      hv[h] = u;
      return;
    }
    h = (h + 1) & mask;
  }
}

__global__ __launch_bounds__(kThreads) void k_hash_build(const uint64_t* __restrict__ ukeys,
                                                         int64_t M, const int32_t* m_dev,
                                                         uint64_t* hk, int32_t* hv, uint64_t mask) {
  const int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (u >= (m_dev ? (int64_t)*m_dev : M)) return;
  hash_insert(hk, hv, mask, ukeys[u], (int32_t)u);
}

// ---------------------------------------------------------------- column directory
// Global key of the k = 0 voxel of the column holding voxel key `key` (the
// tile found by its key offset: tiles own ascending key ranges).
__device__ __forceinline__ uint64_t column_key(uint64_t key, const Grid* __restrict__ tiles,
                                               int32_t ntiles) {
  int32_t lo = 0, hi = ntiles - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (tiles[mid].koff <= key) lo = mid;
    else hi = mid - 1;
  }
  const uint64_t nz = (uint64_t)tiles[lo].n[2];
  return key - (key - tiles[lo].koff) % nz;
}

// mode 0: count the columns (first voxels of a column) into *ncol;
// mode 1: insert each column with its first compact id;
// mode 2: each column's last voxel writes the end of its id range.
__global__ __launch_bounds__(kThreads) void k_columns(int mode, const uint64_t* __restrict__ ukeys,
                                                      int64_t M, const int32_t* m_dev,
                                                      const Grid* __restrict__ tiles,
                                                      int32_t ntiles, uint64_t* ck, int2* cv,
                                                      uint64_t mask, int32_t* ncol) {
  const int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t m = m_dev ? (int64_t)*m_dev : M;
  const bool in = u < m;
  const uint64_t c = in ? column_key(ukeys[u], tiles, ntiles) : 0;
  const bool head = in && !(u > 0 && column_key(ukeys[u - 1], tiles, ntiles) == c);
  if (mode == 0) {
    // one atomic per wave
    const uint64_t b = __ballot(head);
    if (lane_id() == 0 && b) atomicAdd(ncol, (int32_t)__popcll(b));
    return;
  }
  if (!in) return;
  if (mode == 2) {
    if (u + 1 < m && column_key(ukeys[u + 1], tiles, ntiles) == c) return;
    uint64_t h = mix64(c) & mask;
    while (true) {  // inserted by mode 1 (an empty slot would mean it was not)
      const uint64_t k = ck[h];
      if (k == c) break;
      if (k == kEmptyKey) return;
      h = (h + 1) & mask;
    }
    cv[h].y = (int32_t)(u + 1);
    return;
  }
  if (!head) return;
  uint64_t h = mix64(c) & mask;
  while (true) {
    const unsigned long long prev = atomicCAS((unsigned long long*)&ck[h],
                                              (unsigned long long)kEmptyKey,
                                              (unsigned long long)c);
    if (prev == kEmptyKey) {
      cv[h] = make_int2((int32_t)u, (int32_t)u + 1);
      return;
    }
    h = (h + 1) & mask;
  }
}

// ---------------------------------------------------------------- mixed map
__global__ __launch_bounds__(kThreads) void k_slice_counts(const uint64_t* __restrict__ ukeys,
                                                           int64_t M, int64_t nz,
                                                           int32_t* __restrict__ cnt) {
  extern __shared__ int32_t sh[];
  const bool priv = nz <= 4096;
  if (priv) {
    for (int64_t i = threadIdx.x; i < nz; i += kThreads) sh[i] = 0;
    __syncthreads();
  }
  for (int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x; u < M;
       u += (int64_t)gridDim.x * kThreads) {
    const int64_t k = (int64_t)(ukeys[u] % (uint64_t)nz);
    if (priv)
      atomicAdd(&sh[k], 1);
    else
      atomicAdd(&cnt[k], 1);
  }
  if (priv) {
    __syncthreads();
    for (int64_t i = threadIdx.x; i < nz; i += kThreads)
      if (sh[i]) atomicAdd(&cnt[i], sh[i]);
  }
}

__global__ __launch_bounds__(kThreads) void k_mixed_place(const uint64_t* __restrict__ ukeys,
                                                          int64_t M, int64_t nz,
                                                          const uint8_t* __restrict__ sdense,
                                                          const int64_t* __restrict__ soff,
                                                          int32_t* __restrict__ stab, uint64_t* hk,
                                                          int32_t* hv, uint64_t mask) {
  const int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (u >= M) return;
  const uint64_t g = ukeys[u];
  const int64_t k = (int64_t)(g % (uint64_t)nz);
  if (sdense[k])
    stab[soff[k] + (int64_t)(g / (uint64_t)nz)] = (int32_t)u;
  else
    hash_insert(hk, hv, mask, g, (int32_t)u);
}

// ---------------------------------------------------------------- host side
static chs_status validate_params(const chs_build_params* p) {
  if (p->flavor < CHS_DENSE || p->flavor > CHS_MIXED) {
    set_error("unknown flavor %d", p->flavor);
    return CHS_E_INVALID;
  }
  if (p->dims != 2 && p->dims != 3) {
    set_error("dims must be 2 or 3, got %d", p->dims);
    return CHS_E_INVALID;
  }
  for (int a = 0; a < p->dims; ++a)
    if (!(p->cell[a] > 0.0) || !std::isfinite(p->cell[a])) {
      set_error("cell[%d] must be finite and > 0", a);
      return CHS_E_INVALID;
    }
  if (p->mixed_dense_pct < 0 || p->mixed_dense_pct > 100) {
    set_error("mixed_dense_pct must be in [0, 100]");
    return CHS_E_INVALID;
  }
  if (p->reserved != 0 || p->max_dense_cells < 0) {
    set_error("reserved must be 0 and max_dense_cells >= 0");
    return CHS_E_INVALID;
  }
  return CHS_OK;
}

static chs_status validate(const double* xyz, int64_t n, const chs_build_params* p,
                           chs_index* out) {
  if (!out) {
    set_error("out is NULL");
    return CHS_E_INVALID;
  }
  if (!xyz || !p) {
    set_error("xyz or params is NULL");
    return CHS_E_INVALID;
  }
  if (n < 1 || n > (int64_t)INT32_MAX) {
    set_error("n = %lld outside [1, 2^31 - 1]", (long long)n);
    return CHS_E_INVALID;
  }
  return validate_params(p);
}

template <class K>
static chs_status build_sorted(chs_index ix, const double* xyz, int64_t n, const double* origin_d,
                               const int64_t* toff_d, int bits) {
  const Alloc& al = ix->al;
  hipStream_t st = al.stream;
  Buf keys(&al), vals(&al), tk(&al), tv(&al), xyz4(&al);
  CHS_TRY(keys.alloc(sizeof(K) * n));
  CHS_TRY(vals.alloc(sizeof(uint32_t) * n));
  CHS_TRY(tk.alloc(sizeof(K) * n));
  CHS_TRY(tv.alloc(sizeof(uint32_t) * n));
  CHS_TRY(xyz4.alloc(sizeof(float4) * n));
  k_keys<K><<<grid_for(n), kThreads, 0, st>>>(xyz, n, ix->tiles_d, origin_d, toff_d, ix->ntiles,
                                              keys.as<K>(), vals.as<uint32_t>(), xyz4.as<float4>());
  CHS_LAUNCH_CHECK();
  if (sizeof(K) == 4)
    CHS_TRY(radix_sort_u32(al, (uint32_t*)keys.p, vals.as<uint32_t>(), (uint32_t*)tk.p,
                           tv.as<uint32_t>(), n, bits));
  else
    CHS_TRY(radix_sort_u64(al, (uint64_t*)keys.p, vals.as<uint32_t>(), (uint64_t*)tk.p,
                           tv.as<uint32_t>(), n, bits));
  CHS_TRY(ix->own(&ix->pts, n));
  CHS_TRY(ix->own(&ix->sxyz, 3 * n));
  CHS_TRY(ix->own(&ix->perm, n));
  CHS_TRY(ix->own(&ix->inv_perm, n));
  k_gather_points<<<grid_for(n), kThreads, 0, st>>>(vals.as<uint32_t>(), xyz4.as<float4>(), n,
                                                    ix->pts, ix->sxyz, ix->perm, ix->inv_perm);
  CHS_LAUNCH_CHECK();
  xyz4.release();
  tk.release();
  tv.release();
  // non-empty voxels: run heads of the sorted keys, compacted by a prefix sum
  Buf flag(&al), uidx(&al);
  CHS_TRY(flag.alloc(sizeof(int32_t) * n));
  CHS_TRY(uidx.alloc(sizeof(int32_t) * (n + 1)));
  k_run_heads<K><<<grid_for(n), kThreads, 0, st>>>(keys.as<K>(), n, flag.as<int32_t>());
  CHS_LAUNCH_CHECK();
  CHS_TRY(exclusive_scan_i32_i32(al, flag.as<int32_t>(), uidx.as<int32_t>(), n));
  if (ix->framed) {
    // sized for the worst case (every point its own voxel); the count stays
    // on the device
    ix->M = -1;
    CHS_TRY(ix->own(&ix->m_dev, 1));
    CHS_TRY(ix->own(&ix->ukeys, (size_t)n));
    CHS_TRY(ix->own(&ix->ustart, (size_t)n + 1));
  } else {
    int32_t M = 0;
    CHS_HIP(hipMemcpyAsync(&M, uidx.as<int32_t>() + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CHS_HIP(hipStreamSynchronize(st));
    ix->M = M;
    CHS_TRY(ix->own(&ix->ukeys, (size_t)M));
    CHS_TRY(ix->own(&ix->ustart, (size_t)M + 1));
  }
  k_compact_voxels<K><<<grid_for(n + 1), kThreads, 0, st>>>(keys.as<K>(), flag.as<int32_t>(),
                                                            uidx.as<int32_t>(), n, ix->ukeys,
                                                            ix->ustart, ix->m_dev);
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}

static chs_status build_dense(chs_index ix) {
  const Alloc& al = ix->al;
  hipStream_t st = al.stream;
  const int64_t nc = (int64_t)ix->total_cells;
  Buf cnt(&al);
  CHS_TRY(cnt.alloc(sizeof(int32_t) * nc));
  k_fill_i32<<<4096, kThreads, 0, st>>>(cnt.as<int32_t>(), nc, 0);
  CHS_LAUNCH_CHECK();
  const int64_t mcap = ix->M >= 0 ? ix->M : ix->n;
  k_voxel_counts<<<grid_for(mcap), kThreads, 0, st>>>(ix->ukeys, ix->ustart, mcap, ix->m_dev,
                                                      cnt.as<int32_t>());
  CHS_LAUNCH_CHECK();
  CHS_TRY(ix->own(&ix->dstart, (size_t)nc + 1));
  CHS_TRY(exclusive_scan_i32_i32(al, cnt.as<int32_t>(), ix->dstart, nc));
  return CHS_OK;
}

static chs_status alloc_hash(chs_index ix, int64_t nkeys) {
  uint64_t cap = 64;
  while (cap < (uint64_t)(2 * nkeys)) cap <<= 1;  // load factor <= 0.5
  ix->hcap = cap;
  CHS_TRY(ix->own(&ix->hkeys, cap));
  CHS_TRY(ix->own(&ix->hvals, cap));
  k_fill_u64<<<1024, kThreads, 0, ix->al.stream>>>(ix->hkeys, (int64_t)cap, kEmptyKey);
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}

static chs_status build_sparse(chs_index ix) {
  const int64_t mcap = ix->M >= 0 ? ix->M : ix->n;
  CHS_TRY(alloc_hash(ix, mcap));
  k_hash_build<<<grid_for(mcap), kThreads, 0, ix->al.stream>>>(ix->ukeys, mcap, ix->m_dev,
                                                               ix->hkeys, ix->hvals, ix->hcap - 1);
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}

// The column directory of the sparse and mixed maps: a column's voxels are
// adjacent in the compact order, so one probe per column of a search box
// finds them all (instead of one probe per voxel).  Sized from the column
// count, or, for framed builds (nothing read back), from the point count.
static chs_status build_columns(chs_index ix) {
  const Alloc& al = ix->al;
  hipStream_t st = al.stream;
  const int64_t mcap = ix->M >= 0 ? ix->M : ix->n;
  int64_t ncol = mcap;
  if (!ix->framed) {
    Buf cnt(&al);
    CHS_TRY(cnt.alloc(sizeof(int32_t)));
    k_fill_i32<<<1, kThreads, 0, st>>>(cnt.as<int32_t>(), 1, 0);
    CHS_LAUNCH_CHECK();
    k_columns<<<grid_for(mcap), kThreads, 0, st>>>(0, ix->ukeys, mcap, ix->m_dev, ix->tiles_d,
                                                     ix->ntiles, nullptr, nullptr, 0,
                                                     cnt.as<int32_t>());
    CHS_LAUNCH_CHECK();
    int32_t h = 0;
    CHS_HIP(hipMemcpyAsync(&h, cnt.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CHS_HIP(hipStreamSynchronize(st));
    ncol = h;
  }
  uint64_t cap = 64;
  while (cap < (uint64_t)(2 * ncol)) cap <<= 1;  // load factor <= 0.5
  ix->ccap = cap;
  CHS_TRY(ix->own(&ix->ckeys, cap));
  CHS_TRY(ix->own(&ix->cvals, cap));
  k_fill_u64<<<1024, kThreads, 0, st>>>(ix->ckeys, (int64_t)cap, kEmptyKey);
  CHS_LAUNCH_CHECK();
  for (int mode = 1; mode <= 2; ++mode) {
    k_columns<<<grid_for(mcap), kThreads, 0, st>>>(mode, ix->ukeys, mcap, ix->m_dev, ix->tiles_d,
                                                     ix->ntiles, ix->ckeys, ix->cvals, cap - 1,
                                                     nullptr);
    CHS_LAUNCH_CHECK();
  }
  return CHS_OK;
}

static chs_status build_mixed(chs_index ix) {
  const Alloc& al = ix->al;
  hipStream_t st = al.stream;
  const Grid& g = ix->grid();
  const int64_t nz = g.n[2], nxy = g.n[0] * g.n[1];
  Buf cnt(&al);
  CHS_TRY(cnt.alloc(sizeof(int32_t) * nz));
  k_fill_i32<<<grid_for(nz), kThreads, 0, st>>>(cnt.as<int32_t>(), nz, 0);
  CHS_LAUNCH_CHECK();
  const size_t shmem = nz <= 4096 ? sizeof(int32_t) * nz : 0;
  k_slice_counts<<<256, kThreads, shmem, st>>>(ix->ukeys, ix->M, nz, cnt.as<int32_t>());
  CHS_LAUNCH_CHECK();
  std::vector<int32_t> hc(nz);
  CHS_HIP(hipMemcpyAsync(hc.data(), cnt.p, sizeof(int32_t) * nz, hipMemcpyDeviceToHost, st));
  CHS_HIP(hipStreamSynchronize(st));
  std::vector<uint8_t> dense(nz, 0);
  std::vector<int64_t> off(nz, -1);
  int64_t ndense = 0, sparse_keys = 0;
  for (int64_t k = 0; k < nz; ++k) {
    // Section 3.3.3: a slice turns dense once mixed_dense_pct % of its voxels hold points
    if (100 * (int64_t)hc[k] >= (int64_t)ix->mixed_pct * nxy) {
      dense[k] = 1;
      off[k] = ndense * nxy;
      ++ndense;
    } else {
      sparse_keys += hc[k];
    }
  }
  ix->n_dense_slices = ndense;
  CHS_TRY(ix->own(&ix->slice_dense, (size_t)nz));
  CHS_TRY(ix->own(&ix->slice_off, (size_t)nz));
  CHS_HIP(hipMemcpyAsync(ix->slice_dense, dense.data(), nz, hipMemcpyHostToDevice, st));
  CHS_HIP(hipMemcpyAsync(ix->slice_off, off.data(), sizeof(int64_t) * nz, hipMemcpyHostToDevice, st));
  CHS_TRY(ix->own(&ix->stab, (size_t)(ndense * nxy)));
  if (ndense * nxy > 0) {
    k_fill_i32<<<4096, kThreads, 0, st>>>(ix->stab, ndense * nxy, -1);
    CHS_LAUNCH_CHECK();
  }
  CHS_TRY(alloc_hash(ix, sparse_keys));
  k_mixed_place<<<grid_for(ix->M), kThreads, 0, st>>>(ix->ukeys, ix->M, nz, ix->slice_dense,
                                                       ix->slice_off, ix->stab, ix->hkeys,
                                                       ix->hvals, ix->hcap - 1);
  CHS_LAUNCH_CHECK();
  // the host vectors must outlive the asynchronous copies
  CHS_HIP(hipStreamSynchronize(st));
  return CHS_OK;
}

// Build over ntiles tiles (a plain index is one tile).  params[t] gives the
// voxel edges and dims of tile t; the flavor is that of params[0].
// frames (host, [ntiles][6] min x,y,z then max x,y,z, or NULL): bounding
// boxes given by the caller; the build then reads nothing back from the
// device and never waits for the stream.
static chs_status build_impl(chs_index ix, const double* xyz, int64_t n, const int64_t* toff,
                             int ntiles, const chs_build_params* params, const double* frames) {
  const Alloc& al = ix->al;
  hipStream_t st = al.stream;
  ix->ntiles = ntiles;
  ix->tile_off.assign(toff, toff + ntiles + 1);
  ix->framed = frames != nullptr;
  Buf toff_d(&al), origin_d(&al);
  std::vector<double> h(7 * (size_t)ntiles);
  if (frames) {
    for (int t = 0; t < ntiles; ++t) {
      for (int a = 0; a < 3; ++a) {
        h[7 * (size_t)t + a] = frames[6 * (size_t)t + a];
        h[7 * (size_t)t + 3 + a] = frames[6 * (size_t)t + 3 + a];
      }
      h[7 * (size_t)t + 6] = 0.0;
    }
  } else {
    // chunks of at most kBoxChunk points, never straddling two tiles
    std::vector<Chunk> chunks;
    std::vector<int32_t> cfirst(ntiles + 1, 0);
    for (int t = 0; t < ntiles; ++t) {
      cfirst[t] = (int32_t)chunks.size();
      for (int64_t b = toff[t]; b < toff[t + 1]; b += kBoxChunk)
        chunks.push_back(Chunk{b, b + kBoxChunk < toff[t + 1] ? b + kBoxChunk : toff[t + 1]});
    }
    cfirst[ntiles] = (int32_t)chunks.size();
    Buf chunk_d(&al), cfirst_d(&al), part(&al), bb(&al);
    CHS_TRY(chunk_d.alloc(sizeof(Chunk) * chunks.size()));
    CHS_TRY(cfirst_d.alloc(sizeof(int32_t) * (ntiles + 1)));
    CHS_TRY(part.alloc(sizeof(double) * 7 * chunks.size()));
    CHS_TRY(bb.alloc(sizeof(double) * 7 * ntiles));
    CHS_HIP(hipMemcpyAsync(chunk_d.p, chunks.data(), sizeof(Chunk) * chunks.size(),
                           hipMemcpyHostToDevice, st));
    CHS_HIP(hipMemcpyAsync(cfirst_d.p, cfirst.data(), sizeof(int32_t) * (ntiles + 1),
                           hipMemcpyHostToDevice, st));
    k_bbox_chunks<<<(unsigned)chunks.size(), kThreads, 0, st>>>(xyz, chunk_d.as<Chunk>(),
                                                                 part.as<double>());
    CHS_LAUNCH_CHECK();
    k_bbox_tiles<<<(unsigned)ntiles, kThreads, 0, st>>>(part.as<double>(), cfirst_d.as<int32_t>(),
                                                         bb.as<double>());
    CHS_LAUNCH_CHECK();
    CHS_HIP(hipMemcpyAsync(h.data(), bb.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    CHS_HIP(hipStreamSynchronize(st));
  }
  ix->tiles.resize(ntiles);
  ix->origin.resize(3 * (size_t)ntiles);
  ix->max32.resize(3 * (size_t)ntiles);
  uint64_t koff = 0;
  for (int t = 0; t < ntiles; ++t) {
    const double* r = &h[7 * (size_t)t];
    if (r[6] != 0.0) {
      set_error("xyz holds non-finite coordinates (tile %d)", t);
      return CHS_E_INVALID;
    }
    const chs_build_params& p = params[t];
    Grid& g = ix->tiles[t];
    g.dims = p.dims;
    g.pad_ = 0;
    g.poff = toff[t];
    g.koff = koff;
    double prod = 1.0;
    for (int a = 0; a < 3; ++a) {
      ix->origin[3 * t + a] = r[a];
      // recentring is monotone, so the FP32 maximum is fl32(max - min)
      ix->max32[3 * t + a] = (float)(r[3 + a] - r[a]);
      g.s[a] = (a == 2 && p.dims == 2) ? 1.0 : p.cell[a];
      if (a == 2 && p.dims == 2) {
        g.n[2] = 1;
        continue;
      }
      // Eq. 3: n_a = floor((p+_a - p-_a) / s_a) + 1
      const double na = std::floor((double)ix->max32[3 * t + a] / g.s[a]) + 1.0;
      if (!(na < 1.0e9)) {
        set_error("tile %d: grid axis %d would have %g voxels", t, a, na);
        return CHS_E_CAPACITY;
      }
      g.n[a] = (int64_t)na;
      prod *= na;
    }
    if (!(prod + (double)koff < 4.0e18)) {
      set_error("grid would have %g voxels (global index overflows 64 bits)", prod + (double)koff);
      return CHS_E_CAPACITY;
    }
    koff += (uint64_t)g.n[0] * (uint64_t)g.n[1] * (uint64_t)g.n[2];
  }
  ix->total_cells = koff;
  double wsum = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    const Grid& g = ix->tiles[t];
    wsum += (double)(toff[t + 1] - toff[t]) * (g.s[0] < g.s[1] ? g.s[0] : g.s[1]);
  }
  ix->cell_xy = wsum / (double)toff[ntiles];
  if (ix->flavor == CHS_DENSE && ix->total_cells > (uint64_t)ix->ncells_limit()) {
    set_error("dense grid of %llu voxels exceeds the limit %lld; use the sparse or mixed flavor",
              (unsigned long long)ix->total_cells, (long long)ix->ncells_limit());
    return CHS_E_CAPACITY;
  }
  if (ix->flavor == CHS_MIXED && (double)ix->grid().n[0] * (double)ix->grid().n[1] > 2.0e9) {
    set_error("mixed flavor: a z-slice of %lld x %lld voxels is too large",
              (long long)ix->grid().n[0], (long long)ix->grid().n[1]);
    return CHS_E_CAPACITY;
  }
  CHS_TRY(ix->own(&ix->tiles_d, (size_t)ntiles));
  CHS_HIP(hipMemcpyAsync(ix->tiles_d, ix->tiles.data(), sizeof(Grid) * ntiles,
                         hipMemcpyHostToDevice, st));
  CHS_TRY(toff_d.alloc(sizeof(int64_t) * (ntiles + 1)));
  CHS_TRY(origin_d.alloc(sizeof(double) * 3 * ntiles));
  // (from the index's own copies, which outlive the queued copies)
  CHS_HIP(hipMemcpyAsync(toff_d.p, ix->tile_off.data(), sizeof(int64_t) * (ntiles + 1),
                         hipMemcpyHostToDevice, st));
  CHS_HIP(hipMemcpyAsync(origin_d.p, ix->origin.data(), sizeof(double) * 3 * ntiles,
                         hipMemcpyHostToDevice, st));
  const int bits = ceil_log2(ix->total_cells);
  if (bits <= 32)
    CHS_TRY(build_sorted<uint32_t>(ix, xyz, n, origin_d.as<double>(), toff_d.as<int64_t>(), bits));
  else
    CHS_TRY(build_sorted<uint64_t>(ix, xyz, n, origin_d.as<double>(), toff_d.as<int64_t>(), bits));
  if (ix->flavor == CHS_DENSE) CHS_TRY(build_dense(ix));
  if (ix->flavor == CHS_SPARSE) CHS_TRY(build_sparse(ix));
  if (ix->flavor == CHS_MIXED) CHS_TRY(build_mixed(ix));
  if (ix->flavor != CHS_DENSE) CHS_TRY(build_columns(ix));
  // the processing order of "every point" queries (searches then plan
  // nothing for them)
  CHS_TRY(plan_every_point(ix, st));
  // (every host array the queued copies read belongs to the index, and
  // temporaries are released in stream order: nothing to wait for)
  return CHS_OK;
}

static chs_status build_common(const double* xyz, int64_t n, const int64_t* toff, int ntiles,
                               const chs_build_params* params, const chs_allocator* alloc,
                               hipStream_t stream, chs_index* out, const double* frames = nullptr) {
  if (alloc && (!alloc->alloc || !alloc->free)) {
    set_error("allocator callbacks are NULL");
    return CHS_E_INVALID;
  }
  chs_index ix = new chs_index_s();
  ix->al.stream = stream;
  if (alloc) {
    ix->al.a = *alloc;
    ix->al.has = true;
  }
  ix->flavor = params[0].flavor;
  ix->mixed_pct = params[0].mixed_dense_pct > 0 ? params[0].mixed_dense_pct : 80;
  ix->max_dense =
      params[0].max_dense_cells > 0 ? params[0].max_dense_cells : (int64_t)INT32_MAX - 1;
  ix->n = n;
  ix->persistent = ntiles > 1;
  if (hipGetDevice(&ix->device) != hipSuccess) {
    (void)hipGetLastError();
    set_error("no HIP device");
    delete ix;
    return CHS_E_DEVICE;
  }
  chs_status s = build_impl(ix, xyz, n, toff, ntiles, params, frames);
  if (s != CHS_OK) {
    std::string msg = last_error();
    chs_free(ix);
    set_error("%s", msg.c_str());
    return s;
  }
  *out = ix;
  return CHS_OK;
}

}  // namespace chs

using namespace chs;

extern "C" chs_status chs_build(const double* xyz, int64_t n, const chs_build_params* params,
                                const chs_allocator* alloc, hipStream_t stream, chs_index* out) {
  clear_error();
  CHS_TRY(validate(xyz, n, params, out));
  const int64_t toff[2] = {0, n};
  return build_common(xyz, n, toff, 1, params, alloc, stream, out);
}

static chs_status check_batch(const double* xyz, int64_t n, const int64_t* tile_off,
                              int32_t ntiles, const chs_build_params* params, chs_index* out) {
  CHS_TRY(validate(xyz, n, params, out));
  if (!tile_off || ntiles < 1 || ntiles > (1 << 20)) {
    set_error("tile_off is NULL or ntiles = %d outside [1, 2^20]", ntiles);
    return CHS_E_INVALID;
  }
  if (tile_off[0] != 0 || tile_off[ntiles] != n) {
    set_error("tile_off must start at 0 and end at n");
    return CHS_E_INVALID;
  }
  for (int t = 0; t < ntiles; ++t) {
    if (tile_off[t + 1] <= tile_off[t]) {
      set_error("tile %d is empty or tile_off decreases", t);
      return CHS_E_INVALID;
    }
    CHS_TRY(validate_params(&params[t]));
    if (params[t].flavor != params[0].flavor) {
      set_error("all tiles must use the same flavor");
      return CHS_E_INVALID;
    }
  }
  if (ntiles > 1 && params[0].flavor == CHS_MIXED) {
    set_error("the mixed flavor is not available for batched indexes");
    return CHS_E_UNSUPPORTED;
  }
  return CHS_OK;
}

extern "C" chs_status chs_build_batch(const double* xyz, int64_t n, const int64_t* tile_off,
                                      int32_t ntiles, const chs_build_params* params,
                                      const chs_allocator* alloc, hipStream_t stream,
                                      chs_index* out) {
  clear_error();
  CHS_TRY(check_batch(xyz, n, tile_off, ntiles, params, out));
  return build_common(xyz, n, tile_off, ntiles, params, alloc, stream, out);
}

extern "C" chs_status chs_build_batch_framed(const double* xyz, int64_t n,
                                             const int64_t* tile_off, int32_t ntiles,
                                             const chs_build_params* params,
                                             const double* frames, const chs_allocator* alloc,
                                             hipStream_t stream, chs_index* out) {
  clear_error();
  CHS_TRY(check_batch(xyz, n, tile_off, ntiles, params, out));
  if (!frames) {
    set_error("frames is NULL");
    return CHS_E_INVALID;
  }
  if (params[0].flavor == CHS_MIXED) {
    set_error("the mixed flavor sizes its slice tables from the points: not available framed");
    return CHS_E_UNSUPPORTED;
  }
  for (int t = 0; t < ntiles; ++t)
    for (int a = 0; a < 3; ++a) {
      const double lo = frames[6 * (size_t)t + a], hi = frames[6 * (size_t)t + 3 + a];
      if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo <= hi)) {
        set_error("frame of tile %d: axis %d is not a finite range min <= max", t, a);
        return CHS_E_INVALID;
      }
    }
  return build_common(xyz, n, tile_off, ntiles, params, alloc, stream, out, frames);
}

extern "C" void chs_free(chs_index ix) {
  if (!ix) return;
  for (void* p : ix->owned) ix->al.put(p);
  ix->owned.clear();
  delete ix;
}

extern "C" chs_status chs_index_set_option(chs_index ix, int32_t option, int64_t value) {
  clear_error();
  if (!ix) {
    set_error("index is NULL");
    return CHS_E_INVALID;
  }
  if (option == CHS_OPT_PERSISTENT) {
    ix->persistent = value != 0;
    return CHS_OK;
  }
  if (option == CHS_OPT_FILL_STAGE) {
    if (value != 0 && value != 16 && value != 24 && value != 32 && value != 64) {
      set_error("fill stage must be 0 (by mean row length), 16, 24, 32 or 64");
      return CHS_E_INVALID;
    }
    ix->fill_stage = (int32_t)value;
    return CHS_OK;
  }
  if (option == CHS_OPT_RADIUS_SCHEDULE) {
    if (value < 0 || value > 2) {
      set_error("radius schedule must be 0 (auto), 1 (64-query tiles) or 2 (8-query groups)");
      return CHS_E_INVALID;
    }
    ix->radius_sched = (int32_t)value;
    return CHS_OK;
  }
  if (option == CHS_OPT_KNN_SCHEDULE) {
    if (value < 0 || value > 3) {
      set_error("k-NN schedule must be 0 (rings), 1 (density growth), 2 (monotonic growth) "
                "or 3 (one query at a time)");
      return CHS_E_INVALID;
    }
    ix->knn_sched = (int32_t)value;
    return CHS_OK;
  }
  set_error("unknown option %d", option);
  return CHS_E_INVALID;
}

static void fill_info(chs_index ix, int t, chs_index_info_t* out) {
  std::memset(out, 0, sizeof(*out));
  const Grid& g = ix->tiles[t];
  for (int a = 0; a < 3; ++a) {
    out->origin[a] = ix->origin[3 * t + a];
    out->max32[a] = ix->max32[3 * t + a];
    out->cell[a] = g.s[a];
    out->ncell[a] = g.n[a];
  }
  out->dims = g.dims;
  out->flavor = ix->flavor;
}

// The non-empty voxel count of a framed index, read from the device on
// first use (waits for the index's stream).
static chs_status resolve_m(chs_index ix) {
  if (ix->M >= 0) return CHS_OK;
  int32_t m = 0;
  CHS_HIP(hipMemcpyAsync(&m, ix->m_dev, sizeof(int32_t), hipMemcpyDeviceToHost, ix->al.stream));
  CHS_HIP(hipStreamSynchronize(ix->al.stream));
  ix->M = m;
  return CHS_OK;
}

extern "C" chs_status chs_index_info(chs_index ix, chs_index_info_t* out) {
  clear_error();
  if (!ix || !out) {
    set_error("index or out is NULL");
    return CHS_E_INVALID;
  }
  CHS_TRY(resolve_m(ix));
  fill_info(ix, 0, out);
  out->n_points = ix->n;
  out->n_nonempty = ix->M;
  out->n_dense_slices = ix->n_dense_slices;
  out->device_bytes = ix->device_bytes;
  out->ntiles = ix->ntiles;
  return CHS_OK;
}

extern "C" chs_status chs_tile_info(chs_index ix, int32_t tile, chs_index_info_t* out) {
  clear_error();
  if (!ix || !out || tile < 0 || tile >= ix->ntiles) {
    set_error("index or out is NULL, or tile out of range");
    return CHS_E_INVALID;
  }
  fill_info(ix, tile, out);
  out->n_points = ix->tile_off[tile + 1] - ix->tile_off[tile];
  out->n_nonempty = -1;
  out->device_bytes = ix->device_bytes;
  out->ntiles = ix->ntiles;
  return CHS_OK;
}

extern "C" chs_status chs_index_arrays(chs_index ix, chs_index_arrays_t* out) {
  clear_error();
  if (!ix || !out) {
    set_error("index or out is NULL");
    return CHS_E_INVALID;
  }
  CHS_TRY(resolve_m(ix));
  out->perm = ix->perm;
  out->inv_perm = ix->inv_perm;
  out->sorted_xyz = ix->sxyz;
  out->points = reinterpret_cast<const float*>(ix->pts);
  out->cell_keys = ix->ukeys;
  out->cell_start = ix->ustart;
  out->dense_start = ix->flavor == CHS_DENSE ? ix->dstart : nullptr;
  out->slice_dense = ix->flavor == CHS_MIXED ? ix->slice_dense : nullptr;
  return CHS_OK;
}

extern "C" chs_status chs_index_coords(chs_index ix, float* out, hipStream_t st) {
  clear_error();
  if (!ix || !out) {
    set_error("index or out is NULL");
    return CHS_E_INVALID;
  }
  k_coords<<<grid_for(ix->n), kThreads, 0, st>>>(ix->pts, ix->inv_perm, ix->n, out);
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}
