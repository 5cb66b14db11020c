// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/chs.h"

#pragma clang fp contract(off)

namespace chs {

constexpr int kWave = 64;

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();
const char* last_error();

#define CHS_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) {                                                            \
      ::chs::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                       __LINE__);                                                      \
      return CHS_E_DEVICE;                                                             \
    }                                                                                  \
  } while (0)

#define CHS_TRY(expr)                 \
  do {                                \
    chs_status _s = (expr);           \
    if (_s != CHS_OK) return _s;      \
  } while (0)

#define CHS_LAUNCH_CHECK() CHS_HIP(hipGetLastError())

// ---------------------------------------------------------------- memory
// Device memory through the caller's allocator, or stream-ordered
// hipMallocAsync when none is given.
struct Alloc {
  chs_allocator a{};
  bool has = false;
  hipStream_t stream = nullptr;
  void* get(size_t bytes) const;
  void put(void* p) const;
};

// A temporary device buffer released when it goes out of scope.
struct Buf {
  const Alloc* al = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  Buf() = default;
  explicit Buf(const Alloc* a) : al(a) {}
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  ~Buf() { release(); }
  chs_status alloc(size_t nbytes);
  void release() {
    if (p && al) al->put(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------- grid
// Geometry of one tile's grid as the kernels see it.  A plain index is one
// tile; a batched index concatenates the tiles' voxel key spaces, tile t's
// voxel (0,0,0) having the global key koff.
struct Grid {
  double s[3];    // voxel edges
  int64_t n[3];   // n_x, n_y, n_z
  uint64_t koff;  // global key of the tile's first voxel
  int64_t poff;   // first input point of the tile (results are tile-local)
  int32_t dims;
  int32_t pad_;
};

// Voxel storage as the kernels see it (global over all tiles).
struct Voxels {
  int32_t flavor;
  int32_t M;                 // non-empty voxels
  int64_t npts;              // stored points
  const int32_t* dstart;     // DENSE: [total voxels + 1]
  const uint64_t* hkeys;     // SPARSE/MIXED: open-addressing keys (EMPTY = ~0)
  const int32_t* hvals;      //   -> compact voxel id
  uint64_t hmask;            //   capacity - 1 (power of two)
  const int32_t* ustart;     // compact voxel id -> first stored position, [M+1]
  const uint8_t* slice_dense;  // MIXED: [n_z]
  const int64_t* slice_off;    // MIXED: [n_z] offset of a dense slice's table
  const int32_t* stab;         // MIXED: dense slice tables, compact id or -1
  // SPARSE/MIXED column directory: open-addressing table keyed by the
  // global key of a column's k = 0 voxel -> the compact ids [first, end) of
  // its non-empty voxels (adjacent: the key is z-fastest, Eq. 7)
  const uint64_t* ukeys;     // compact id -> global key, [M]
  const uint64_t* ckeys;
  const int2* cvals;
  uint64_t cmask;
};

constexpr uint64_t kEmptyKey = ~0ull;

}  // namespace chs

struct chs_index_s {
  chs::Alloc al;
  int device = 0;
  int32_t flavor = 0, mixed_pct = 80;
  int32_t ntiles = 1;
  int64_t n = 0, M = 0;
  uint64_t total_cells = 1;  // voxels over all tiles
  int64_t n_dense_slices = 0;
  int64_t device_bytes = 0;
  int64_t max_dense = (int64_t)INT32_MAX - 1;
  bool persistent = false;  // searches pull waves from a work counter
  int32_t knn_sched = 0;  // k-NN schedule: 0 rings, 1 density growth (Alg. 2), 2 monotonic, 3 solo
  int32_t fill_stage = 0;    // radius fill: LDS entries per lane (0: by mean row length)
  int32_t radius_sched = 0;  // radius schedule: 0 auto, 1 64-query tiles, 2 8-query groups
  double cell_xy = 1.0;      // point-weighted mean of the tiles' smaller xy voxel edge
  // per tile, host copies (tile 0 is the whole cloud of a plain index)
  std::vector<chs::Grid> tiles;
  std::vector<double> origin;   // [3 * ntiles]
  std::vector<float> max32;     // [3 * ntiles]
  std::vector<int64_t> tile_off;  // [ntiles + 1] input point ranges
  std::vector<int64_t> tile_m;    // non-empty voxels per tile
  chs::Grid* tiles_d = nullptr;   // device copy of `tiles`
  // stored (voxel-ordered) cloud
  int32_t* perm = nullptr;
  int32_t* inv_perm = nullptr;
  float* sxyz = nullptr;      // SoA [3][n]
  float4* pts = nullptr;      // [n] x, y, z, original index bits
  uint64_t* ukeys = nullptr;  // [M]
  int32_t* ustart = nullptr;  // [M+1]
  // flavor maps
  int32_t* dstart = nullptr;
  uint64_t* hkeys = nullptr;
  int32_t* hvals = nullptr;
  uint64_t hcap = 0;
  uint8_t* slice_dense = nullptr;
  int64_t* slice_off = nullptr;
  int32_t* stab = nullptr;
  uint64_t* ckeys = nullptr;  // column directory (SPARSE/MIXED)
  int2* cvals = nullptr;
  uint64_t ccap = 0;
  // cached processing order for "every point" queries: centres in waves of
  // at most 64 that never straddle two tiles
  float4* allq = nullptr;
  int32_t* wave_tile = nullptr;   // batched only: tile of each wave
  int32_t* wave_start = nullptr;  //   first query of each wave
  int32_t* tile_qend = nullptr;   //   end of each tile's queries
  int64_t allq_waves = 0;
  // host data read by copies queued on the stream, kept for the index's
  // life (so that no build step waits for the stream to free them)
  std::vector<int32_t> tplan_h;  // per tile: Hilbert bits, z bits, rank, 0
  std::vector<int32_t> wtile_h, wstart_h, qend_h;
  // framed builds (bounding boxes given by the caller): nothing is read back
  // from the device, so the non-empty voxel count stays there until asked
  bool framed = false;
  int32_t* m_dev = nullptr;
  std::vector<void*> owned;

  int64_t ncells_limit() const { return max_dense; }
  const chs::Grid& grid() const { return tiles[0]; }
  chs::Voxels voxels() const {
    chs::Voxels v;
    v.flavor = flavor;
    v.M = (int32_t)(M >= 0 ? M : n);  // framed: the capacity bounds the ids
    v.npts = n;
    v.dstart = dstart;
    v.hkeys = hkeys;
    v.hvals = hvals;
    v.hmask = hcap ? hcap - 1 : 0;
    v.ustart = ustart;
    v.slice_dense = slice_dense;
    v.slice_off = slice_off;
    v.stab = stab;
    v.ukeys = ukeys;
    v.ckeys = ckeys;
    v.cvals = cvals;
    v.cmask = ccap ? ccap - 1 : 0;
    return v;
  }
  // index-owned allocation
  template <class T>
  chs_status own(T** out, size_t count) {
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 256;
    void* p = al.get(bytes);
    if (!p) {
      chs::set_error("allocator returned NULL for %zu bytes", bytes);
      return CHS_E_NOMEM;
    }
    owned.push_back(p);
    device_bytes += (int64_t)bytes;
    *out = static_cast<T*>(p);
    return CHS_OK;
  }
};

namespace chs {

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Broadcast of lane 0's value.  Applied to a value every lane already holds,
// it tells the compiler that the value is wave-uniform, so it lives in
// scalar registers and the loops it bounds are not divergent.
__device__ __forceinline__ int32_t first_lane(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float first_lane(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int64_t first_lane(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double first_lane(double v) {
  return __longlong_as_double(first_lane((int64_t)__double_as_longlong(v)));
}

// Reductions over the full wave (every lane active); the result is uniform.
template <class T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    T o = __shfl_xor(v, m, kWave);
    v = o < v ? o : v;
  }
  return first_lane(v);
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    T o = __shfl_xor(v, m, kWave);
    v = o > v ? o : v;
  }
  return first_lane(v);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Voxel coordinate along one axis: floor of the IEEE FP64 quotient, as a
// double (may be negative or beyond the grid for query boxes).
__device__ __forceinline__ double vfloor(double v, double s) { return floor(v / s); }

// Same, clamped into the grid (0-based, Eq. 5).
__device__ __forceinline__ int64_t voxel_clamped(double v, double s, int64_t n) {
  double c = floor(v / s);
  if (c > (double)(n - 1)) return n - 1;
  if (c < 0.0) return 0;
  return (int64_t)c;
}

// splitmix64 finaliser, used to spread voxel keys over the hash table.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

// Stored-position range [b, e) of the voxels (i, j, k0..k1) of one column.
// Because the global index is z-fastest (Eq. 7), these voxels are adjacent
// in the stored order and their points form one contiguous run.  Voxel
// coordinates outside the tile give an empty run, and every table value is
// checked against the table's extent before use.  The flavor is a
// compile-time constant (a run-time flavor test inside divergent lookup
// loops was once compiled into a lane mask reused under another exec mask,
// which sent sparse lookups into the mixed slice table, a NULL pointer
// there).
template <int FL>
__device__ __forceinline__ void column_run(const Voxels& vx, const Grid& g, int64_t i, int64_t j,
                                           int64_t k0, int64_t k1, int32_t* b, int32_t* e) {
  *b = 0;
  *e = 0;
  if (k0 < 0) k0 = 0;
  if (k1 > g.n[2] - 1) k1 = g.n[2] - 1;
  if (i < 0 || i >= g.n[0] || j < 0 || j >= g.n[1] || k0 > k1) return;
  const uint64_t base =
      g.koff + ((uint64_t)i * (uint64_t)g.n[1] + (uint64_t)j) * (uint64_t)g.n[2];
  int32_t rb, re;
  if (FL == CHS_DENSE) {
    rb = vx.dstart[base + k0];
    re = vx.dstart[base + k1 + 1];
  } else {
    // one probe of the column directory, then the column's voxels (sorted
    // by key) bound the range: the first with k >= k0, the first with k > k1
    uint64_t h = mix64(base) & vx.cmask;
    int2 cr = make_int2(0, 0);
    while (true) {
      const uint64_t ck = vx.ckeys[h];
      if (ck == base) {
        cr = vx.cvals[h];
        break;
      }
      if (ck == kEmptyKey) return;
      h = (h + 1) & vx.cmask;
    }
    if (cr.x < 0 || cr.y > vx.M || cr.x >= cr.y) return;
    int32_t lo = cr.x, hi = cr.y;
    const uint64_t kb = base + (uint64_t)k0, ke = base + (uint64_t)k1;
    while (lo < hi) {  // first id with key >= kb
      const int32_t mid = (lo + hi) >> 1;
      if (vx.ukeys[mid] < kb) lo = mid + 1;
      else hi = mid;
    }
    const int32_t u0 = lo;
    hi = cr.y;
    while (lo < hi) {  // first id with key > ke
      const int32_t mid = (lo + hi) >> 1;
      if (vx.ukeys[mid] <= ke) lo = mid + 1;
      else hi = mid;
    }
    if (lo == u0) return;
    rb = vx.ustart[u0];
    re = vx.ustart[lo];
  }
  if (rb < 0) rb = 0;
  if (re > vx.npts) re = (int32_t)vx.npts;
  if (re > rb) {
    *b = rb;
    *e = re;
  }
}

// The stored points seen through the constant address space: the index
// never changes during a search, and loads from this space at wave-uniform
// addresses are issued by the scalar unit even in kernels that also store
// (where the compiler cannot prove a global pointer read-only).
typedef float f4v __attribute__((ext_vector_type(4)));
typedef const f4v __attribute__((address_space(4)))* const_pts;
__device__ __forceinline__ const_pts as_const(const float4* p) { return (const_pts)p; }
__device__ __forceinline__ float4 load_const(const_pts p, int32_t i) {
  const f4v v = p[i];
  return make_float4(v.x, v.y, v.z, v.w);
}

// Block index remapped so that consecutive logical blocks run on the same
// XCD (the hardware deals blocks round-robin over the 8 XCDs, each with its
// own L2): spatially adjacent query tiles then share an L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  constexpr uint32_t X = 8;
  const uint32_t per = nb / X, rem = nb % X;
  const uint32_t x = b % X, i = b / X;
  // XCD x owns logical blocks [x*per + min(x, rem), ...)
  return x * per + (x < rem ? x : rem) + i;
}

// ---------------------------------------------------------------- primitives
// Exclusive prefix sum of n values into out[0..n], out[n] = total.
chs_status exclusive_scan_i32_i32(const Alloc& al, const int32_t* in, int32_t* out, int64_t n);
chs_status exclusive_scan_i32_i64(const Alloc& al, const int32_t* in, int64_t* out, int64_t n);

// Stable LSD radix sort of (key, value) pairs on bits [0, bits).  The result
// ends in (keys, vals); (tk, tv) are scratch of the same size.
chs_status radix_sort_u32(const Alloc& al, uint32_t* keys, uint32_t* vals, uint32_t* tk,
                          uint32_t* tv, int64_t n, int bits);
chs_status radix_sort_u64(const Alloc& al, uint64_t* keys, uint32_t* vals, uint64_t* tk,
                          uint32_t* tv, int64_t n, int bits);

// Hilbert index of (x, y) on a 2^m x 2^m grid.
__device__ __forceinline__ uint64_t hilbert2(uint32_t x, uint32_t y, int m) {
  uint64_t d = 0;
  for (int b = m - 1; b >= 0; --b) {
    const uint32_t s = 1u << b;
    const uint32_t rx = (x & s) ? 1u : 0u;
    const uint32_t ry = (y & s) ? 1u : 0u;
    d += (uint64_t)s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = s - 1 - (x & (s - 1));
        y = s - 1 - (y & (s - 1));
      } else {
        x &= s - 1;
        y &= s - 1;
      }
      uint32_t t = x;
      x = y;
      y = t;
    } else {
      x &= s - 1;
      y &= s - 1;
    }
  }
  return d;
}

// Processing order of a query batch: centres as float4 (x, y, z recentred
// FP32, caller index in w), sorted along a Hilbert curve over the (i, j)
// columns so that 64 consecutive queries are spatial neighbours.
struct QueryPlan {
  Buf q4;
  const float4* q = nullptr;
  int64_t nq = 0;
  int64_t nwaves = 0;
  const int32_t* wave_tile = nullptr;   // batched: tile, first query of each wave
  const int32_t* wave_start = nullptr;
  const int32_t* tile_qend = nullptr;   //   and the end of each tile's queries
  Buf wt, ws, qe;                       // per-tile query sets: those tables
  explicit QueryPlan(const Alloc* al) : q4(al), wt(al), ws(al), qe(al) {}
};
chs_status plan_queries(chs_index ix, const chs_queries* qs, QueryPlan* plan, hipStream_t stream);
chs_status plan_every_point(chs_index ix, hipStream_t stream);

// Host validation of a query batch against the index.
chs_status check_queries(chs_index ix, const chs_queries* qs);

// chs_knn with the temporaries taken from `al` (validates its arguments).
chs_status knn_impl(chs_index ix, const chs_queries* qs, int32_t k, float r_max, int32_t* idx,
                    float* d2, const Alloc& al, hipStream_t stream, int64_t* visited = nullptr);

int ceil_log2(uint64_t v);

}  // namespace chs
