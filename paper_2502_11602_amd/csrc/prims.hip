// Device-wide primitives: error state, allocation, exclusive scan and a
// stable LSD radix sort (a sequence of stable counting sorts on 8-bit
// digits).
#include <cstdarg>

#include "common.h"

#pragma clang fp contract(off)

namespace chs {

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

// ---------------------------------------------------------------- memory
void* Alloc::get(size_t bytes) const {
  if (bytes == 0) bytes = 256;
  if (has) return a.alloc(bytes, a.ctx);
  void* p = nullptr;
  if (hipMallocAsync(&p, bytes, stream) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void Alloc::put(void* p) const {
  if (!p) return;
  if (has) {
    a.free(p, a.ctx);
  } else {
    (void)hipFreeAsync(p, stream);
  }
}

chs_status Buf::alloc(size_t nbytes) {
  release();
  p = al->get(nbytes);
  if (!p) {
    set_error("allocator returned NULL for %zu bytes", nbytes);
    return CHS_E_NOMEM;
  }
  bytes = nbytes;
  return CHS_OK;
}

int ceil_log2(uint64_t v) {
  int b = 0;
  while (b < 64 && (1ull << b) < v) ++b;
  return b;
}

// ---------------------------------------------------------------- scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

template <class T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* total) {
  // wave-level inclusive scan, then a scan over the 4 wave totals in LDS
  __shared__ T s_w[kScanThreads / kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  T x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) s_w[w] = x;
  __syncthreads();
  T base = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kScanThreads / kWave; ++i) {
    T t = s_w[i];
    if (i < w) base += t;
    all += t;
  }
  __syncthreads();
  *total = all;
  return base + x - v;
}

template <class Tin, class Tout>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const Tin* __restrict__ in,
                                                              Tout* __restrict__ part, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  Tout s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += (Tout)in[base + i];
  Tout tot;
  (void)block_exclusive_sum<Tout>(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// out[i] = offset[block] + exclusive prefix within the block; the block that
// holds the last element also writes out[n] = grand total.
template <class Tin, class Tout>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const Tin* __restrict__ in,
                                                             Tout* __restrict__ out, int64_t n,
                                                             const Tout* __restrict__ offs) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  Tout v[kScanItems];
  Tout s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? (Tout)in[base + i] : (Tout)0;
    s += v[i];
  }
  Tout tot;
  Tout run = block_exclusive_sum<Tout>(s, &tot) + (offs ? offs[blockIdx.x] : (Tout)0);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  const int64_t tile_end = (int64_t)(blockIdx.x + 1) * kScanTile;
  if (threadIdx.x == kScanThreads - 1 && tile_end >= n) {
    // this is the last block: run now equals the grand total
    out[n] = run;
  }
}

template <class T>
__global__ void k_store_zero(T* out) {
  if (threadIdx.x == 0) *out = (T)0;
}

template <class Tin, class Tout>
static chs_status scan_impl(const Alloc& al, const Tin* in, Tout* out, int64_t n) {
  if (n <= 0) {
    // a kernel rather than a memset, so that captured graphs replay it
    k_store_zero<Tout><<<1, kWave, 0, al.stream>>>(out);
    CHS_LAUNCH_CHECK();
    return CHS_OK;
  }
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    k_scan_apply<Tin, Tout><<<1, kScanThreads, 0, al.stream>>>(in, out, n, nullptr);
    CHS_LAUNCH_CHECK();
    return CHS_OK;
  }
  Buf part(&al), offs(&al);
  CHS_TRY(part.alloc(sizeof(Tout) * nb));
  CHS_TRY(offs.alloc(sizeof(Tout) * (nb + 1)));
  k_scan_reduce<Tin, Tout><<<(unsigned)nb, kScanThreads, 0, al.stream>>>(in, part.as<Tout>(), n);
  CHS_LAUNCH_CHECK();
  CHS_TRY((scan_impl<Tout, Tout>(al, part.as<Tout>(), offs.as<Tout>(), nb)));
  k_scan_apply<Tin, Tout><<<(unsigned)nb, kScanThreads, 0, al.stream>>>(in, out, n, offs.as<Tout>());
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}

chs_status exclusive_scan_i32_i32(const Alloc& al, const int32_t* in, int32_t* out, int64_t n) {
  return scan_impl<int32_t, int32_t>(al, in, out, n);
}
chs_status exclusive_scan_i32_i64(const Alloc& al, const int32_t* in, int64_t* out, int64_t n) {
  return scan_impl<int32_t, int64_t>(al, in, out, n);
}

// ---------------------------------------------------------------- radix sort
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;  // 4096 items per block
constexpr int kDigits = 256;

template <class K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K* __restrict__ keys, int64_t n,
                                                             int shift, int nbits,
                                                             int32_t* __restrict__ hist,
                                                             int64_t nblocks) {
  __shared__ int32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t mask = (1u << nbits) - 1u;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & mask], 1);
  }
  __syncthreads();
  // digit-major layout: an exclusive scan over it gives every (digit, block)
  // its first output position
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

template <class K>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n, int shift, int nbits,
    const int32_t* __restrict__ offs, int64_t nblocks) {
  __shared__ int32_t s_run[kDigits];
  __shared__ int32_t s_wc[kSortThreads / kWave][kDigits];
  const int tid = threadIdx.x, w = tid / kWave;
  const uint32_t mask = (1u << nbits) - 1u;
  s_run[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint64_t lt = lanemask_lt();
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + tid;
    const bool valid = i < n;
    K key = valid ? kin[i] : (K)0;
    uint32_t val = valid ? vin[i] : 0u;
    const uint32_t d = (uint32_t)(key >> shift) & mask;
#pragma unroll
    for (int q = 0; q < kSortThreads / kWave; ++q) s_wc[q][tid] = 0;
    __syncthreads();
    // lanes of this wave holding the same digit (wave-wide multi-split)
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) s_wc[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int32_t pos = s_run[d] + rank;
      for (int q = 0; q < w; ++q) pos += s_wc[q][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int q = 0; q < kSortThreads / kWave; ++q) add += s_wc[q][tid];
    s_run[tid] += add;
    __syncthreads();
  }
}

template <class K>
static chs_status radix_impl(const Alloc& al, K* keys, uint32_t* vals, K* tk, uint32_t* tv,
                             int64_t n, int bits) {
  if (n <= 1 || bits <= 0) return CHS_OK;
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  Buf hist(&al), offs(&al);
  CHS_TRY(hist.alloc(sizeof(int32_t) * nb * kDigits));
  CHS_TRY(offs.alloc(sizeof(int32_t) * (nb * kDigits + 1)));
  K* src_k = keys;
  uint32_t* src_v = vals;
  K* dst_k = tk;
  uint32_t* dst_v = tv;
  for (int shift = 0; shift < bits; shift += 8) {
    const int nbits = (bits - shift) < 8 ? (bits - shift) : 8;
    k_radix_hist<K><<<(unsigned)nb, kSortThreads, 0, al.stream>>>(src_k, n, shift, nbits,
                                                                  hist.as<int32_t>(), nb);
    CHS_LAUNCH_CHECK();
    CHS_TRY(exclusive_scan_i32_i32(al, hist.as<int32_t>(), offs.as<int32_t>(), nb * kDigits));
    k_radix_scatter<K><<<(unsigned)nb, kSortThreads, 0, al.stream>>>(
        src_k, src_v, dst_k, dst_v, n, shift, nbits, offs.as<int32_t>(), nb);
    CHS_LAUNCH_CHECK();
    K* t1 = src_k; src_k = dst_k; dst_k = t1;
    uint32_t* t2 = src_v; src_v = dst_v; dst_v = t2;
  }
  if (src_k != keys) {
    CHS_HIP(hipMemcpyAsync(keys, src_k, sizeof(K) * n, hipMemcpyDeviceToDevice, al.stream));
    CHS_HIP(hipMemcpyAsync(vals, src_v, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, al.stream));
  }
  return CHS_OK;
}

chs_status radix_sort_u32(const Alloc& al, uint32_t* keys, uint32_t* vals, uint32_t* tk,
                          uint32_t* tv, int64_t n, int bits) {
  return radix_impl<uint32_t>(al, keys, vals, tk, tv, n, bits);
}
chs_status radix_sort_u64(const Alloc& al, uint64_t* keys, uint32_t* vals, uint64_t* tk,
                          uint32_t* tv, int64_t n, int bits) {
  return radix_impl<uint64_t>(al, keys, vals, tk, tv, n, bits);
}

}  // namespace chs

extern "C" const char* chs_last_error(void) { return chs::last_error(); }
extern "C" const char* chs_version(void) { return "chs 0.1.0 gfx950"; }
