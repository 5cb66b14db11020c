// k-NN without allocation (chs_knn_noalloc): the same search as chs_knn
// (Section 3.4.2), with every temporary carved from a fixed device array.
#include <mutex>
#include <vector>

#include "common.h"

namespace chs {

// ---------------------------------------------------------------- k-NN without allocation
// chs_knn_noalloc takes every temporary of chs_knn (the query plan with its
// sort buffers, the list of waves left to the second launch, the persistent
// work counter) from this fixed array instead of an allocator.  Each GPU holds its own copy for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress returns
// for the device, never through the symbol itself.
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int64_t kNoallocMaxQueries = (int64_t)1 << 19;  // plan: <= 57 bytes per query
// "every point" queries on a plain index: the wave list, 4 bytes per 64
// points, within the array
constexpr int64_t kNoallocMaxPoints = (int64_t)1 << 28;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct Arena {
  char* base;
  size_t cap, used;
};

// bump allocation inside the array; nothing is freed before the call ends
static void* arena_alloc(size_t bytes, void* ctx) {
  Arena* a = static_cast<Arena*>(ctx);
  const size_t off = (a->used + 255) & ~(size_t)255;
  if (off > a->cap || bytes > a->cap - off) return nullptr;
  a->used = off + bytes;
  return a->base + off;
}
static void arena_free(void*, void*) {}

static std::mutex g_scratch_mu;
static std::vector<char*> g_scratch;  // per device ordinal

// The array's device address on the current device (looked up once per
// device, with that device current).
static chs_status scratch_base(char** out) {
  int dev = 0;
  CHS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    CHS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned NULL for the scratch array");
      return CHS_E_DEVICE;
    }
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return CHS_OK;
}

}  // namespace chs

using namespace chs;

extern "C" chs_status chs_knn_noalloc(chs_index ix, const chs_queries* qs, int32_t k,
                                      float r_max, int32_t* idx, float* d2, hipStream_t st) {
  clear_error();
  CHS_TRY(check_queries(ix, qs));
  if ((qs->xyz || qs->point_idx) && qs->nq > kNoallocMaxQueries) {
    set_error("chs_knn_noalloc: nq = %lld index or coordinate queries exceed the limit %lld",
              (long long)qs->nq, (long long)kNoallocMaxQueries);
    return CHS_E_CAPACITY;
  }
  if (!qs->xyz && !qs->point_idx && ix->ntiles == 1 && !ix->persistent &&
      ix->n > kNoallocMaxPoints) {
    set_error("chs_knn_noalloc: every-point queries over %lld points exceed the limit %lld",
              (long long)ix->n, (long long)kNoallocMaxPoints);
    return CHS_E_CAPACITY;
  }
  char* base = nullptr;
  CHS_TRY(scratch_base(&base));
  Arena arena{base, kScratchBytes, 0};
  Alloc al;
  al.has = true;
  al.a.alloc = arena_alloc;
  al.a.free = arena_free;
  al.a.ctx = &arena;
  al.stream = st;
  return knn_impl(ix, qs, k, r_max, idx, d2, al, st);
}
