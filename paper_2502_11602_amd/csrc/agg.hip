// Gaussian-weighted neighbourhood aggregation over fixed neighbour lists
// and its gradient (a project addition on top of the index):
//   out[q,c] = sum_t w_qt f[j_t, c],   w_qt = exp(-|x_j - x_q|^2 / (2 sigma^2)),
//   x_q = x[qidx[q]], j_t = nbr[q,t] (negative entries are padding).
// The squared distance is the unfused sum (dx*dx + dy*dy) + dz*dz in the
// compute type.  Every sum runs in a fixed order and the backward pass uses
// no atomics: the (query, slot) pairs are regrouped by neighbour with a
// stable radix sort and reduced segment by segment, so results are
// bitwise reproducible.
//
// Work layout: one wavefront per query (forward, backward pair pass) or per
// point (backward point pass).  The lanes first take one list slot each and
// gather its neighbour, coordinates and weight in parallel; then they hold
// channels, and the wave walks the slots in order with the slot's values
// broadcast, reading each feature row with one coalesced load per 64
// channels, several rows in flight at a time.
#include <cmath>

#include "common.h"

#pragma clang fp contract(off)

namespace chs {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

enum { AGG_F32 = 0, AGG_F64 = 1, AGG_BF16 = 2 };

__device__ __forceinline__ float bf16_to_f32(uint16_t v) {
  return __uint_as_float((uint32_t)v << 16);
}
// round to nearest even
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <class TF, class TA>
__device__ __forceinline__ TA load_f(const TF* p, int64_t i);
template <>
__device__ __forceinline__ float load_f<float, float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ double load_f<double, double>(const double* p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ float load_f<uint16_t, float>(const uint16_t* p, int64_t i) {
  return bf16_to_f32(p[i]);
}

template <class TF, class TA>
__device__ __forceinline__ void store_f(TF* p, int64_t i, TA v);
template <>
__device__ __forceinline__ void store_f<float, float>(float* p, int64_t i, float v) { p[i] = v; }
template <>
__device__ __forceinline__ void store_f<double, double>(double* p, int64_t i, double v) { p[i] = v; }
template <>
__device__ __forceinline__ void store_f<uint16_t, float>(uint16_t* p, int64_t i, float v) {
  p[i] = f32_to_bf16(v);
}

__device__ __forceinline__ float gexp(float v) { return expf(v); }
__device__ __forceinline__ double gexp(double v) { return exp(v); }

template <class TA>
__device__ __forceinline__ TA wave_sum(TA v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// value of lane src (src uniform)
__device__ __forceinline__ int32_t lane_get(int32_t v, int src) {
  return __builtin_amdgcn_readlane(v, src);
}
__device__ __forceinline__ float lane_get(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_get(double v, int src) {
  const int64_t b = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)b, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)((uint64_t)b >> 32), src);
  return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}

// slots walked per step: their feature rows are loaded together
constexpr int kRows = 4;

// the next up to kRows set bits of m (ascending), removed from m
__device__ __forceinline__ void take_slots(uint64_t& m, int (&src)[kRows], bool (&ok)[kRows]) {
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    ok[u] = m != 0;
    src[u] = ok[u] ? __builtin_ctzll(m) : 0;
    m &= m - 1;
  }
}

template <class TX, class TA>
__device__ __forceinline__ TA sqdist3(const TX* __restrict__ x, int64_t j, TA qx, TA qy, TA qz) {
  const TA dx = (TA)x[j * 3 + 0] - qx, dy = (TA)x[j * 3 + 1] - qy, dz = (TA)x[j * 3 + 2] - qz;
  return (dx * dx + dy * dy) + dz * dz;
}

struct AggArgs {
  const void* x;
  const int32_t* qidx;
  const int32_t* nbr;
  int64_t N, Q;
  int32_t K, C;
  double inv2s2;  // 1 / (2 sigma^2)
  double invs2;   // 1 / sigma^2
};

// ---------------------------------------------------------------- forward
// out[q, c] accumulates w * f[j, c] over the valid slots in slot order.
template <class TX, class TF, class TA>
__global__ __launch_bounds__(kThreads) void k_agg_fwd(AggArgs A, const TF* __restrict__ f,
                                                      TF* __restrict__ out) {
  const int lane = lane_id();
  const int64_t q = (int64_t)blockIdx.x * kWaves + first_lane((int32_t)(threadIdx.x / kWave));
  if (q >= A.Q) return;
  const TX* __restrict__ x = static_cast<const TX*>(A.x);
  const int64_t iq = A.qidx[q];
  const bool qok = iq >= 0 && iq < A.N;
  const TA qx = qok ? (TA)x[iq * 3] : (TA)0, qy = qok ? (TA)x[iq * 3 + 1] : (TA)0,
           qz = qok ? (TA)x[iq * 3 + 2] : (TA)0;
  const TA i2 = (TA)A.inv2s2;
  for (int c0 = 0; c0 < A.C; c0 += kWave) {
    const int c = c0 + lane;
    const bool cin = c < A.C;
    TA acc = 0;
    for (int t0 = 0; qok && t0 < A.K; t0 += kWave) {
      // lane l: slot t0 + l, its neighbour and weight
      const int t = t0 + lane;
      int32_t jl = -1;
      TA wl = 0;
      if (t < A.K) {
        const int64_t jj = A.nbr[q * A.K + t];
        if (jj >= 0 && jj < A.N) {
          jl = (int32_t)jj;
          wl = gexp(-(sqdist3<TX, TA>(x, jj, qx, qy, qz) * i2));
        }
      }
      uint64_t m = __ballot(jl >= 0);
      while (m) {
        int src[kRows];
        bool ok[kRows];
        take_slots(m, src, ok);
        // (broadcasts stay outside the per-lane channel test)
        int32_t jv[kRows];
        TA wv[kRows], fv[kRows];
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
          jv[u] = lane_get(jl, src[u]);
          wv[u] = lane_get(wl, src[u]);
          fv[u] = (ok[u] && cin) ? load_f<TF, TA>(f, (int64_t)jv[u] * A.C + c) : (TA)0;
        }
#pragma unroll
        for (int u = 0; u < kRows; ++u)
          if (ok[u] && cin) acc += wv[u] * fv[u];
      }
    }
    if (cin) store_f<TF, TA>(out, q * A.C + c, acc);
  }
}

// ---------------------------------------------------------------- backward
// pass 1, one wave per query: per pair (q, t) the weight w and the scalar
// s = (sum_c g[q,c] f[j,c]) w / sigma^2; the centre-role gradient
// gq[q] = sum_t s (x_j - x_q) in slot order; and the sort keys regrouping
// pairs by j.
template <class TX, class TF, class TA>
__global__ __launch_bounds__(kThreads) void k_agg_bwd_pairs(AggArgs A, const TF* __restrict__ f,
                                                            const TF* __restrict__ g,
                                                            TA* __restrict__ pw, TA* __restrict__ ps,
                                                            TA* __restrict__ gq,
                                                            uint32_t* __restrict__ key,
                                                            uint32_t* __restrict__ val) {
  const int lane = lane_id();
  const int64_t q = (int64_t)blockIdx.x * kWaves + first_lane((int32_t)(threadIdx.x / kWave));
  if (q >= A.Q) return;
  const TX* __restrict__ x = static_cast<const TX*>(A.x);
  const int64_t iq = A.qidx[q];
  const bool qok = iq >= 0 && iq < A.N;
  const TA qx = qok ? (TA)x[iq * 3] : (TA)0, qy = qok ? (TA)x[iq * 3 + 1] : (TA)0,
           qz = qok ? (TA)x[iq * 3 + 2] : (TA)0;
  const TA i2 = (TA)A.inv2s2, is2 = (TA)A.invs2;
  // the gradient row of q for the first 64 channels stays in registers
  const TA g0 = lane < A.C ? load_f<TF, TA>(g, q * A.C + lane) : (TA)0;
  TA cx = 0, cy = 0, cz = 0;
  for (int t0 = 0; t0 < A.K; t0 += kWave) {
    // lane l: slot t0 + l, its neighbour, offset and weight
    const int t = t0 + lane;
    const int64_t p = q * A.K + t;
    int32_t jl = -1;
    TA wl = 0, dxl = 0, dyl = 0, dzl = 0, sl = 0;
    if (t < A.K) {
      const int64_t jj = A.nbr[p];
      if (qok && jj >= 0 && jj < A.N) {
        jl = (int32_t)jj;
        dxl = (TA)x[jj * 3 + 0] - qx;
        dyl = (TA)x[jj * 3 + 1] - qy;
        dzl = (TA)x[jj * 3 + 2] - qz;
        wl = gexp(-(((dxl * dxl + dyl * dyl) + dzl * dzl) * i2));
      }
    }
    uint64_t m = __ballot(jl >= 0);
    while (m) {
      int src[kRows];
      bool ok[kRows];
      take_slots(m, src, ok);
      int32_t jv[kRows];
      TA a[kRows];
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        jv[u] = lane_get(jl, src[u]);
        a[u] = 0;
      }
      for (int c0 = 0; c0 < A.C; c0 += kWave) {
        const int c = c0 + lane;
        const TA gc = c0 == 0 ? g0 : (c < A.C ? load_f<TF, TA>(g, q * A.C + c) : (TA)0);
        TA fv[kRows];
#pragma unroll
        for (int u = 0; u < kRows; ++u)
          fv[u] = (ok[u] && c < A.C) ? load_f<TF, TA>(f, (int64_t)jv[u] * A.C + c) : (TA)0;
#pragma unroll
        for (int u = 0; u < kRows; ++u) a[u] += wave_sum(gc * fv[u]);
      }
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        if (!ok[u]) continue;
        const TA s = a[u] * lane_get(wl, src[u]) * is2;
        cx += s * lane_get(dxl, src[u]);
        cy += s * lane_get(dyl, src[u]);
        cz += s * lane_get(dzl, src[u]);
        if (lane == src[u]) sl = s;
      }
    }
    if (t < A.K) {
      pw[p] = wl;
      ps[p] = sl;
      key[p] = jl >= 0 ? (uint32_t)jl : (uint32_t)A.N;  // padding sorts last
      val[p] = (uint32_t)p;
    }
  }
  if (lane == 0) {
    gq[q * 3 + 0] = cx;
    gq[q * 3 + 1] = cy;
    gq[q * 3 + 2] = cz;
    key[A.Q * A.K + q] = qok ? (uint32_t)iq : (uint32_t)A.N;
    val[A.Q * A.K + q] = (uint32_t)q;
  }
}

// Segment starts of ascending keys: start[b] = number of keys below b for
// b in [0, nb], one binary search per bin (what a histogram and an exclusive
// scan give, without atomics: padding slots share one key, and atomics on it
// serialise).
__global__ __launch_bounds__(kThreads) void k_bin_starts(const uint32_t* __restrict__ key, int64_t n,
                                                         int64_t nb, int32_t* __restrict__ start) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b > nb) return;
  int64_t lo = 0, hi = n;  // first index whose key is >= b
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)key[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  start[b] = (int32_t)lo;
}

// pass 2, one wave per point j: neighbour-role sums over the pairs that name
// j (ascending pair order) and the centre-role sums over the queries
// centred on j (ascending query order).
template <class TX, class TF, class TA>
__global__ __launch_bounds__(kThreads) void k_agg_bwd_points(
    AggArgs A, const TF* __restrict__ g, const TA* __restrict__ pw, const TA* __restrict__ ps,
    const TA* __restrict__ gq, const uint32_t* __restrict__ pair_sorted,
    const int32_t* __restrict__ pstart, const uint32_t* __restrict__ cent_sorted,
    const int32_t* __restrict__ cstart, TX* __restrict__ gx, TF* __restrict__ gf) {
  const int lane = lane_id();
  const int64_t j = (int64_t)blockIdx.x * kWaves + first_lane((int32_t)(threadIdx.x / kWave));
  if (j >= A.N) return;
  const TX* __restrict__ x = static_cast<const TX*>(A.x);
  const TA xj = (TA)x[j * 3], yj = (TA)x[j * 3 + 1], zj = (TA)x[j * 3 + 2];
  const int32_t b = pstart[j], e = pstart[j + 1];
  TA ax = 0, ay = 0, az = 0;
  for (int c0 = 0; c0 < A.C; c0 += kWave) {
    const int c = c0 + lane;
    const bool cin = c < A.C;
    TA acc = 0;
    for (int32_t u0 = b; u0 < e; u0 += kWave) {
      // lane l: pair u0 + l, its centre, weight and (first chunk) the
      // coordinate term s (x_q - x_j)
      const int32_t u = u0 + lane;
      int32_t ql = 0;
      TA wl = 0, txl = 0, tyl = 0, tzl = 0;
      if (u < e) {
        const int64_t p = pair_sorted[u];
        ql = (int32_t)(p / A.K);
        wl = pw[p];
        if (c0 == 0) {
          const int64_t iq = A.qidx[ql];
          const TA s = ps[p];
          // d/dx_j of w = -w (x_j - x_q) / sigma^2
          txl = s * ((TA)x[iq * 3] - xj);
          tyl = s * ((TA)x[iq * 3 + 1] - yj);
          tzl = s * ((TA)x[iq * 3 + 2] - zj);
        }
      }
      const int n = e - u0 < kWave ? e - u0 : kWave;
      for (int v0 = 0; v0 < n; v0 += kRows) {
        // (broadcasts stay outside the per-lane channel test)
        TA gv[kRows], wv[kRows];
#pragma unroll
        for (int u1 = 0; u1 < kRows; ++u1) {
          const int v = v0 + u1 < n ? v0 + u1 : 0;
          const int32_t qv = lane_get(ql, v);
          wv[u1] = lane_get(wl, v);
          gv[u1] = (v0 + u1 < n && cin) ? load_f<TF, TA>(g, (int64_t)qv * A.C + c) : (TA)0;
        }
#pragma unroll
        for (int u1 = 0; u1 < kRows; ++u1) {
          if (v0 + u1 >= n) continue;
          if (cin) acc += wv[u1] * gv[u1];
          if (c0 == 0) {
            ax += lane_get(txl, v0 + u1);
            ay += lane_get(tyl, v0 + u1);
            az += lane_get(tzl, v0 + u1);
          }
        }
      }
    }
    if (cin) store_f<TF, TA>(gf, j * A.C + c, acc);
  }
  const int32_t cb = cstart[j], ce = cstart[j + 1];
  for (int32_t u = cb; u < ce; ++u) {
    const int64_t q = cent_sorted[u];
    ax += gq[q * 3];
    ay += gq[q * 3 + 1];
    az += gq[q * 3 + 2];
  }
  if (lane == 0) {
    gx[j * 3] = (TX)ax;
    gx[j * 3 + 1] = (TX)ay;
    gx[j * 3 + 2] = (TX)az;
  }
}

static unsigned blocks_for(int64_t waves) { return (unsigned)((waves + kWaves - 1) / kWaves); }

static chs_status check_agg(const void* x, const int32_t* qidx, const int32_t* nbr, int64_t N,
                            int64_t Q, int32_t K, const void* f, int32_t C, double sigma,
                            int32_t xdt, int32_t fdt) {
  if (!x || !f || (Q > 0 && (!qidx || !nbr))) {
    set_error("x, f, qidx or nbr is NULL");
    return CHS_E_INVALID;
  }
  // the backward regroups the Q*K pair slots (plus Q centre slots) with
  // int32 positions
  if (N < 1 || N > (int64_t)INT32_MAX - 1 || Q < 0 || K < 0 || C < 1 || K > (int64_t)INT32_MAX ||
      Q > (int64_t)INT32_MAX || Q * (int64_t)K + Q > (int64_t)INT32_MAX) {
    set_error("sizes out of range (N=%lld Q=%lld K=%d C=%d)", (long long)N, (long long)Q, K, C);
    return CHS_E_INVALID;
  }
  if (!(sigma > 0.0) || !std::isfinite(sigma)) {
    set_error("sigma must be finite and > 0");
    return CHS_E_INVALID;
  }
  const bool ok = (xdt == AGG_F32 && (fdt == AGG_F32 || fdt == AGG_BF16)) ||
                  (xdt == AGG_F64 && fdt == AGG_F64);
  if (!ok) {
    set_error("unsupported dtype pair (x %d, f %d): use (f32, f32), (f32, bf16) or (f64, f64)",
              xdt, fdt);
    return CHS_E_UNSUPPORTED;
  }
  return CHS_OK;
}

static AggArgs make_args(const void* x, const int32_t* qidx, const int32_t* nbr, int64_t N,
                         int64_t Q, int32_t K, int32_t C, double sigma) {
  AggArgs A;
  A.x = x;
  A.qidx = qidx;
  A.nbr = nbr;
  A.N = N;
  A.Q = Q;
  A.K = K;
  A.C = C;
  A.inv2s2 = 1.0 / (2.0 * sigma * sigma);
  A.invs2 = 1.0 / (sigma * sigma);
  return A;
}

template <class TX, class TF, class TA>
static chs_status bwd_impl(const Alloc& al, const AggArgs& A, const TF* f, const TF* g, TX* gx,
                           TF* gf) {
  hipStream_t st = al.stream;
  const int64_t np = A.Q * (int64_t)A.K, nk = np + A.Q;
  Buf pw(&al), ps(&al), gq(&al), key(&al), val(&al), tk(&al), tv(&al), start(&al);
  CHS_TRY(pw.alloc(sizeof(TA) * (np > 0 ? np : 1)));
  CHS_TRY(ps.alloc(sizeof(TA) * (np > 0 ? np : 1)));
  CHS_TRY(gq.alloc(sizeof(TA) * 3 * (A.Q > 0 ? A.Q : 1)));
  CHS_TRY(key.alloc(sizeof(uint32_t) * (nk > 0 ? nk : 1)));
  CHS_TRY(val.alloc(sizeof(uint32_t) * (nk > 0 ? nk : 1)));
  CHS_TRY(tk.alloc(sizeof(uint32_t) * (nk > 0 ? nk : 1)));
  CHS_TRY(tv.alloc(sizeof(uint32_t) * (nk > 0 ? nk : 1)));
  // bins 0..N-1 for points, N for padding; pairs first, then centres
  const int64_t nb = A.N + 1;
  CHS_TRY(start.alloc(sizeof(int32_t) * 2 * (nb + 1)));
  if (A.Q > 0) {
    k_agg_bwd_pairs<TX, TF, TA><<<blocks_for(A.Q), kThreads, 0, st>>>(
        A, f, g, pw.as<TA>(), ps.as<TA>(), gq.as<TA>(), key.as<uint32_t>(), val.as<uint32_t>());
    CHS_LAUNCH_CHECK();
  }
  const int bits = ceil_log2((uint64_t)nb);
  uint32_t* K = key.as<uint32_t>();
  uint32_t* V = val.as<uint32_t>();
  // stable regrouping: pairs by neighbour, centres by centre point
  CHS_TRY(radix_sort_u32(al, K, V, tk.as<uint32_t>(), tv.as<uint32_t>(), np, bits));
  CHS_TRY(radix_sort_u32(al, K + np, V + np, tk.as<uint32_t>(), tv.as<uint32_t>(), A.Q, bits));
  int32_t* S0 = start.as<int32_t>();
  const unsigned sb = (unsigned)((nb + 1 + kThreads - 1) / kThreads);
  k_bin_starts<<<sb, kThreads, 0, st>>>(K, np, nb, S0);
  CHS_LAUNCH_CHECK();
  k_bin_starts<<<sb, kThreads, 0, st>>>(K + np, A.Q, nb, S0 + nb + 1);
  CHS_LAUNCH_CHECK();
  k_agg_bwd_points<TX, TF, TA><<<blocks_for(A.N), kThreads, 0, st>>>(
      A, g, pw.as<TA>(), ps.as<TA>(), gq.as<TA>(), V, S0, V + np, S0 + nb + 1, gx, gf);
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}

}  // namespace chs

using namespace chs;

extern "C" chs_status chs_gauss_agg_fwd(const void* x, const int32_t* qidx, const int32_t* nbr,
                                        int64_t N, int64_t Q, int32_t K, const void* f, int32_t C,
                                        double sigma, int32_t x_dtype, int32_t f_dtype, void* out,
                                        hipStream_t st) {
  clear_error();
  CHS_TRY(check_agg(x, qidx, nbr, N, Q, K, f, C, sigma, x_dtype, f_dtype));
  if (Q > 0 && !out) {
    set_error("out is NULL");
    return CHS_E_INVALID;
  }
  if (Q == 0) return CHS_OK;
  const AggArgs A = make_args(x, qidx, nbr, N, Q, K, C, sigma);
  if (x_dtype == AGG_F64)
    k_agg_fwd<double, double, double><<<blocks_for(Q), kThreads, 0, st>>>(
        A, static_cast<const double*>(f), static_cast<double*>(out));
  else if (f_dtype == AGG_BF16)
    k_agg_fwd<float, uint16_t, float><<<blocks_for(Q), kThreads, 0, st>>>(
        A, static_cast<const uint16_t*>(f), static_cast<uint16_t*>(out));
  else
    k_agg_fwd<float, float, float><<<blocks_for(Q), kThreads, 0, st>>>(
        A, static_cast<const float*>(f), static_cast<float*>(out));
  CHS_LAUNCH_CHECK();
  return CHS_OK;
}

extern "C" chs_status chs_gauss_agg_bwd(const void* x, const int32_t* qidx, const int32_t* nbr,
                                        int64_t N, int64_t Q, int32_t K, const void* f, int32_t C,
                                        double sigma, int32_t x_dtype, int32_t f_dtype,
                                        const void* grad_out, void* grad_x, void* grad_f,
                                        const chs_allocator* alloc, hipStream_t st) {
  clear_error();
  CHS_TRY(check_agg(x, qidx, nbr, N, Q, K, f, C, sigma, x_dtype, f_dtype));
  if ((Q > 0 && !grad_out) || !grad_x || !grad_f) {
    set_error("grad_out, grad_x or grad_f is NULL");
    return CHS_E_INVALID;
  }
  if (alloc && (!alloc->alloc || !alloc->free)) {
    set_error("allocator callbacks are NULL");
    return CHS_E_INVALID;
  }
  Alloc al;
  al.stream = st;
  if (alloc) {
    al.a = *alloc;
    al.has = true;
  }
  const AggArgs A = make_args(x, qidx, nbr, N, Q, K, C, sigma);
  if (x_dtype == AGG_F64)
    return bwd_impl<double, double, double>(al, A, static_cast<const double*>(f),
                                            static_cast<const double*>(grad_out),
                                            static_cast<double*>(grad_x),
                                            static_cast<double*>(grad_f));
  if (f_dtype == AGG_BF16)
    return bwd_impl<float, uint16_t, float>(al, A, static_cast<const uint16_t*>(f),
                                            static_cast<const uint16_t*>(grad_out),
                                            static_cast<float*>(grad_x),
                                            static_cast<uint16_t*>(grad_f));
  return bwd_impl<float, float, float>(al, A, static_cast<const float*>(f),
                                       static_cast<const float*>(grad_out),
                                       static_cast<float*>(grad_x), static_cast<float*>(grad_f));
}
