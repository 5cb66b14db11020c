// CPU oracle for the Cheesemap grid index (Laso & Yermo, arXiv 2502.11602).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
// GPU library is checked against.  Only the test suite, the smoke check and
// the CPU-baseline leg of the benchmark load it; the GPU library never links,
// includes or calls anything here, and nothing here comes from the GPU side.
//
// What it computes, step by step, in the paper's order and notation:
//   * bounding box p-, p+ of the cloud                      (Section 3.1, Eq. 1-2)
//   * grid size n_a = floor((p+_a - p-_a)/s) + 1            (Section 3.2, Eq. 3)
//   * point -> voxel (i,j,k) = floor((p_a - p-_a)/s)        (Section 3.2, Eq. 5)
//   * global voxel index g = i*n_y*n_z + j*n_z + k          (Section 3.3.1, Eq. 6-7)
//   * reordering of the points by voxel (counting sort)     (Section 3.5, "Reordering")
//   * dense / sparse / mixed voxel storage                  (Section 3.3.1-3.3.3)
//   * kernel-based search: sphere, cube, cylinder           (Section 3.4.1, Alg. 1;
//                                                            Section 2)
//   * k-NN search with taboo box, sorted capped candidate
//     list and density-based radius growth                  (Section 3.4.2, Alg. 2;
//                                                            Section 3.5)
//   * Gaussian-weighted neighbourhood aggregation and its analytic gradient,
//     in FP64 (a project addition, not in the paper).
//
// Readings where the paper is silent (the same list is kept with the design
// notes): coordinates are recentred to p- in FP64 and stored as FP32; the
// squared distance is the unfused FP32 sum (dx*dx + dy*dy) + dz*dz; the sphere
// is closed (D <= fl32(r*r)); voxel indices are 0-based; the voxel of a value v
// is min(n_a - 1, floor(v / s_a)) with an IEEE FP64 divide; points inside a
// voxel keep ascending original index; k-NN ties are broken by original
// index; the density-growth radius is (k / rho)^(1/3) as in Alg. 2, replaced
// by r + s when it would not grow; a zero starting radius becomes s.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared -pthread
// (no fast-math: every FP32 operation must round as IEEE binary32).

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

constexpr double kPadRel = 1.0 / 262144.0;   // 2^-18 relative box padding
constexpr double kPadAbs = 8.673617379884035e-19;  // 2^-60 absolute floor

struct Range {
  int64_t begin = 0, end = 0;
};

enum Flavor { DENSE = 0, SPARSE = 1, MIXED = 2 };

struct OIndex {
  int dims = 3;
  int flavor = DENSE;
  int mixed_pct = 80;
  double s[3] = {1, 1, 1};
  int64_t n = 0;
  double origin[3] = {0, 0, 0};
  float max32[3] = {0, 0, 0};
  int64_t ncell[3] = {1, 1, 1};
  std::vector<float> x32[3];    // recentred FP32 coordinates, original order
  std::vector<uint64_t> key;    // voxel global index per point, original order
  std::vector<int32_t> perm;    // perm[pos] = original index of the pos-th stored point
  std::vector<float> sx[3];     // coordinates in stored (voxel) order
  std::vector<uint64_t> ukeys;  // ascending non-empty voxel indices
  std::vector<int64_t> ustart;  // their first stored positions, plus N at the end
  // dense flavor: voxel g holds [dstart[g], dstart[g+1])
  std::vector<int64_t> dstart;
  // sparse flavor (and sparse slices of the mixed flavor): hashmap g -> range
  std::unordered_map<uint64_t, Range> hmap;
  // mixed flavor: per z-slice non-empty count, dense flag and dense tables
  std::vector<int64_t> slice_nonempty;
  std::vector<uint8_t> slice_dense;
  std::vector<std::vector<Range>> slice_table;

  uint64_t ncells() const { return (uint64_t)ncell[0] * ncell[1] * ncell[2]; }
};

// Eq. 5 with the 0-based, clamped reading: voxel coordinate of a recentred
// value along one axis.  Used for the points (v >= 0) when building.
inline int64_t voxel_of(double v, double s, int64_t n) {
  double c = std::floor(v / s);
  if (c > (double)(n - 1)) return n - 1;
  if (c < 0) return 0;
  return (int64_t)c;
}

// Eq. 7 (Eq. 6 when n_z = 1).
inline uint64_t global_index(int64_t i, int64_t j, int64_t k, const int64_t* nc) {
  return ((uint64_t)i * (uint64_t)nc[1] + (uint64_t)j) * (uint64_t)nc[2] + (uint64_t)k;
}

// Squared distance, FP32, unfused, fixed association order.
// Compiled with -ffp-contract=off, so no multiply-add is fused.
static_assert(FLT_EVAL_METHOD == 0, "FP32 expressions must be evaluated in FP32");
inline float sqdist(float qx, float qy, float qz, float px, float py, float pz) {
  const float dx = qx - px;
  const float dy = qy - py;
  const float dz = qz - pz;
  return (dx * dx + dy * dy) + dz * dz;
}

// Does voxel (i,j,k) exist, and which stored points does it hold?
// Dense: every voxel exists (Section 3.5, "Voxels in dense Cheesemap").
// Sparse: hashmap keyed by g (Section 3.3.2).  Mixed: per z-slice table or
// hashmap (Section 3.3.3).
bool lookup(const OIndex& ix, int64_t i, int64_t j, int64_t k, Range* out) {
  uint64_t g = global_index(i, j, k, ix.ncell);
  if (ix.flavor == DENSE) {
    out->begin = ix.dstart[g];
    out->end = ix.dstart[g + 1];
    return true;
  }
  if (ix.flavor == MIXED && ix.slice_dense[k]) {
    *out = ix.slice_table[k][(size_t)(i * ix.ncell[1] + j)];
    return true;  // a dense slice stores all its voxels, empty ones too
  }
  auto it = ix.hmap.find(g);
  if (it == ix.hmap.end()) return false;
  *out = it->second;
  return true;
}

// Voxel index range covered by the real interval [lo, hi] along one axis,
// clamped to the grid (empty when the interval misses the grid).
bool axis_range(double lo, double hi, double s, int64_t n, int64_t* a, int64_t* b) {
  double clo = std::floor(lo / s), chi = std::floor(hi / s);
  if (chi < 0 || clo > (double)(n - 1)) return false;
  *a = clo < 0 ? 0 : (int64_t)clo;
  *b = chi > (double)(n - 1) ? n - 1 : (int64_t)chi;
  return true;
}

struct Box {
  int64_t lo[3], hi[3];
  bool empty;
};

// Search kernels (Section 3.4.1 and Section 2): a closed sphere, a cube
// (L-infinity ball, half side r) and a vertical cylinder (disc of radius r,
// z ignored).  Each gives a bounding box and an inside test (the paper's
// box() / is_inside() pair); Alg. 1 is the same for all of them.
enum Kernel { kSphere = 0, kCube = 1, kCylinder = 2 };

// Voxel box covering the bounding box of the kernel around c (Section
// 3.4.1, Eq. 8-9), padded by a relative 2^-18 (floor 2^-60) so that FP32
// rounding can never admit a point lying in a voxel outside the box.  The
// cylinder's box spans every z voxel.
Box kernel_box(const OIndex& ix, const double c[3], double r, int kernel = kSphere) {
  Box b;
  b.empty = false;
  double pad = std::max(r * (1.0 + kPadRel), kPadAbs);
  for (int a = 0; a < 3; ++a) {
    if (a == 2 && ix.dims == 2) {
      b.lo[2] = 0;
      b.hi[2] = 0;
      continue;
    }
    if (a == 2 && kernel == kCylinder) {
      b.lo[2] = 0;
      b.hi[2] = ix.ncell[2] - 1;
      continue;
    }
    if (!axis_range(c[a] - pad, c[a] + pad, ix.s[a], ix.ncell[a], &b.lo[a], &b.hi[a])) {
      b.empty = true;
      b.lo[a] = 0;
      b.hi[a] = -1;
    }
  }
  return b;
}

// The centre of query q; false when the query names no point of the cloud
// (an index outside [0, n)) or no place (a non-finite coordinate): such a
// query has no neighbours.
bool query_coords(const OIndex& ix, const int32_t* pidx, const double* qxyz, int64_t q,
                  float out[3]) {
  if (pidx) {
    int32_t p = pidx[q];
    if (p < 0 || (int64_t)p >= ix.n) return false;
    for (int a = 0; a < 3; ++a) out[a] = ix.x32[a][p];
  } else if (qxyz) {
    for (int a = 0; a < 3; ++a) {
      if (!std::isfinite(qxyz[q * 3 + a])) return false;
      out[a] = (float)(qxyz[q * 3 + a] - ix.origin[a]);
    }
  } else {
    for (int a = 0; a < 3; ++a) out[a] = ix.x32[a][q];
  }
  return true;
}

// is_inside for each kernel, in FP32 like the distance: differences
// fl32(c - p); sphere D <= fl32(r*r); cube |dx|, |dy|, |dz| <= r; cylinder
// fl32(dx*dx + dy*dy) <= fl32(r*r), unfused.
bool is_inside(int kernel, const float c[3], float px, float py, float pz, float r, float R) {
  if (kernel == kCube) {
    const float dx = c[0] - px, dy = c[1] - py, dz = c[2] - pz;
    return std::fabs(dx) <= r && std::fabs(dy) <= r && std::fabs(dz) <= r;
  }
  if (kernel == kCylinder) {
    const float dx = c[0] - px, dy = c[1] - py;
    const float dx2 = dx * dx, dy2 = dy * dy;
    const float h = dx2 + dy2;
    return h <= R;
  }
  return sqdist(c[0], c[1], c[2], px, py, pz) <= R;  // closed sphere
}

// ---- Alg. 1: kernel-based search -----------------------------------------
void radius_one(const OIndex& ix, const float c32[3], float r, std::vector<int32_t>& outv,
                int64_t* visited, int kernel = kSphere) {
  const float R = r * r;  // fl32(r*r)
  double c[3] = {c32[0], c32[1], c32[2]};
  Box b = kernel_box(ix, c, (double)r, kernel);
  int64_t nvis = 0;
  if (!b.empty) {
    for (int64_t i = b.lo[0]; i <= b.hi[0]; ++i)
      for (int64_t j = b.lo[1]; j <= b.hi[1]; ++j)
        for (int64_t k = b.lo[2]; k <= b.hi[2]; ++k) {
          Range rg;
          if (!lookup(ix, i, j, k, &rg)) continue;  // voxel does not exist
          ++nvis;
          for (int64_t p = rg.begin; p < rg.end; ++p)
            if (is_inside(kernel, c32, ix.sx[0][p], ix.sx[1][p], ix.sx[2][p], r, R))
              outv.push_back(ix.perm[p]);
        }
  }
  if (visited) *visited = nvis;
}

// ---- Alg. 2: k-NN search -----------------------------------------------
struct Cand {
  float d;
  int32_t id;
};
inline bool cand_less(const Cand& a, const Cand& b) {
  return a.d < b.d || (a.d == b.d && a.id < b.id);
}

// Sorted candidate list capped at k entries (Section 3.5, "Candidate list"):
// binary-search insertion, entries beyond k are dropped.
struct CappedList {
  int k;
  std::vector<Cand> v;
  explicit CappedList(int k_) : k(k_) { v.reserve((size_t)k_ + 1); }
  void insert(Cand c) {
    if ((int)v.size() == k && !cand_less(c, v.back())) return;
    auto pos = std::upper_bound(v.begin(), v.end(), c, cand_less);
    v.insert(pos, c);
    if ((int)v.size() > k) v.pop_back();
  }
};

// monotonic: grow the radius by the smallest voxel edge at every step
// instead of from the density of the candidates found (the baseline the
// paper compares its density growth with, Section 3.5); the result is the
// same, only the voxels visited differ.
void knn_one(const OIndex& ix, const float c32[3], int k, float r_max, int32_t* idx_out,
             float* d2_out, int64_t* visited, bool monotonic = false) {
  const double c[3] = {c32[0], c32[1], c32[2]};
  const int nax = ix.dims;
  double s_min = ix.s[0];
  for (int a = 1; a < nax; ++a) s_min = std::min(s_min, ix.s[a]);
  // initial radius: distance from c to the nearest wall of its voxel (Eq. 11)
  double r = INFINITY;
  for (int a = 0; a < nax; ++a) {
    int64_t v = voxel_of(c[a], ix.s[a], ix.ncell[a]);
    double lo = (double)v * ix.s[a], hi = (double)(v + 1) * ix.s[a];
    r = std::min(r, std::min(std::fabs(c[a] - lo), std::fabs(c[a] - hi)));
  }
  if (!(r > 0)) r = s_min;  // a centre on a wall would start at radius 0
  CappedList cand(k);
  Box taboo;  // visited voxels form a box (Section 3.5, "Taboo list")
  taboo.empty = true;
  int64_t nvis = 0;
  int64_t np_hat = 0;  // |P^|
  auto covers_grid = [&](const Box& b) {
    if (b.empty) return false;
    for (int a = 0; a < 3; ++a)
      if (b.lo[a] != 0 || b.hi[a] != ix.ncell[a] - 1) return false;
    return true;
  };
  auto in_taboo = [&](int64_t i, int64_t j, int64_t kk) {
    return !taboo.empty && i >= taboo.lo[0] && i <= taboo.hi[0] && j >= taboo.lo[1] &&
           j <= taboo.hi[1] && kk >= taboo.lo[2] && kk <= taboo.hi[2];
  };
  while (np_hat < k && !covers_grid(taboo)) {
    Box b = kernel_box(ix, c, r);
    if (!b.empty) {
      for (int64_t i = b.lo[0]; i <= b.hi[0]; ++i)
        for (int64_t j = b.lo[1]; j <= b.hi[1]; ++j)
          for (int64_t kk = b.lo[2]; kk <= b.hi[2]; ++kk) {
            if (in_taboo(i, j, kk)) continue;
            Range rg;
            if (!lookup(ix, i, j, kk, &rg)) continue;
            ++nvis;
            for (int64_t p = rg.begin; p < rg.end; ++p) {
              float D = sqdist(c32[0], c32[1], c32[2], ix.sx[0][p], ix.sx[1][p], ix.sx[2][p]);
              cand.insert(Cand{D, ix.perm[p]});
            }
          }
      taboo = b;  // boxes are nested because r only grows
    }
    // P^ = candidates within the current radius (Eq. 10)
    const float T = (float)(r * r);
    np_hat = 0;
    for (const Cand& e : cand.v)
      if (e.d <= T) ++np_hat;
    double r_new;
    if (np_hat > 0 && !monotonic) {
      double rho = (double)np_hat / ((4.0 / 3.0) * M_PI * r * r * r);  // Eq. 12
      r_new = std::cbrt((double)k / rho);                               // Alg. 2
      if (!(r_new > r)) r_new = r + s_min;  // density did not make it grow
    } else {
      r_new = r + s_min;  // monotonic growth
    }
    r = r_new;
  }
  const float Rmax = std::isinf(r_max) ? INFINITY : r_max * r_max;
  for (int t = 0; t < k; ++t) {
    if (t < (int)cand.v.size() && cand.v[t].d <= Rmax) {
      idx_out[t] = cand.v[t].id;
      d2_out[t] = cand.v[t].d;
    } else {
      idx_out[t] = -1;
      d2_out[t] = INFINITY;
    }
  }
  if (visited) *visited = nvis;
}

template <class F>
void parallel_for(int64_t n, int nthreads, F f) {
  if (nthreads <= 1 || n < 2 * nthreads) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=] { f(a, b); });
  }
  for (auto& x : th) x.join();
}

struct RadiusResult {
  std::vector<int32_t> nbr;
};

}  // namespace

extern "C" {

// status: 0 ok, 1 invalid argument, 3 capacity (dense table too large)
void* orc_build(const double* xyz, int64_t n, int dims, int flavor, const double* cell,
                int mixed_pct, int64_t max_dense_cells, int* status) {
  *status = 1;
  if (!xyz || n < 1 || n > INT32_MAX || (dims != 2 && dims != 3) || flavor < 0 || flavor > 2)
    return nullptr;
  for (int a = 0; a < 3; ++a)
    if (!(cell[a] > 0) || !std::isfinite(cell[a])) return nullptr;
  for (int64_t p = 0; p < n * 3; ++p)
    if (!std::isfinite(xyz[p])) return nullptr;
  OIndex* ix = new OIndex();
  ix->dims = dims;
  ix->flavor = flavor;
  ix->mixed_pct = mixed_pct;
  ix->n = n;
  for (int a = 0; a < 3; ++a) ix->s[a] = cell[a];
  // Eq. 1: p- (exact FP64 minimum), used as the origin
  for (int a = 0; a < 3; ++a) {
    double m = xyz[a];
    for (int64_t p = 1; p < n; ++p) m = std::min(m, xyz[p * 3 + a]);
    ix->origin[a] = m;
  }
  // recentre, store FP32; Eq. 2: p+ of the recentred cloud
  for (int a = 0; a < 3; ++a) {
    ix->x32[a].resize(n);
    float mx = 0.0f;
    for (int64_t p = 0; p < n; ++p) {
      float v = (float)(xyz[p * 3 + a] - ix->origin[a]);
      ix->x32[a][p] = v;
      mx = std::max(mx, v);
    }
    ix->max32[a] = mx;
  }
  // Eq. 3: n_a = floor((p+_a - p-_a) / s) + 1;  2D: one voxel along z
  for (int a = 0; a < 3; ++a)
    ix->ncell[a] = (int64_t)std::floor((double)ix->max32[a] / ix->s[a]) + 1;
  if (dims == 2) ix->ncell[2] = 1;
  const uint64_t ncells = ix->ncells();
  if (flavor == DENSE && (int64_t)ncells > max_dense_cells) {
    delete ix;
    *status = 3;
    return nullptr;
  }
  // Eq. 5 + Eq. 7: voxel key of every point
  ix->key.resize(n);
  for (int64_t p = 0; p < n; ++p) {
    int64_t v[3] = {0, 0, 0};
    for (int a = 0; a < dims; ++a) v[a] = voxel_of(ix->x32[a][p], ix->s[a], ix->ncell[a]);
    ix->key[p] = global_index(v[0], v[1], v[2], ix->ncell);
  }
  // counting sort by key: per-voxel counts, exclusive prefix sum, stable
  // scatter in original order (Section 3.5, "Reordering")
  std::map<uint64_t, int64_t> counts;
  for (int64_t p = 0; p < n; ++p) counts[ix->key[p]] += 1;
  ix->ukeys.reserve(counts.size());
  ix->ustart.reserve(counts.size() + 1);
  std::unordered_map<uint64_t, int64_t> cursor;
  cursor.reserve(counts.size() * 2);
  int64_t acc = 0;
  for (auto& kv : counts) {
    ix->ukeys.push_back(kv.first);
    ix->ustart.push_back(acc);
    cursor[kv.first] = acc;
    acc += kv.second;
  }
  ix->ustart.push_back(acc);
  ix->perm.assign(n, -1);
  for (int64_t p = 0; p < n; ++p) ix->perm[cursor[ix->key[p]]++] = (int32_t)p;
  for (int a = 0; a < 3; ++a) {
    ix->sx[a].resize(n);
    for (int64_t q = 0; q < n; ++q) ix->sx[a][q] = ix->x32[a][ix->perm[q]];
  }
  const int64_t M = (int64_t)ix->ukeys.size();
  // voxel storage
  if (flavor == DENSE) {
    // every voxel, empty or not: start table over all n_x*n_y*n_z voxels
    ix->dstart.assign(ncells + 1, 0);
    std::vector<int64_t> cnt(ncells, 0);
    for (int64_t u = 0; u < M; ++u) cnt[ix->ukeys[u]] = ix->ustart[u + 1] - ix->ustart[u];
    int64_t run = 0;
    for (uint64_t g = 0; g < ncells; ++g) {
      ix->dstart[g] = run;
      run += cnt[g];
    }
    ix->dstart[ncells] = run;
  } else {
    const int64_t nz = ix->ncell[2], nxy = ix->ncell[0] * ix->ncell[1];
    if (flavor == MIXED) {
      ix->slice_nonempty.assign(nz, 0);
      for (int64_t u = 0; u < M; ++u) ix->slice_nonempty[ix->ukeys[u] % (uint64_t)nz] += 1;
      ix->slice_dense.assign(nz, 0);
      ix->slice_table.resize(nz);
      for (int64_t k = 0; k < nz; ++k) {
        // a slice becomes dense once mixed_pct % of its voxels hold points
        if (100 * ix->slice_nonempty[k] >= (int64_t)mixed_pct * nxy) {
          ix->slice_dense[k] = 1;
          ix->slice_table[k].assign(nxy, Range{});
        }
      }
    }
    ix->hmap.reserve(M * 2);
    for (int64_t u = 0; u < M; ++u) {
      uint64_t g = ix->ukeys[u];
      Range rg{ix->ustart[u], ix->ustart[u + 1]};
      if (flavor == MIXED) {
        int64_t k = (int64_t)(g % (uint64_t)nz);
        if (ix->slice_dense[k]) {
          ix->slice_table[k][(size_t)(g / (uint64_t)nz)] = rg;
          continue;
        }
      }
      ix->hmap.emplace(g, rg);
    }
  }
  *status = 0;
  return ix;
}

void orc_free(void* h) { delete static_cast<OIndex*>(h); }

void orc_geometry(const void* h, double* origin, float* max32, int64_t* ncell) {
  const OIndex* ix = static_cast<const OIndex*>(h);
  for (int a = 0; a < 3; ++a) {
    origin[a] = ix->origin[a];
    max32[a] = ix->max32[a];
    ncell[a] = ix->ncell[a];
  }
}

int64_t orc_n_nonempty(const void* h) { return (int64_t) static_cast<const OIndex*>(h)->ukeys.size(); }

// x32 and sorted: SoA [3][n]
void orc_point_arrays(const void* h, float* x32, uint64_t* keys, int32_t* perm, float* sorted) {
  const OIndex* ix = static_cast<const OIndex*>(h);
  const int64_t n = ix->n;
  for (int a = 0; a < 3; ++a) {
    if (x32) std::memcpy(x32 + a * n, ix->x32[a].data(), n * sizeof(float));
    if (sorted) std::memcpy(sorted + a * n, ix->sx[a].data(), n * sizeof(float));
  }
  if (keys) std::memcpy(keys, ix->key.data(), n * sizeof(uint64_t));
  if (perm) std::memcpy(perm, ix->perm.data(), n * sizeof(int32_t));
}

void orc_cells(const void* h, uint64_t* ukeys, int64_t* ustart) {
  const OIndex* ix = static_cast<const OIndex*>(h);
  std::memcpy(ukeys, ix->ukeys.data(), ix->ukeys.size() * sizeof(uint64_t));
  std::memcpy(ustart, ix->ustart.data(), ix->ustart.size() * sizeof(int64_t));
}

// returns the table length (n_cells + 1), or -1 when the index is not dense
int64_t orc_dense_start(const void* h, int64_t* out) {
  const OIndex* ix = static_cast<const OIndex*>(h);
  if (ix->flavor != DENSE) return -1;
  if (out) std::memcpy(out, ix->dstart.data(), ix->dstart.size() * sizeof(int64_t));
  return (int64_t)ix->dstart.size();
}

// mixed flavor only: per z-slice non-empty voxel count and dense flag
int64_t orc_slices(const void* h, int64_t* nonempty, uint8_t* dense) {
  const OIndex* ix = static_cast<const OIndex*>(h);
  if (ix->flavor != MIXED) return -1;
  const int64_t nz = ix->ncell[2];
  if (nonempty) std::memcpy(nonempty, ix->slice_nonempty.data(), nz * sizeof(int64_t));
  if (dense) std::memcpy(dense, ix->slice_dense.data(), nz);
  return nz;
}

// Queries: pidx = point indices into the cloud, or qxyz = FP64 absolute
// coordinates [nq,3], or both NULL = every point of the cloud in index order.
void* orc_kernel_search(const void* h, const int32_t* pidx, const double* qxyz, int64_t nq,
                        int kernel, float r, int nthreads, int64_t* offsets, int64_t* visited) {
  const OIndex* ix = static_cast<const OIndex*>(h);
  std::vector<std::vector<int32_t>> part((size_t)std::max(1, nthreads));
  std::vector<int64_t> cnt(nq, 0);
  int64_t chunk = (nq + std::max(1, nthreads) - 1) / std::max(1, nthreads);
  parallel_for(nq, nthreads, [&](int64_t a, int64_t b) {
    size_t t = (size_t)(a / std::max<int64_t>(1, chunk));
    std::vector<int32_t>& out = part[t];
    for (int64_t q = a; q < b; ++q) {
      float c[3];
      size_t before = out.size();
      if (query_coords(*ix, pidx, qxyz, q, c))
        radius_one(*ix, c, r, out, visited ? visited + q : nullptr, kernel);
      cnt[q] = (int64_t)(out.size() - before);
    }
  });
  offsets[0] = 0;
  for (int64_t q = 0; q < nq; ++q) offsets[q + 1] = offsets[q] + cnt[q];
  RadiusResult* res = new RadiusResult();
  res->nbr.reserve(offsets[nq]);
  for (auto& v : part) res->nbr.insert(res->nbr.end(), v.begin(), v.end());
  return res;
}

void* orc_radius(const void* h, const int32_t* pidx, const double* qxyz, int64_t nq, float r,
                 int nthreads, int64_t* offsets, int64_t* visited) {
  return orc_kernel_search(h, pidx, qxyz, nq, kSphere, r, nthreads, offsets, visited);
}

void orc_radius_copy(void* res, int32_t* nbr) {
  RadiusResult* r = static_cast<RadiusResult*>(res);
  std::memcpy(nbr, r->nbr.data(), r->nbr.size() * sizeof(int32_t));
}

void orc_radius_free(void* res) { delete static_cast<RadiusResult*>(res); }

// idx / d2: [nq, k], sorted by (d2, index); padded with (-1, +inf)
int orc_knn(const void* h, const int32_t* pidx, const double* qxyz, int64_t nq, int k,
            float r_max, int nthreads, int32_t* idx, float* d2, int64_t* visited,
            int monotonic) {
  const OIndex* ix = static_cast<const OIndex*>(h);
  if (k < 1 || std::isnan(r_max) || r_max < 0) return 1;
  parallel_for(nq, nthreads, [&](int64_t a, int64_t b) {
    for (int64_t q = a; q < b; ++q) {
      float c[3];
      if (query_coords(*ix, pidx, qxyz, q, c)) {
        knn_one(*ix, c, k, r_max, idx + q * k, d2 + q * k, visited ? visited + q : nullptr,
                monotonic != 0);
      } else {
        for (int i = 0; i < k; ++i) {
          idx[q * k + i] = -1;
          d2[q * k + i] = INFINITY;
        }
      }
    }
  });
  return 0;
}

// ---- Gaussian-weighted aggregation (project addition), FP64 ------------
// out[q,c] = sum_t w_qt f[j_t, c],  w = exp(-|x_j - x_q|^2 / (2 sigma^2)),
// x_q = x[qidx[q]], j_t = nbr[q,t] (entries < 0 are padding).
void orc_agg_fwd(const double* x, const int32_t* qidx, const int32_t* nbr, int64_t N, int64_t Q,
                 int32_t K, const double* f, int32_t C, double sigma, double* out) {
  (void)N;
  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
  for (int64_t q = 0; q < Q; ++q) {
    const double* xq = x + (int64_t)qidx[q] * 3;
    for (int32_t c = 0; c < C; ++c) out[q * C + c] = 0.0;
    for (int32_t t = 0; t < K; ++t) {
      int32_t j = nbr[q * K + t];
      if (j < 0) continue;
      const double* xj = x + (int64_t)j * 3;
      double D = 0.0;
      for (int a = 0; a < 3; ++a) D += (xj[a] - xq[a]) * (xj[a] - xq[a]);
      double w = std::exp(-D * inv2s2);
      for (int32_t c = 0; c < C; ++c) out[q * C + c] += w * f[(int64_t)j * C + c];
    }
  }
}

// Analytic gradient of sum_{q,c} gout[q,c] * out[q,c] with the neighbour
// lists held fixed.  With a = sum_c gout[q,c] f[j,c] and dw/dx_j =
// -w (x_j - x_q) / sigma^2:  grad_f[j] += w gout[q];
// grad_x[j] += a w (x_q - x_j) / sigma^2;  grad_x[qidx[q]] += a w (x_j - x_q) / sigma^2.
void orc_agg_bwd(const double* x, const int32_t* qidx, const int32_t* nbr, int64_t N, int64_t Q,
                 int32_t K, const double* f, int32_t C, double sigma, const double* gout,
                 double* grad_x, double* grad_f) {
  const double s2 = sigma * sigma, inv2s2 = 1.0 / (2.0 * s2);
  for (int64_t p = 0; p < N * 3; ++p) grad_x[p] = 0.0;
  for (int64_t p = 0; p < N * (int64_t)C; ++p) grad_f[p] = 0.0;
  for (int64_t q = 0; q < Q; ++q) {
    const int64_t iq = qidx[q];
    const double* xq = x + iq * 3;
    for (int32_t t = 0; t < K; ++t) {
      int32_t j = nbr[q * K + t];
      if (j < 0) continue;
      const double* xj = x + (int64_t)j * 3;
      double D = 0.0;
      for (int a = 0; a < 3; ++a) D += (xj[a] - xq[a]) * (xj[a] - xq[a]);
      double w = std::exp(-D * inv2s2);
      double acoef = 0.0;
      for (int32_t c = 0; c < C; ++c) {
        acoef += gout[q * C + c] * f[(int64_t)j * C + c];
        grad_f[(int64_t)j * C + c] += w * gout[q * C + c];
      }
      double sc = acoef * w / s2;
      for (int a = 0; a < 3; ++a) {
        double d = xj[a] - xq[a];
        grad_x[(int64_t)j * 3 + a] -= sc * d;
        grad_x[iq * 3 + a] += sc * d;
      }
    }
  }
}

}  // extern "C"
