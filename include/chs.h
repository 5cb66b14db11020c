/* chs.h -- C ABI of the MI355X grid point index (Cheesemap, Laso & Yermo,
 * arXiv 2502.11602).
 *
 * The index is the paper's uniform voxel grid (Section 3.2) stored in one of
 * its three flavors (Section 3.3: dense, sparse, mixed), built on the GPU by
 * keying every point with its voxel's global index (Eq. 5-7), counting the
 * points per voxel, prefix-summing the counts and scattering the points into
 * voxel order (the reordering of Section 3.5).  It answers batches of
 * fixed-radius sphere queries (the kernel-based search of Section 3.4.1,
 * Alg. 1) and k-nearest-neighbour queries (Section 3.4.2, Alg. 2).
 *
 * Conventions shared by every call:
 *  - Array pointers are DEVICE pointers unless marked (host).  Every call is
 *    enqueued on `stream`; only the calls documented as synchronising wait
 *    for it.
 *  - Inputs are borrowed for the duration of the call.  Outputs of fixed size
 *    are allocated by the caller.  Memory the library keeps (the index) or
 *    needs temporarily comes from the `chs_allocator` given to chs_build; a
 *    NULL allocator means stream-ordered hipMallocAsync / hipFreeAsync.
 *  - Temporaries of a call are allocated for, and freed on, the call's
 *    stream.  Searches on one index may run concurrently on different
 *    streams: each call has its own work counter and query plan.
 *  - Calls never abort.  They return a chs_status; on failure the message of
 *    chs_last_error() says why, the caller's outputs are left untouched
 *    unless stated otherwise, and nothing leaks.  Arguments are validated on
 *    the host before anything is enqueued.
 *  - Geometry: coordinates are FP64 [n,3] row-major (x, y, z), absolute.  The
 *    index recentres them on the cloud's minimum corner p- (Eq. 1) in FP64
 *    and stores FP32.  The squared distance of a point p to a centre c is the
 *    unfused FP32 value D = (dx*dx + dy*dy) + dz*dz with dx = fl32(c_x - p_x),
 *    and a point is inside a sphere of radius r when D <= fl32(r*r) (closed
 *    sphere).  Results are bit-exact against that definition.
 */
#ifndef CHS_H
#define CHS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum chs_status {
  CHS_OK = 0,
  CHS_E_INVALID = 1,     /* bad argument (NULL, size, non-finite, range)      */
  CHS_E_NOMEM = 2,       /* the allocator returned NULL                        */
  CHS_E_CAPACITY = 3,    /* a table would exceed its limit (dense voxel count) */
  CHS_E_DEVICE = 4,      /* a HIP runtime error                                */
  CHS_E_UNSUPPORTED = 5  /* valid but not implemented for this configuration   */
} chs_status;

/* Voxel storage, Section 3.3: DENSE keeps every voxel of the grid (3.3.1),
 * SPARSE keeps only non-empty voxels in a hash map keyed by the global index
 * (3.3.2), MIXED splits the grid into z-slices, each dense once at least
 * mixed_dense_pct percent of its voxels hold points and sparse otherwise
 * (3.3.3). */
typedef enum chs_flavor { CHS_DENSE = 0, CHS_SPARSE = 1, CHS_MIXED = 2 } chs_flavor;

typedef struct chs_allocator {
  void* (*alloc)(size_t bytes, void* ctx); /* device memory, >= 256-byte aligned */
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} chs_allocator;

typedef struct chs_build_params {
  int32_t flavor;          /* chs_flavor                                        */
  int32_t dims;            /* 3: voxels on x,y,z; 2: columns on x,y (n_z = 1)   */
  double cell[3];          /* voxel edge per axis in metres, > 0 (Section 3.2,
                              footnote: edges may differ per axis); cell[2] is
                              ignored when dims == 2                            */
  int32_t mixed_dense_pct; /* MIXED: slice turns dense at this percentage of
                              non-empty voxels (the paper's default is 80)      */
  int32_t reserved;        /* must be 0                                         */
  int64_t max_dense_cells; /* DENSE: refuse grids with more voxels (0 = 2^31-2) */
} chs_build_params;

typedef struct chs_index_s* chs_index;

/* A batch of query centres.  Exactly one of:
 *   xyz       [nq,3] FP64 absolute coordinates (recentred by the library),
 *   point_idx [nq]   int32 indices into the indexed cloud (the centre is that
 *                    point's stored FP32 position; the paper's benchmark
 *                    queries are cloud points, Section 4.4),
 *   neither          every indexed point, in index order (nq must equal n).
 * nq == 0 is an empty batch whatever the pointers.  A point index outside
 * [0, n) or a non-finite coordinate makes an empty query (no neighbours,
 * k-NN row of (-1, +inf)).  Row q of every result belongs to the caller's
 * q-th query. */
typedef struct chs_queries {
  const double* xyz;
  const int32_t* point_idx;
  int64_t nq;
} chs_queries;

/* Build the index over n points xyz [n,3] (FP64, device).  Computes the
 * bounding box p-, p+ (Eq. 1-2), the grid size n_a = floor((p+_a - p-_a)/s_a)
 * + 1 (Eq. 3), each point's voxel (Eq. 5, 0-based, clamped to n_a - 1) and
 * global index g = (i*n_y + j)*n_z + k (Eq. 6-7), the per-voxel counts, their
 * exclusive prefix sum and the stable scatter of the points into voxel order
 * (ascending g, then ascending original index), and the flavor's voxel map;
 * then the processing order of "every point" queries (a Hilbert order over
 * the voxel columns), so that such searches plan nothing.  Synchronises
 * `stream` to size the grid from the bounding box and the voxel tables from
 * the number of non-empty voxels (and, for MIXED, the per-slice counts).
 * n in [1, 2^31 - 1].  Non-finite coordinates give CHS_E_INVALID; a dense
 * grid above max_dense_cells gives CHS_E_CAPACITY; an allocator returning
 * NULL gives CHS_E_NOMEM (everything allocated so far is released and *out
 * is untouched).  On success *out (host)
 * owns its device memory until chs_free. */
chs_status chs_build(const double* xyz, int64_t n, const chs_build_params* params,
                     const chs_allocator* alloc, hipStream_t stream, chs_index* out);

typedef struct chs_index_info_t {
  double origin[3];     /* p-, FP64                                      */
  float max32[3];       /* p+ - p- after recentring, FP32                */
  double cell[3];
  int64_t ncell[3];     /* n_x, n_y, n_z                                  */
  int64_t n_points;
  int64_t n_nonempty;   /* voxels holding at least one point             */
  int64_t n_dense_slices; /* MIXED: slices stored densely                 */
  int64_t device_bytes; /* memory held by the index                      */
  int32_t flavor, dims;
  int32_t ntiles;       /* 1, or the number of tiles of a batched index  */
  int32_t reserved;
} chs_index_info_t;

/* Host-side description of a built index: the bounding-box corner p- and
 * the recentred extent (Section 3.1, Eq. 1-2), the voxel edges and the grid
 * size n_x, n_y, n_z (Section 3.2, Eq. 3), the number of non-empty voxels
 * and, for MIXED, of slices stored densely (Section 3.3.3).  For a batched
 * index: tile 0's geometry and the totals.  No device work. */
chs_status chs_index_info(chs_index index, chs_index_info_t* out /* host */);

/* Batched build: ntiles independent clouds stored back to back in xyz
 * [n,3]; tile t holds input points [tile_off[t], tile_off[t+1]) (tile_off
 * is a host array of ntiles+1 entries, from 0 to n, strictly increasing).
 * Each tile gets its own bounding box, grid and voxel edges (params[t],
 * host array of ntiles entries, one flavor for all; MIXED is single-tile
 * only: its slice tables are per z layer of one grid, and a batch's tiles
 * each have their own z layers).  The tiles' voxel key spaces are
 * concatenated, so keying, sorting and the voxel maps run once for the
 * whole batch.  The chs_radius_* / chs_kernel_* / chs_knn searches on a
 * batched index take "every point" queries (each point queries its own
 * tile); per-tile query sets go through the *_tiles calls.  Rows follow the
 * caller's order and neighbour indices are tile-local (input index minus
 * tile_off[t]). */
chs_status chs_build_batch(const double* xyz, int64_t n, const int64_t* tile_off /* host */,
                           int32_t ntiles, const chs_build_params* params /* host */,
                           const chs_allocator* alloc, hipStream_t stream, chs_index* out);

/* A batched build that never waits for the stream and reads nothing back
 * from the device, so that it can be captured in a graph (hipStreamBeginCapture)
 * and replayed: as chs_build_batch, with each tile's bounding box given by
 * the caller instead of computed, frames (host, [ntiles][6] FP64: p-_x,
 * p-_y, p-_z, p+_x, p+_y, p+_z; the corners of Eq. 1-2), and the voxel
 * tables sized for the worst case (every point its own voxel).  With frames
 * equal to the tiles' exact minimum and maximum coordinates every array and
 * search result equals chs_build_batch's; a frame that does not hold its
 * tile's points gives a valid index whose FP32 frame is fl32(p - frame
 * minimum), its outlying points in the border voxels.  DENSE or SPARSE only
 * (MIXED decides its slices from the points: CHS_E_UNSUPPORTED).  The
 * non-empty voxel count stays on the device until chs_index_info or
 * chs_index_arrays reads it (they then wait for the stream).  Temporaries
 * and the index come from `alloc` (under capture: from the capturing
 * allocator's pool). */
chs_status chs_build_batch_framed(const double* xyz, int64_t n, const int64_t* tile_off /* host */,
                                  int32_t ntiles, const chs_build_params* params /* host */,
                                  const double* frames /* host */, const chs_allocator* alloc,
                                  hipStream_t stream, chs_index* out);

/* Geometry of one tile of a batched index (n_nonempty is -1). */
chs_status chs_tile_info(chs_index index, int32_t tile, chs_index_info_t* out /* host */);

/* Options of a built index (the searches' launch and schedule; results never
 * depend on them).
 * CHS_OPT_PERSISTENT (default: on for batched indexes, off otherwise):
 * searches launch one wave per hardware slot and the waves pull 64-query
 * work items (largest tiles first) from a device counter until none is left,
 * instead of one wave per work item.  Results are identical either way.
 * CHS_OPT_KNN_SCHEDULE (default 0): how chs_knn grows the visited voxels.
 * 0 = rings: one voxel per step, a query is done once its k-th distance is
 * below the distance to the visited box's faces.  1 = density growth, the
 * schedule of Alg. 2 (Section 3.4.2): the radius starts at the distance to
 * the nearest wall of the query's voxel (Eq. 11) and grows from the density
 * of the candidates within it (Eq. 12), a query being done once k of them
 * lie within the radius.  2 = monotonic growth: as 1 with the radius grown
 * by the smallest voxel edge at every step, the baseline that Section 3.5
 * compares density growth with.  3 = one query at a time: a wave grows each
 * query's own visited box ring by ring and tests 64 candidates per step
 * (for query sets that sample the cloud sparsely, whose 64-query tiles
 * would stream the empty space between their queries).  Results are
 * identical; only the cost differs. */
/* CHS_OPT_FILL_STAGE (default 0): the radius fill stages each query's
 * matches in on-chip memory (LDS) before writing them out, 16, 24, 32 or 64
 * entries per query; 0 picks the size from the mean row length total / nq.
 * Results are identical. */
/* CHS_OPT_RADIUS_SCHEDULE (default 0): how the kernel-based searches share
 * work.  1 = tiles: a wave takes 64 nearby queries and tests every point of
 * their common voxel box against all of them; 2 = groups: a wave takes 8
 * nearby queries at a time and tests the points of their own, smaller
 * common box.  0 picks groups for spheres and cubes with r >= 1.5 voxel
 * edges, tiles otherwise.  Results are identical (the fill stage applies to
 * tiles). */
typedef enum chs_option {
  CHS_OPT_PERSISTENT = 1,
  CHS_OPT_KNN_SCHEDULE = 4,
  CHS_OPT_FILL_STAGE = 5,
  CHS_OPT_RADIUS_SCHEDULE = 6
} chs_option;
chs_status chs_index_set_option(chs_index index, int32_t option, int64_t value);

/* Device arrays of a built index, borrowed (valid until chs_free, never to
 * be written): the reordered cloud of Section 3.5 ("Reordering", points
 * stored voxel by voxel) and the voxel maps of Section 3.3.  perm[pos] = original index of the pos-th stored point;
 * inv_perm = its inverse; sorted_xyz = SoA [3][n] FP32 recentred coordinates
 * in stored order; points = [n] x,y,z,FP32 + original index (int32 bits) in
 * stored order; cell_keys [M] = ascending non-empty global voxel indices
 * (uint64); cell_start [M+1] = first stored position of each, then n;
 * dense_start [n_x*n_y*n_z + 1] (DENSE only, else NULL) = first stored
 * position of every voxel; slice_dense [n_z] (MIXED only, else NULL) = 1
 * when slice k is stored densely. */
typedef struct chs_index_arrays_t {
  const int32_t* perm;
  const int32_t* inv_perm;
  const float* sorted_xyz;
  const float* points;
  const uint64_t* cell_keys;
  const int32_t* cell_start;
  const int32_t* dense_start;
  const uint8_t* slice_dense;
} chs_index_arrays_t;

chs_status chs_index_arrays(chs_index index, chs_index_arrays_t* out /* host */);

/* The index's FP32 coordinates in input order: out [n,3] (FP32, device,
 * caller-allocated) receives fl32(p - p-) for every point p, the recentring
 * of Section 3.1 (Eq. 1) that every distance of the searches uses; each tile
 * of a batched index in its own frame.  Enqueued on `stream`. */
chs_status chs_index_coords(chs_index index, float* out, hipStream_t stream);

/* Fixed-radius search, count pass (Alg. 1 with a spherical kernel B(c, r),
 * Section 3.4.1): offsets [nq+1] (int64, device) receives the exclusive
 * prefix sum of the per-query neighbour counts |{p : D(c, p) <= fl32(r*r)}|,
 * and *total (host) its last entry.  Synchronises `stream` to read total;
 * with total NULL nothing is read or waited for (the total is offsets[nq] on
 * the device), so the call can be captured in a graph.  r must be finite
 * and >= 0. */
chs_status chs_radius_count(chs_index index, const chs_queries* queries, float r,
                            int64_t* offsets, int64_t* total, hipStream_t stream);

/* Fill pass of Alg. 1 (Section 3.4.1; the points inside the kernel are
 * appended to the query's list): writes the original indices of each
 * query's neighbours into nbr[offsets[q] - offsets[0] .. offsets[q+1] -
 * offsets[0]) (int32, device, `total` entries, as given by
 * chs_radius_count for the same queries and r, where offsets[0] = 0).  A
 * consecutive range [a, b) of a counted set fills on its own with the
 * queries and offsets advanced by a (offsets + a, base offsets[a]) and total
 * = offsets[b] - offsets[a]: rows too many for one buffer are filled range
 * by range (chs_fill_chunks picks the ranges).  The order inside a row is
 * deterministic but unspecified (the neighbour relation is a set).  Every
 * write stays inside nbr[0, total): a row is clipped at total, and a row
 * that starts before offsets[0] or has offsets[q] > offsets[q+1] is not
 * written, so offsets that belong to other queries or another r give wrong
 * rows but never write outside nbr. */
chs_status chs_radius_fill(chs_index index, const chs_queries* queries, float r,
                           const int64_t* offsets, int32_t* nbr, int64_t total,
                           hipStream_t stream);

/* The order in which the searches process a query batch (Hilbert order of
 * the centres' voxel columns, then z; per tile on a batched index): order
 * (device, [nq] int32) receives the caller's query indices in that order.
 * Queries reordered by it are spatially coherent in any consecutive range,
 * which is what a range-by-range fill (chs_fill_chunks) needs to keep its
 * ranges' query groups tight: ranges of a random query order each spread
 * over the whole cloud.  Does not synchronise. */
chs_status chs_query_order(chs_index index, const chs_queries* queries, int32_t* order,
                           hipStream_t stream);

/* Splits a counted set of nq queries into consecutive ranges that each
 * fill within max_entries neighbour entries (a memory budget for the fill's
 * output), as few as possible: bounds (host) receives q_0 = 0 < q_1 < ... <
 * q_m = nq and entry_bounds (host) offsets[q_i], so range i is the queries
 * [q_i, q_{i+1}) with entry_bounds[i+1] - entry_bounds[i] entries.  offsets:
 * device, [nq+1], from chs_radius_count / chs_kernel_count.  *nchunks
 * (host) = m.  With cap = 0 only *nchunks is computed (bounds and
 * entry_bounds may be NULL); otherwise they hold cap entries and cap < m + 1
 * is CHS_E_CAPACITY (*nchunks set).  A single query with more than
 * max_entries neighbours is CHS_E_CAPACITY; decreasing offsets are
 * CHS_E_INVALID.  Copies offsets to the host and synchronises `stream`. */
chs_status chs_fill_chunks(const int64_t* offsets, int64_t nq, int64_t max_entries,
                           int64_t* bounds /* host */, int64_t* entry_bounds /* host */,
                           int64_t cap, int64_t* nchunks /* host */, hipStream_t stream);

/* The whole fixed-radius search of Alg. 1 (Section 3.4.1): count +
 * allocation of the neighbour array through `alloc` (NULL = the index's
 * allocator) + fill.  *nbr (host) receives the device pointer, which the
 * caller releases with the same allocator (or hipFree for NULL); it is NULL
 * when total is 0.  Synchronises `stream` once.  If the allocation fails
 * (CHS_E_NOMEM) offsets already hold the count pass's result and *nbr,
 * *total are untouched. */
chs_status chs_radius_search(chs_index index, const chs_queries* queries, float r,
                             const chs_allocator* alloc, int64_t* offsets, int32_t** nbr,
                             int64_t* total, hipStream_t stream);

/* Other kernels of Alg. 1 (Section 3.4.1: the search works for any kernel
 * that gives a bounding box and an inside test; the cube and the cylinder of
 * Section 2).  With differences dx = fl32(qx - px) etc. and R = fl32(r*r):
 *   CHS_KERNEL_SPHERE    (dx*dx + dy*dy) + dz*dz <= R  (the chs_radius_* calls)
 *   CHS_KERNEL_CUBE      |dx| <= r and |dy| <= r and |dz| <= r  (half side r)
 *   CHS_KERNEL_CYLINDER  dx*dx + dy*dy <= R, any z (a vertical cylinder)
 * all in FP32 with unfused operations.  Arguments, outputs, ownership and
 * errors as chs_radius_count / chs_radius_fill / chs_radius_search; an
 * unknown kernel is CHS_E_INVALID. */
typedef enum chs_kernel {
  CHS_KERNEL_SPHERE = 0,
  CHS_KERNEL_CUBE = 1,
  CHS_KERNEL_CYLINDER = 2
} chs_kernel;
chs_status chs_kernel_count(chs_index index, const chs_queries* queries, int32_t kernel, float r,
                            int64_t* offsets, int64_t* total, hipStream_t stream);
chs_status chs_kernel_fill(chs_index index, const chs_queries* queries, int32_t kernel, float r,
                           const int64_t* offsets, int32_t* nbr, int64_t total,
                           hipStream_t stream);
chs_status chs_kernel_search(chs_index index, const chs_queries* queries, int32_t kernel, float r,
                             const chs_allocator* alloc, int64_t* offsets, int32_t** nbr,
                             int64_t* total, hipStream_t stream);

/* Per-tile query sets on a batched index (the searches of Alg. 1 and Alg. 2
 * run on each tile's own grid): the queries [q_off[t], q_off[t+1]) belong to
 * tile t (q_off: host, ntiles+1 entries, from 0 to nq, non-decreasing).
 * Exactly one of xyz (FP64 absolute; recentred on the tile's p-, Eq. 1) and
 * point_idx (tile-local: 0 .. n_t - 1; others make empty queries) is given.
 * Rows follow the caller's order and neighbour indices are tile-local.
 * Arguments, outputs and errors otherwise as chs_kernel_count /
 * chs_kernel_fill / chs_knn.  Each call copies its tables from q_off and
 * waits for the stream once. */
chs_status chs_kernel_count_tiles(chs_index index, const chs_queries* queries,
                                  const int64_t* q_off /* host */, int32_t kernel, float r,
                                  int64_t* offsets, int64_t* total, hipStream_t stream);
chs_status chs_kernel_fill_tiles(chs_index index, const chs_queries* queries,
                                 const int64_t* q_off /* host */, int32_t kernel, float r,
                                 const int64_t* offsets, int32_t* nbr, int64_t total,
                                 hipStream_t stream);
chs_status chs_knn_tiles(chs_index index, const chs_queries* queries,
                         const int64_t* q_off /* host */, int32_t k, float r_max, int32_t* idx,
                         float* d2, hipStream_t stream);

/* k-nearest-neighbour search (Section 3.4.2): for every query, the min(k, n)
 * points first in the order (D, original index), written to idx [nq,k]
 * (int32) and their squared distances D to d2 [nq,k] (FP32), ascending;
 * with a finite r_max only entries with D <= fl32(r_max*r_max) are kept.
 * Missing entries are (-1, +inf).  1 <= k <= 64; r_max >= 0 or +inf.
 * Does not synchronise. */
chs_status chs_knn(chs_index index, const chs_queries* queries, int32_t k, float r_max,
                   int32_t* idx, float* d2, hipStream_t stream);

/* chs_knn that also reports how many voxels each query's search visits,
 * the cost measure by which Section 3.5 compares density growth with
 * monotonic growth (CHS_OPT_KNN_SCHEDULE picks the schedule).
 * visited: device, [nq][2] int64, written for every valid query (invalid
 * queries' entries are left as they are):
 *   [q][0] the query's own taboo box, Alg. 2 run for it alone: under
 *          density or monotonic growth the voxels of the padded bounding
 *          box of B(c, r), clamped to the grid, at the first radius of the
 *          schedule holding k of its neighbours (or whose box is the whole
 *          grid; with a finite r_max, at the radius where the search
 *          stopped); empty voxels count (on a dense map every voxel exists,
 *          Section 3.5).  Under rings, equal to [q][1];
 *   [q][1] the visited box of the wave that searched the query together
 *          with up to 63 nearby ones, when the query's list became final:
 *          the voxels the GPU actually scanned for it.
 * A single-tile index without CHS_OPT_PERSISTENT only (CHS_E_UNSUPPORTED
 * otherwise).  Arguments, results, errors and synchronisation otherwise as
 * chs_knn. */
chs_status chs_knn_visited(chs_index index, const chs_queries* queries, int32_t k, float r_max,
                           int32_t* idx, float* d2, int64_t* visited, hipStream_t stream);

/* chs_knn for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, results and errors as chs_knn, but no allocator is called.
 * Every temporary (the query plan with its sort buffers, the list of waves
 * left to the search's second launch, the persistent work counter) is carved
 * from a fixed 32 MiB device array that the library holds on each GPU it
 * runs on until the process ends.  Index or coordinate queries: nq <= 2^19;
 * "every point" queries use the order the build planned, n <= 2^28 on a
 * plain index, any n on a batched or persistent one (CHS_E_CAPACITY beyond,
 * checked before any device work).  Call
 * with the index's device current.  All calls on one GPU share that GPU's
 * array: two calls in flight at once (on different streams or threads) race
 * and give wrong results.  Does not synchronise. */
chs_status chs_knn_noalloc(chs_index index, const chs_queries* queries, int32_t k, float r_max,
                           int32_t* idx, float* d2, hipStream_t stream);

/* ---- Gaussian-weighted neighbourhood aggregation (a project addition) ----
 * out[q,c] = sum_t w_qt f[j_t, c] with w_qt = exp(-D(x_j, x_q) / (2 sigma^2)),
 * x_q = x[qidx[q]], j_t = nbr[q,t]; negative or out-of-range entries of nbr
 * are padding and contribute nothing.  D is the unfused squared distance in
 * the compute type.  Typical neighbour lists come from chs_knn (the k nearest
 * within r_max) over the same points.
 *   x     [N,3]  coordinates (recentred), x_dtype
 *   f     [N,C]  features, f_dtype;   out, grad_out, grad_f [Q,C] f_dtype
 *   qidx  [Q]    centre point of each query; nbr [Q,K] int32
 * Sizes: 1 <= N < 2^31 - 1, C >= 1 and Q * (K + 1) <= 2^31 - 1 (the backward
 * regroups the pair slots with 32-bit positions), else CHS_E_INVALID.
 * dtype pairs: (CHS_F32, CHS_F32), (CHS_F32, CHS_BF16) computing in FP32, and
 * (CHS_F64, CHS_F64) computing in FP64; others give CHS_E_UNSUPPORTED.  Sums
 * run in a fixed order, so results are bitwise reproducible. */
typedef enum chs_dtype { CHS_F32 = 0, CHS_F64 = 1, CHS_BF16 = 2 } chs_dtype;

chs_status chs_gauss_agg_fwd(const void* x, const int32_t* qidx, const int32_t* nbr, int64_t N,
                             int64_t Q, int32_t K, const void* f, int32_t C, double sigma,
                             int32_t x_dtype, int32_t f_dtype, void* out, hipStream_t stream);

/* Gradient of sum_{q,c} grad_out[q,c] out[q,c] with the neighbour lists held
 * fixed: grad_x [N,3] (x_dtype; both the neighbour and the centre role of
 * every point) and grad_f [N,C] (f_dtype), both fully overwritten.  Pairs
 * are regrouped by neighbour with a stable sort and summed segment by
 * segment (no floating-point atomics).  Temporaries (about 24 bytes per pair)
 * come from `alloc` (NULL: stream-ordered hipMallocAsync). */
chs_status chs_gauss_agg_bwd(const void* x, const int32_t* qidx, const int32_t* nbr, int64_t N,
                             int64_t Q, int32_t K, const void* f, int32_t C, double sigma,
                             int32_t x_dtype, int32_t f_dtype, const void* grad_out, void* grad_x,
                             void* grad_f, const chs_allocator* alloc, hipStream_t stream);

/* Release the index and its device memory (stream-ordered on the stream it
 * was built with).  NULL is ignored. */
void chs_free(chs_index index);

/* Message of the last failure on the calling thread ("" if none).  Valid
 * until the next call on the same thread. */
const char* chs_last_error(void);

/* Library version string, e.g. "chs 0.1.0 gfx950". */
const char* chs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CHS_H */
