/*
 * spmspv.h -- C ABI of the MI355X (gfx950) SpMSpV library.
 *
 * Computes y <- A x over a semiring where A is an m-by-n sparse matrix in
 * compressed sparse column (CSC) form and x, y are sparse vectors in list
 * form (index array + value array), following Azad and Bulu\c{c}, "A
 * work-efficient parallel sparse matrix-sparse vector multiplication
 * algorithm": problem statement in Background / Notation; CSC and list
 * vectors in Background / "Sparse matrix and vector data structures"; the
 * method is Algorithm 1 (SpMSpV-bucket) with its preprocessing step
 * Algorithm 2 (Estimate-Buckets).
 *
 * Conventions for every call:
 *   - Pointers are DEVICE pointers unless their name starts with h_.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     All device work is ordered on that stream.  Calls return after
 *     enqueueing unless documented as synchronous.
 *   - Indices are int32; colptr is int32 (nnz < 2^31); products and
 *     offsets that can exceed 2^31 are int64.
 *   - Status is the int return value (SPMSPV_OK = 0, negative = error).
 *     No call throws.  A call that fails validation writes nothing to its
 *     outputs.  spmspv_last_error() returns a thread-local detail string.
 *   - The library never allocates device memory after spmspv_create.  The
 *     caller owns A's arrays, x, y, BFS/PageRank outputs and the workspace;
 *     they must outlive the handle.
 *   - A handle is not reentrant: calls on one handle must not overlap in
 *     time on different streams (they share the workspace).  Use one handle
 *     per concurrent stream.
 */
#ifndef SPMSPV_H
#define SPMSPV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spmspv_matrix* spmspv_handle;

/* Semirings (Algorithm 1's Mult / Add pair).
 *   PLUS_TIMES_F32     : Mult = a*x (fp32, rounded), Add = +.
 *                        A values float, x float, y float.  Each product
 *                        is rounded to fp32; a row's products are summed
 *                        in fp64 (in any order) and the sum is rounded to
 *                        fp32 once, so |y - exact| <= 2^-24 |exact| plus
 *                        k * 2^-53 * sum|terms| for a row of k terms.
 *   MIN_SELECT2ND_I32  : Mult = select2nd(a, x) = x, Add = min.
 *                        A values ignored, x int32, y int32.
 *   OR_AND_BOOL        : Mult = (a != 0) AND (x != 0), Add = OR.
 *                        A values (or pattern), x uint8, y uint8 (0/1).
 * Output pattern is structural: y holds every row reached by a selected
 * column, once (the unique indices of all buckets, Algorithm 1 step 2),
 * even when its value equals the semiring zero.                          */
enum spmspv_semiring {
    SPMSPV_PLUS_TIMES_F32 = 0,
    SPMSPV_MIN_SELECT2ND_I32 = 1,
    SPMSPV_OR_AND_BOOL = 2
};

enum spmspv_status {
    SPMSPV_OK = 0,
    SPMSPV_EINVAL = -1,        /* bad argument or invalid input data          */
    SPMSPV_ENOMEM = -2,        /* workspace smaller than spmspv_workspace_size */
    SPMSPV_ECAPACITY = -3,     /* y_capacity < nnz(y); required size reported */
    SPMSPV_EHIP = -4,          /* a HIP runtime call failed                    */
    SPMSPV_EUNSUPPORTED = -5,  /* valid request this build cannot serve        */
    SPMSPV_EDEVICE = -6        /* the device reported an error bit (see text)  */
};

/* Flags (bitwise OR). */
enum spmspv_flags {
    SPMSPV_SORTED_OUTPUT = 1,  /* y indices strictly ascending (sorted variant,
                                  Algorithm 1 with per-bucket ordering)        */
    SPMSPV_VALIDATE = 2,       /* check inputs on the host before launching:
                                  synchronous, O(nnz) at create, O(f) per run */
    SPMSPV_X_VAL_IS_INDEX = 4, /* MIN_SELECT2ND: x value of entry p is
                                  x_idx[p]; x_val may be NULL                  */
    SPMSPV_X_ALL_TRUE = 8,     /* OR_AND: every x value is true; x_val may be
                                  NULL                                         */
    SPMSPV_USE_GRAPH = 16,     /* bfs_run: replay the level loop as a captured
                                  hipGraph                                     */
    SPMSPV_PROFILE = 32,       /* record each kernel's own start and end
                                  timestamps in HIP events (see
                                  spmspv_profile_read)                        */
    SPMSPV_WITH_TRANSPOSE = 64,/* create: also build the CSR form of A so the
                                  pull direction is available                 */
    SPMSPV_SYMMETRIC = 128,    /* create: caller states A == A^T (pattern and
                                  values); the pull direction reads A's
                                  columns as rows, no transpose is built      */
    SPMSPV_DIRECTION_OPT = 256,/* bfs_run: choose push or pull per level
                                  (Beamer's frontier-edge heuristic); needs a
                                  handle created with one of the two flags
                                  above                                       */
    SPMSPV_PERSISTENT = 8192,  /* bfs_run (push, no direction switching) on a
                                  graph whose longest column has at most 64
                                  entries: levels with at most 65536 frontier
                                  vertices run in one cooperative persistent
                                  kernel (one grid barrier per level, direct
                                  atomic discovery, same levels and minimum
                                  parents); larger frontiers take the
                                  bucketing levels.  Ignored otherwise        */
    SPMSPV_PULL_ROWWISE = 4096,/* spmspv_run with the pull direction, min-
                                  select2nd or or-and: one thread per row
                                  not masked, stopping at the first x hit (the
                                  bottom-up BFS step) instead of the
                                  merge-path row kernel                       */
    SPMSPV_AUTO_SCHEDULE = 2048,/* spmspv_run: use the schedule spmspv_autotune
                                  found for the density band nearest f / n  */
    SPMSPV_MSBFS = 1024,       /* spmspv_batch_workspace_size / _attach: also
                                  hold per-source frontiers and visited
                                  bitmaps for msbfs_run                       */
    SPMSPV_USE_SELECTOR = 512, /* spmspv_run / bfs_run / pagerank_run: a small
                                  MLP loaded with spmspv_selector_load picks
                                  the bucket count (or the pull direction)
                                  per call from features the scan computes on
                                  the device; one extra host synchronisation
                                  per call or step.  bfs_run with
                                  SPMSPV_USE_GRAPH on a handle with a row
                                  form instead consumes the decision on the
                                  device (direction only, inside the captured
                                  level graph, no host synchronisation)       */
    SPMSPV_LEFT = 16384,       /* spmspv_run / _masked / _graphblas /
                                  _bitvector: left multiplication y' <- x' A
                                  (Background, Notation: the row-vector case),
                                  x' over A's m rows, y' over its n columns,
                                  y'(j) = Add over stored A(i,j), i in x', of
                                  Mult(A(i,j), x'(i)) (select2nd yields the x
                                  entry, as on the right).  Runs the push
                                  multiply on A^T through the CSR copy, so
                                  the handle needs SPMSPV_WITH_TRANSPOSE or
                                  SPMSPV_SYMMETRIC (EUNSUPPORTED otherwise);
                                  no selector, pull or tuned schedule         */
    SPMSPV_DETERMINISTIC = 32768 /* spmspv_workspace_size / _create (also
                                  _dcsc_): add the deterministic mode's
                                  storage (a second product list of nnz
                                  entries and a count matrix, about 10
                                  bytes per stored entry, plus 256 KiB).  spmspv_run /
                                  _masked with plus-times: y(i) is the fp32
                                  fold of row i's products, each rounded to
                                  fp32, in product order (x order, then the
                                  column's storage order), so its bits do
                                  not depend on the schedule, the bucket
                                  count or the GPU's timing; y ascending.
                                  Runs the scan, the product list, a stable
                                  radix sort by row (Algorithm 2's count
                                  matrix fixes every run's position) and a
                                  sequential fold per row (a row with k
                                  products takes k dependent adds), with no
                                  host synchronisation inside the call (the
                                  kernels read the product count on the
                                  device).  Min and
                                  or are order-free: their calls ignore it.
                                  EUNSUPPORTED on a handle created without
                                  it; with LEFT, the order is x' order then
                                  the row's storage order in the CSR copy   */
};

/* Launch schedule.  Changing it never changes int / bool results or any
 * output index set; fp32 plus-times sums may differ in rounding order.
 * Plus-times calls merge in fp64 cells: with merge_variant 0 a schedule
 * tile above 2^14 rows runs as 2^14 for them.                            */
typedef struct {
    int direction;      /* 0 = push (vector-driven, Algorithm 1); 1 = pull
                           (matrix-driven: scan every row of A against x;
                           needs SPMSPV_WITH_TRANSPOSE or SPMSPV_SYMMETRIC)  */
    int tile_log2;      /* rows per bucket = 2^tile_log2; buckets = ceil(m / 2^t)  */
    int scatter_block;  /* threads per bucketing workgroup (64..1024, power of 2)  */
    int scatter_items;  /* products per thread per chunk (1..16, power of 2)       */
    int merge_block;    /* threads per merge workgroup (64..1024, power of 2)      */
    int merge_variant;  /* 0 = sparse accumulator in LDS, one workgroup per bucket
                           (tile_log2 8..15);
                           1 = sparse accumulator in HBM (Algorithm 1 step 2
                               with the SPA in memory): a dense m-long array of
                               cells and a touched-row bitmap in the workspace,
                               updated with global atomics by several
                               workgroups per bucket, then walked in row order
                               and left empty; any bucket width (tile_log2
                               8..30).  Push calls of spmspv_run / _masked /
                               _graphblas / _bitvector and bfs_run; batched
                               calls merge in LDS                          */
    int launch;         /* push calls of spmspv_run / spmspv_run_masked:
                           0, 1 = three launches (scan, bucketing, merge: the
                               default, faster on gfx950),
                           2 = one launch of all three phases (one workgroup
                               per compute unit, exchanging through tagged
                               words; needs f <= 4096 per compute unit, at most
                               1024 buckets and no other work on the device
                               during the call, else EUNSUPPORTED or EDEVICE) */
} spmspv_schedule;

/* Bytes of device workspace spmspv_create needs for an m-by-n matrix with
 * nnz stored entries: buckets sized for nnz entries in total (the bound in
 * "Performance optimizations / Memory allocation"), per-call scan and bucket
 * counters, and BFS frontier buffers.  Pure host computation.
 * EINVAL if m, n < 1, nnz < 0, nnz >= 2^31 or bytes == NULL.            */
int spmspv_workspace_size(int64_t m, int64_t n, int64_t nnz, int flags, size_t* h_bytes);

/* Bind a CSC matrix (colptr int32[n+1], rowids int32[nnz], values float[nnz]
 * or NULL for a pattern matrix whose entries are all 1 / true) and a
 * workspace of ws_bytes device bytes.  Row ids inside a column may be in any
 * order (CSC does not require sorted columns).  Duplicate (i, j) entries are
 * combined with the semiring's Add, exactly as repeated products are.
 * Synchronous: runs set-up kernels on `stream` (row counts that size the
 * buckets, the maximum column length) and waits for them.  With
 * SPMSPV_VALIDATE it also checks colptr[0] == 0, colptr monotone,
 * colptr[n] == nnz and every row id in [0, m) on the device (EINVAL
 * otherwise).  The matrix arrays are borrowed, not copied.
 * Errors: EINVAL (null pointers, bad sizes, invalid CSC), ENOMEM (workspace
 * too small), EHIP.                                                       */
int spmspv_create(spmspv_handle* h_out, int64_t m, int64_t n, int64_t nnz, const int32_t* colptr,
                  const int32_t* rowids, const float* values, void* workspace, size_t ws_bytes, int flags,
                  void* stream);

/* ---- DCSC input (Background, "Sparse matrix and vector data structures":
 * only the nzc non-empty columns are stored, so the matrix takes O(nzc +
 * nnz) space instead of CSC's O(n + nnz)).  jc int32[nzc] holds the stored
 * column ids, strictly ascending in [0, n); cp int32[nzc+1] their starts
 * (cp[0] = 0, non-decreasing, cp[nzc] = nnz); rowids / values as for CSC.
 * The handle builds the auxiliary column index the format description
 * mentions (first stored column of every chunk of about n / nzc ids, in the
 * workspace), so an x entry finds its column in expected constant time; an
 * x entry naming a column absent from jc selects nothing.  The workspace
 * still holds per-x-entry tables sized by n (x may list every column).
 * Flags: SPMSPV_VALIDATE only (no transpose, so no pull direction and no
 * SPMSPV_LEFT).  The handle serves spmspv_run / _masked / _graphblas /
 * _bitvector (three-launch push multiply; no selector), the batched calls,
 * msbfs_run and bfs_run (bucketing levels only); pagerank_run and cc_run
 * need per-id column degrees and return EUNSUPPORTED.  Errors as for
 * spmspv_create, plus EINVAL for nzc outside [0, min(n, nnz)] or nzc == 0
 * with nnz > 0, and (on the device) jc not strictly ascending in [0, n). */
int spmspv_dcsc_workspace_size(int64_t m, int64_t n, int64_t nzc, int64_t nnz, int flags, size_t* h_bytes);
int spmspv_create_dcsc(spmspv_handle* h_out, int64_t m, int64_t n, int64_t nzc, int64_t nnz, const int32_t* jc,
                       const int32_t* cp, const int32_t* rowids, const float* values, void* workspace,
                       size_t ws_bytes, int flags, void* stream);

/* y <- A x (Algorithm 1 with Algorithm 2's counting), enqueued on `stream`.
 *   f                 : number of x entries (0 <= f <= n); indices must be
 *                       distinct (checked only with SPMSPV_VALIDATE; with
 *                       duplicates the device sets an error bit and y is
 *                       unspecified, memory stays safe).
 *   x_idx [f], x_val [f] : x in list form, any order.  x_val element type
 *                       per semiring (see enum); may be NULL with
 *                       X_VAL_IS_INDEX / X_ALL_TRUE.
 *   y_idx [y_capacity], y_val [y_capacity] : output list.  Unsorted order is
 *                       unspecified; with SPMSPV_SORTED_OUTPUT indices are
 *                       strictly ascending.  y_val may be NULL (pattern only).
 *   d_nnz_y           : device int64, receives nnz(y) (nullable).
 *   h_nnz_y           : host int64 (nullable).  When non-NULL the call waits
 *                       for the stream, stores nnz(y), and reports device
 *                       error bits (EDEVICE) and ECAPACITY.
 * nnz(y) <= min(m, sum of selected column lengths).  When nnz(y) exceeds
 * y_capacity only the first y_capacity entries are written; a capacity of m
 * always suffices.                                                        */
int spmspv_run(spmspv_handle A, int semiring, int flags, int64_t f, const int32_t* x_idx, const void* x_val,
               int32_t* y_idx, void* y_val, int64_t y_capacity, int64_t* d_nnz_y, int64_t* h_nnz_y,
               void* stream);

/* spmspv_run with an output mask (the masked SpMSpV of Conclusions and
 * Future Work): `mask` is a device bitmap of ceil(m / 32) uint32 words; row
 * i is excluded from y when bit (i & 31) of word i >> 5 is set, and its
 * products are dropped before bucketing.  NULL mask = spmspv_run.       */
int spmspv_run_masked(spmspv_handle A, int semiring, int flags, int64_t f, const int32_t* x_idx,
                      const void* x_val, const uint32_t* mask, int32_t* y_idx, void* y_val, int64_t y_capacity,
                      int64_t* d_nnz_y, int64_t* h_nnz_y, void* stream);

/* Breadth-first search from `root` by repeated SpMSpV on the frontier
 * (Results, "Performance of SpMSpV algorithms when used in BFS"; the
 * frontier-expansion pattern of the Introduction), with the visited set as
 * a mask applied to each product (the masked SpMSpV of Conclusions and
 * Future Work).  Requires m == n.  Edges are j -> i for stored A(i, j).
 *   semiring MIN_SELECT2ND_I32 : x value = vertex id, so a reached vertex's
 *       parent is its smallest in-neighbour on the previous level.
 *   semiring OR_AND_BOOL       : reachability only; parent must be NULL.
 *   level [n]  : out, hop count from root, -1 if unreached.
 *   parent [n] : out (nullable), parent[root] = root, -1 if unreached.
 *   h_num_levels : out (nullable), number of non-empty levels.
 * Synchronous (waits once per batch of levels to test for an empty
 * frontier).  With SPMSPV_USE_GRAPH the per-level kernels are captured
 * once in a hipGraph and replayed.                                        */
int bfs_run(spmspv_handle A, int semiring, int32_t root, int flags, int32_t* level, int32_t* parent,
            int32_t* h_num_levels, void* stream);

/* ---- autotuner.  Bucket count (tile_log2), bucketing workgroup shape,
 * merge workgroup size and direction are searched by timing the library's
 * own calls (coordinate descent, two passes, then the pull direction when
 * the handle has it), per density band, on inputs drawn on the device
 * (each column with probability `density`, values in (0, 1]).  The paper's
 * CPU choice of 4t buckets ("Performance optimizations") is the analogue
 * this replaces.  The best schedule of each band is kept in the handle and
 * used by spmspv_run with SPMSPV_AUTO_SCHEDULE.  Never changes int / bool
 * results or index sets.                                                 */
typedef struct {
    double density;           /* band                                      */
    int64_t f;                /* x entries drawn for it                    */
    spmspv_schedule sched;    /* fastest schedule found                    */
    double us;                /* its time per call (microseconds)          */
    double default_us;        /* the default schedule's time per call      */
} spmspv_tune_entry;

/* Synchronous.  x_idx [n], x_val [n] (float, plus-times only; NULL
 * otherwise), y_idx [m], y_val [m] (4 bytes per entry) are caller scratch.
 * reps timed calls per candidate.  h_out [ndens] (nullable).  1 <= ndens
 * <= 64, densities in (0, 1].                                            */
int spmspv_autotune(spmspv_handle A, int semiring, const double* h_densities, int ndens, int reps, int32_t* x_idx,
                    void* x_val, int32_t* y_idx, void* y_val, spmspv_tune_entry* h_out, void* stream);

/* The tuned schedule spmspv_run would use for f x entries (EINVAL before
 * spmspv_autotune).                                                       */
int spmspv_tuned_schedule(spmspv_handle A, int64_t f, spmspv_schedule* h_sched);

/* Persisted tuning tables.  spmspv_tuning_save writes the handle's table
 * (after spmspv_autotune; EINVAL before) to the text file `path`, keyed by
 * the device (name, gfx architecture, compute units), the library's device
 * sources (spmspv_source_digest) and the matrix (m, n, nnz and a hash of
 * 4096 evenly spaced entries of its column pointers and of its row ids);
 * format version 1.  spmspv_tuning_load installs a saved table on a handle
 * whose device, library and matrix all match (then AUTO_SCHEDULE calls use
 * it), else EUNSUPPORTED and the handle is unchanged; EINVAL for a missing,
 * malformed or other-version file.  Both read a few device values and
 * wait for `stream`.                                                      */
int spmspv_tuning_save(spmspv_handle A, const char* path, void* stream);
int spmspv_tuning_load(spmspv_handle A, const char* path, void* stream);

/* Digest of the device sources this library was built from (16 hex
 * digits; the selector's weights and tuning tables record it).            */
const char* spmspv_source_digest(void);

/* Tune the batched-call schedule on one given batch (arguments as for
 * spmspv_run_batch), keep the fastest with spmspv_set_batch_schedule's
 * effect, and report it and its time per call.  Synchronous.             */
int spmspv_autotune_batch(spmspv_handle A, int semiring, int flags, int nbatch, const int64_t* x_off,
                          const int32_t* x_idx, const void* x_val, int64_t* y_off, int32_t* y_idx, void* y_val,
                          int64_t y_capacity, int reps, spmspv_schedule* h_best, double* h_us, void* stream);

/* Read / replace the launch schedule (NULL restores the default).  While
 * the default is in place, spmspv_run sizes the scatter chunk per call from
 * the expected product count f * nnz / n: the largest chunk, up to 4096
 * products, that still gives every compute unit one (see
 * spmspv_effective_schedule).                                             */
int spmspv_get_schedule(spmspv_handle A, spmspv_schedule* h_sched);
int spmspv_set_schedule(spmspv_handle A, const spmspv_schedule* h_sched);

/* The schedule spmspv_run(A, semiring, flags, f, ...) would launch with:
 * the tile that semiring merges with, and for push calls the launch mode
 * (1 = three launches, 2 = one launch).                                  */
int spmspv_effective_schedule(spmspv_handle A, int semiring, int64_t f, int flags, spmspv_schedule* h_sched);

/* Statistics of the most recent spmspv_run / BFS level (synchronous):
 * h_out[0] = products W (sum of selected column lengths, the work bound of
 * the lower-bound section), [1] = nnz(y), [2] = non-empty selected columns,
 * [3] = maximum selected column length, [4] = device error bits,
 * [5] = selector class of the last SPMSPV_USE_SELECTOR call.  h_out holds
 * 6 entries.                                                              */
int spmspv_last_stats(spmspv_handle A, int64_t* h_out, void* stream);

/* Per-kernel timing of calls made with SPMSPV_PROFILE: waits for the
 * recorded events, writes the summed milliseconds of each phase
 * (0 = scan, 1 = bucket scatter, 2 = merge + compaction) to h_ms[3] and the
 * number of profiled calls to *h_calls, then clears the record.  A call
 * made in one launch records its kernel under phase 0 (1 and 2 stay 0).  */
int spmspv_profile_read(spmspv_handle A, double* h_ms, int64_t* h_calls);

/* Release the handle (host memory and HIP events only; the caller frees
 * its device arrays and workspace).                                       */
int spmspv_destroy(spmspv_handle A);

/* ---- connected components (the paper's introduction lists them among the
 * data-driven uses of SpMSpV).  Label propagation: label(v) = v; each step
 * multiplies x = {(v, label(v)) : v's label changed in the last step (all
 * vertices with out-edges at first)} over min-select2nd, and every row i
 * with y(i) < label(i) takes y(i) and joins the next x; it stops when no
 * label changes.  Result: labels[v] = the smallest vertex that reaches v
 * along edges j -> i of the stored A(i, j); for a symmetric A (undirected
 * graph), the smallest vertex of v's component.  labels: int32 [n]
 * (device).  *h_iters (nullable) = multiplies run.  Square A; uses the
 * handle's BFS buffers.  Synchronous (one host check per 8 steps).     */
int cc_run(spmspv_handle A, int flags, int32_t* labels, int32_t* h_iters, void* stream);

/* ---- masked multiply with accumulate and replace: w<mask, replace> =
 * w accum (A x), the generalisation of the BFS visited mask that the
 * paper's conclusions name as future work, with the rules of the GraphBLAS
 * standard.
 *   t = A x over `semiring` (structural pattern, as spmspv_run).
 *   Mask: mask_idx == NULL: every row is in the mask.  Otherwise the rows
 *     listed in mask_idx[0..mask_count) (distinct, in [0, m)); with
 *     mask_val (uint8 [mask_count]) non-NULL a listed row counts only if its
 *     value is nonzero (a value mask), else every listed row does (a
 *     structural mask).  SPMSPV_MASK_COMPLEMENT inverts membership (with no
 *     mask list: no row is in the mask).
 *   w: w_idx [w_count] strictly ascending rows in [0, m), w_val [w_count]
 *     (element type of y: float, int32 or uint8).
 *   accum: NONE, ADD (the semiring's Add: + in fp32, min, or), FIRST (w),
 *     SECOND (t).  z(i) = accum(w(i), t(i)) where both exist and an
 *     operator is given; t(i) where t has the row; w(i) where only w has
 *     it and an operator is given.
 *   Result: z(i) for rows in the mask; for the other rows w(i), or nothing
 *     with SPMSPV_MASK_REPLACE.  y is always ascending.
 * The mask is applied inside the product (products of rows outside it are
 * dropped before bucketing), then t and w are merged.  flags: VALIDATE
 * (host checks of x, the mask list and w's order), X_VAL_IS_INDEX,
 * X_ALL_TRUE, LEFT (then x lies over A's rows and the mask, w and y over
 * its columns).  Device checks report mask or w indices out of range
 * (EDEVICE) and a w that is not ascending.  Uses the handle's list scratch
 * for its temporaries.  Push direction always.                            */
enum spmspv_mask_flags {
    SPMSPV_MASK_COMPLEMENT = 1,
    SPMSPV_MASK_REPLACE = 2
};
enum spmspv_accum {
    SPMSPV_ACCUM_NONE = 0,
    SPMSPV_ACCUM_ADD = 1,
    SPMSPV_ACCUM_FIRST = 2,
    SPMSPV_ACCUM_SECOND = 3
};
int spmspv_run_graphblas(spmspv_handle A, int semiring, int flags, int64_t f, const int32_t* x_idx,
                         const void* x_val, const int32_t* mask_idx, const uint8_t* mask_val, int64_t mask_count,
                         int mask_flags, int accum, const int32_t* w_idx, const void* w_val, int64_t w_count,
                         int32_t* y_idx, void* y_val, int64_t y_capacity, int64_t* d_nnz_y, int64_t* h_nnz_y,
                         void* stream);

/* ---- bitvector x and y (Background, "Sparse matrix and vector data
 * structures": a bitmap over the vector's length plus the values of the
 * present indices in ascending index order).  y is produced in the same
 * format as x (the paper's rule for the output format).
 *   x_bits  uint32[ceil(len_x / 32)]: bit (i mod 32) of word i / 32 set when
 *           index i is present; len_x = n (m with SPMSPV_LEFT).  A set bit
 *           at or past len_x is ignored and reported (EDEVICE with h_nnz_y).
 *   x_val   the present entries' values, ascending by index (type per
 *           semiring; NULL with X_VAL_IS_INDEX / X_ALL_TRUE).
 *   y_bits  uint32[ceil(len_y / 32)], every word written (len_y = m, or n
 *           with SPMSPV_LEFT); y_val [y_capacity] the present entries'
 *           values ascending by index (nullable: pattern only).
 *   d_nnz_y / h_nnz_y as for spmspv_run (ECAPACITY when nnz(y) exceeds
 *           y_capacity: y_bits still holds every row of y, y_val the
 *           values of the first y_capacity rows).
 * Flags: X_VAL_IS_INDEX, X_ALL_TRUE, LEFT, SORTED_OUTPUT (implied).  The
 * bitmap is expanded to its index list on the device, the product runs as
 * a device-sized spmspv_run (push, the handle's schedule), and the merge
 * writes y's bitmap from its tiles' bitmaps of touched rows; the index
 * lists use the handle's list scratch.                                   */
int spmspv_run_bitvector(spmspv_handle A, int semiring, int flags, const uint32_t* x_bits, const void* x_val,
                         uint32_t* y_bits, void* y_val, int64_t y_capacity, int64_t* d_nnz_y, int64_t* h_nnz_y,
                         void* stream);

/* ---- allocation-free multiply.  For callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, hosts that forbid
 * allocation): y <- A x as spmspv_create followed by spmspv_run would
 * compute it, with no handle and no workspace argument.  The workspace lives
 * in a device array of the library's own, 64 MiB per device, held until the
 * process ends, so the call allocates nothing: matrices whose
 * spmspv_workspace_size(m, n, nnz, 0) exceeds 64 MiB are refused with
 * EINVAL (about nnz <= 5M with m, n <= 1M; *h_scratch_bytes, when
 * non-NULL, receives the size needed).  Arguments and results are those of
 * spmspv_create and spmspv_run (flags: SORTED_OUTPUT, X_VAL_IS_INDEX,
 * X_ALL_TRUE); each call also sizes the buckets from A (one pass over the
 * row ids), which a handle does once.  Every call on a device shares that
 * device's array: calls that overlap on one device (other streams, other
 * host threads) race and must be ordered by the caller.                  */
int spmspv_run_static(int64_t m, int64_t n, int64_t nnz, const int32_t* colptr, const int32_t* rowids,
                      const float* values, int semiring, int flags, int64_t f, const int32_t* x_idx,
                      const void* x_val, int32_t* y_idx, void* y_val, int64_t y_capacity, int64_t* d_nnz_y,
                      int64_t* h_nnz_y, size_t* h_scratch_bytes, void* stream);

/* ---- data-driven PageRank (the Introduction names PageRank among the
 * data-driven SpMSpV uses, where a vertex stops sending updates once its
 * value has converged; the paper gives no formula, this is the delta form):
 *   rank = 0, delta = (1 - d) / n everywhere, every vertex active;
 *   each step: rank += delta; x = { (j, d * delta(j) / outdeg(j)) : j active,
 *   outdeg(j) > 0 } with outdeg(j) the stored entries of column j (edge
 *   j -> i for stored A(i, j)); delta = A x (plus-times SpMSpV); vertex j
 *   stays active when delta(j) > tol * rank(j) (rank before adding);
 *   stop when no vertex is active or after max_iter multiplies.
 * Mass of columns without entries is dropped.  fp32 on the device.       */

/* Scratch bytes pagerank_run needs (16 n + 256). */
int pagerank_scratch_size(spmspv_handle A, size_t* h_bytes);

/* Needs m == n and a pattern handle (values NULL): A_n's entries are
 * 1 / outdeg.  rank [n] (device float) receives the result.  Flags:
 * SPMSPV_USE_SELECTOR picks each multiply's schedule with the loaded
 * selector (one host synchronisation per step; without it the host checks
 * every 8 steps); with SPMSPV_USE_GRAPH as well (and a row form) the
 * selector's direction is consumed on the device, gating the push and pull
 * kernels, and the host checks every 8 steps (bucket count: the handle's
 * schedule; spmspv_selector_classes then reports nothing).
 * *h_iters = multiplies performed.  Synchronous.                          */
int pagerank_run(spmspv_handle A, float damping, float tol, int max_iter, int flags, float* rank, void* scratch,
                 size_t scratch_bytes, int32_t* h_iters, void* stream);

/* ---- batched calls (many x against one A in one launch sequence).
 * x is the concatenation of nbatch vectors: vector b occupies positions
 * [x_off[b], x_off[b+1]) of x_idx / x_val (x_off int64, device, x_off[0]
 * = 0).  Its products are bucketed by key (b, row range), into fixed or
 * counted slices (below; the counting pass plays Algorithm 2's role), and
 * merged per key; the
 * results come out one vector after another, each ascending, vector b at
 * [y_off[b], y_off[b+1]) of y_idx / y_val.  Every x, y and offset array is
 * device memory.  The batch workspace is a second caller-owned buffer. */

/* Bytes of the batch workspace for up to max_batch vectors (<= 1024) with
 * at most max_f x entries and max_products products (sum of selected column
 * lengths, < 2^31) in one call.  With SPMSPV_MSBFS max_f is taken as
 * max_batch * n and max_products <= 0 as max_batch * nnz (the most one BFS
 * level can produce), plus frontier and visited buffers; needs m == n and
 * max_batch * n < 2^31.                                                   */
int spmspv_batch_workspace_size(spmspv_handle A, int max_batch, int64_t max_f, int64_t max_products, int flags,
                                size_t* h_bytes);

/* Bind a batch workspace of ws_bytes device bytes (owned by the caller,
 * borrowed until the handle is destroyed or another is attached).  The
 * scan's look-back words inside it are cleared on `stream` (a hipStream_t,
 * NULL = default stream); batched calls on other streams must be ordered
 * after that clear by the caller. */
int spmspv_batch_attach(spmspv_handle A, int max_batch, int64_t max_f, int64_t max_products, int flags,
                        void* workspace, size_t ws_bytes, void* stream);

/* y_b <- A x_b for b < nbatch, one scan, the bucketing and one merge
 * launch for the whole batch.  Flags: SPMSPV_X_VAL_IS_INDEX, X_ALL_TRUE
 * and SPMSPV_VALIDATE (host check of x_off and of distinct in-range indices
 * per vector; synchronous) as for spmspv_run.  Indices inside one vector
 * must be distinct, as for spmspv_run.
 *   Fixed slices: when the workspace's max_products >= nbatch * nnz(A),
 *   vector b's products for bucket k go to a slice of its own sized by the
 *   stored entries of k's rows, and the bucketing is one pass.  A repeated
 *   index can overflow a slice: the run is dropped (memory stays safe) and
 *   the status is EDEVICE.
 *   Counted slices: otherwise a counting pass sizes every (vector, bucket)
 *   key first; repeated indices are then combined like repeated products.
 * y is always ascending within a vector.  y_off [nbatch+1] receives the
 * output offsets.  With h_nnz_total non-NULL the call waits and reports the
 * total (ECAPACITY when it exceeds y_capacity, or when the products exceed
 * the workspace's max_products; then y is unspecified).  The bucket tile is
 * the narrowest at or above the schedule's for which nbatch * ceil(m / tile)
 * <= 8192 (EUNSUPPORTED if none).                                        */
int spmspv_run_batch(spmspv_handle A, int semiring, int flags, int nbatch, const int64_t* x_off,
                     const int32_t* x_idx, const void* x_val, int64_t* y_off, int32_t* y_idx, void* y_val,
                     int64_t y_capacity, int64_t* h_nnz_total, void* stream);

/* Schedule for batched calls (tile_log2 is the starting tile; NULL restores
 * the handle's schedule) and the effective one for nbatch vectors of the
 * given semiring (plus-times merges in fp64 cells, so its tiles hold at
 * most 2^14 rows; see spmspv_schedule).                                   */
int spmspv_set_batch_schedule(spmspv_handle A, const spmspv_schedule* h_sched);
int spmspv_get_batch_schedule(spmspv_handle A, int semiring, int nbatch, spmspv_schedule* h_sched);

/* Multi-source BFS: nsrc independent searches from h_roots[0..nsrc) run as
 * one batched SpMSpV per level (the frontiers of all sources form one
 * batch; source x's visited bitmap masks its own products).  level and
 * parent are [nsrc][n] int32 (parent nullable; NULL for OR_AND), with the
 * conventions of bfs_run per source.  Needs a batch workspace attached with
 * SPMSPV_MSBFS and max_batch >= nsrc.  Synchronous.
 *   flags: SPMSPV_DIRECTION_OPT on a handle with a row form
 *   (SPMSPV_WITH_TRANSPOSE or SPMSPV_SYMMETRIC; for MIN_SELECT2ND the rows
 *   must be ascending, as a symmetric handle's sorted columns are) switches
 *   all searches to the pull direction once the frontiers' summed column
 *   lengths exceed the sources' unexplored edges / 14 (the frontier-edge
 *   rule summed over sources; the Conclusions name direction switching as
 *   future work): one step then scans each vertex's in-neighbours against
 *   one-bit-per-source frontier masks for every source at once, and the
 *   searches stay pull to the end.  Same levels and parents (the smallest
 *   frontier in-neighbour).  Without a usable row form the flag is
 *   ignored.  One host read per level.                                    */
int msbfs_run(spmspv_handle A, int semiring, int nsrc, const int32_t* h_roots, int flags, int32_t* level,
              int32_t* parent, int32_t* h_num_levels, void* stream);

/* ---- schedule selector (a learned replacement for the fixed bucket count
 * of "Performance optimizations"; see the bucket-count discussion there).
 * The selector is a fully connected network 6 -> 64 -> 64 -> 10 with ReLU
 * after both hidden layers, fp32.  Parameter layout (5258 floats):
 *   W1[64][6], b1[64], W2[64][64], b2[64], W3[10][64], b3[10].
 * Inputs are log2(1 + v) of six per-call quantities the scan produces --
 * f, W (products), max selected column length, n, nnz/n, unvisited rows
 * (BFS; n otherwise) -- each standardised as (v - mean[c]) / std[c].
 * Output class c in 0..8 = push with 2^(c+4) buckets (tile clamped to what
 * LDS holds); 9 = pull direction (push tile of class 8 when the handle has
 * no row form).                                                           */

/* Copy host weights and feature standardisation to the handle (synchronous).
 * EINVAL for non-finite weights or std <= 0 (the selector is then disabled). */
int spmspv_selector_load(spmspv_handle A, const float* h_params, const float* h_mean, const float* h_std,
                         void* stream);

/* Classes chosen per step by the most recent bfs_run or pagerank_run with
 * SPMSPV_USE_SELECTOR: writes min(cap, count) entries, *h_count = count.  */
int spmspv_selector_classes(spmspv_handle A, int32_t* h_out, int32_t cap, int32_t* h_count);

/* Replay a class sequence: while set (count > 0), bfs_run and pagerank_run
 * with SPMSPV_USE_SELECTOR run step k (BFS level / PageRank multiply) with
 * class h_classes[k] (0..9) instead of the network's choice, in the same
 * host-driven loop (steps past the end use the network).  count = 0 clears
 * it.  Used to time a schedule found in hindsight under exactly the loop the
 * selector runs in.                                                       */
int spmspv_force_classes(spmspv_handle A, const int32_t* h_classes, int32_t count);

/* Standardised features of the most recent selector decision (h_out[6],
 * in the order above; synchronous).                                      */
int spmspv_selector_features(spmspv_handle A, float* h_out, void* stream);

/* tile_log2 that class `cls` (0..8) runs with on this handle, before the
 * plus-times narrowing; -1 for 9.  Class c is push with 2^(c+4) buckets
 * (tile ceil(log2 m) - c - 4, between 2^8 and 2^15 rows).                */
int spmspv_class_tile(spmspv_handle A, int cls, int32_t* h_tile_log2);

/* The whole schedule class `cls` (0..9) runs with for `semiring` (its LDS
 * tile, narrowed for plus-times' fp64 cells), or the pull direction for 9
 * (EUNSUPPORTED without a row form).                                      */
int spmspv_class_schedule(spmspv_handle A, int semiring, int cls, spmspv_schedule* h_sched);

/* Number of selector parameters (5258). */
int spmspv_mlp_param_count(void);

/* logits[batch][10] <- MLP(params, X[batch][6]) on the device.          */
int spmspv_mlp_forward(const float* params, const float* X, int batch, float* logits, void* stream);

/* One training step on the device: mean softmax cross-entropy of
 * (X[batch][6], labels[batch] in 0..9), its gradient by backpropagation,
 * then (lr > 0) one Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias
 * correction with `step` >= 1) of params / adam_m / adam_v in place.
 * grad [5258] and d_loss [1] receive the gradient and loss (nullable).
 * 1 <= batch <= 128; one workgroup; sums in a fixed order.               */
int spmspv_mlp_train_step(float* params, float* adam_m, float* adam_v, int step, float lr, const float* X,
                          const int32_t* labels, int batch, float* grad, float* d_loss, void* stream);

/* Static description of a status code; detail of the last error on this
 * host thread. */
const char* spmspv_status_string(int status);
const char* spmspv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPMSPV_H */
