// Internal declarations shared by the HIP kernels and the C-ABI layer of the
// SpMSpV library.  Not installed; the public interface is include/spmspv.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace spv {

constexpr int kWave = 64;

// Wait until every vector memory operation this wave has issued (loads,
// stores, atomics) has completed: s_waitcnt with vmcnt = 0 and the other
// counters at their maximum (gfx9 encoding: vmcnt bits 3:0 and 15:14,
// expcnt 6:4, lgkmcnt 11:8).
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Device error bits (Ctrl::err), sticky until the host reads them.
enum : uint32_t {
    ERR_X_RANGE = 1u,          // an x index outside [0, n)
    ERR_BUCKET_OVERFLOW = 2u,  // a bucket received more entries than its rows
                               // hold in A (only possible with duplicate x)
    ERR_SPIN = 4u,             // a look-back wait exceeded its bound
    ERR_CSC = 8u,              // colptr not monotone / wrong ends (create)
    ERR_ROW_RANGE = 16u,       // a row id outside [0, m) (create)
    ERR_INDEX_RANGE = 32u,     // a mask or accumulation input index outside [0, m)
    ERR_ORDER = 64u            // accumulation input indices not strictly ascending
};

enum Semiring : int { SR_PLUS_TIMES = 0, SR_MIN_SELECT2ND = 1, SR_OR_AND = 2 };

// How the scan phase reads x values.
enum XMode : int { XV_BITS32 = 0, XV_INDEX = 1, XV_U8 = 2, XV_TRUE = 3 };

// Device-resident control block, one per handle (first 256 B of the workspace).
struct alignas(256) Ctrl {
    int32_t f;              // frontier length for device-driven loops (BFS)
    int32_t fnz;            // selected columns with at least one entry
    int32_t W;              // products = sum of selected column lengths
    int32_t maxlen;         // running max selected column length (scan phase)
    uint32_t ticket_scan;   // work tickets of the scan phase (reset by scatter)
    uint32_t ticket_merge;  // work tickets of the merge phase (reset by scan)
    int32_t level;          // BFS level being produced
    uint32_t err;           // sticky error bits
    int64_t nnz_y;          // nnz(y) of the last merge phase
    int32_t maxlen_last;    // maxlen of the last completed scan phase
    int32_t maxdeg;         // longest column of A (create)
    int32_t fnz_last;
    int32_t W_last;
    int32_t* bfs_level;     // BFS output arrays, set by the BFS init kernel so a
    int32_t* bfs_parent;    // captured level graph does not bake them in
    int32_t dir;            // direction of the current BFS level: 0 push, 1 pull
    int32_t policy;         // BFS direction policy: 0 push only, 1 frontier-edge heuristic
    int64_t edges_left;     // stored entries in columns of unvisited vertices
    uint32_t unsorted;      // set at create when some column's row ids are not ascending
    uint32_t pad0;
    int64_t seen;           // BFS: vertices reached so far (selector feature)
    int32_t bfs_mode;       // the selector runs inside a BFS
    int32_t cls;            // class chosen by the selector for the current multiply
    float features[6];      // standardised selector features of the current multiply
    int32_t gen_count;      // entries drawn by the tuning-input generator / appended by a PageRank step
    // Direction-switching BFS after a pull level: that level's emit leaves the
    // next frontier in the pull direction's x bitmap and per-workgroup sums
    // of its column lengths in the pull workspace (chain_ready = 1); the next
    // scan takes the direction decision itself and publishes chain_word =
    // 2 | direction, which the decision kernel then consumes instead of
    // deciding again.
    uint32_t chain_ready;
    uint32_t chain_word;
    // One-launch multiply: call counter whose value tags this call's
    // exchange and look-back words (advanced once per call on the device).
    uint32_t fused_epoch;
    int32_t maxrow;         // longest row of A (create, with the transpose)
    int64_t aux_count;      // masked multiply: length of the masked product before the combine
    int32_t bv_f;           // bitvector call: x entries found in its bitmap
    uint32_t pad[21];
};
static_assert(sizeof(Ctrl) == 256, "Ctrl must stay 256 bytes");

// Scan phase: gather the selected column ranges, prefix-sum their lengths,
// compact the non-empty ones and mark where each product chunk starts.
struct ScanArgs {
    const int32_t* colptr;   // CSC: [n+1]; DCSC: the [nzc+1] column starts
    int32_t n;
    // DCSC (dcsc = 1): column j is the k-th stored one when dc_jc[k] == j,
    // searched in [dc_aux[j >> dc_shift], dc_aux[(j >> dc_shift) + 1]); a
    // column absent from dc_jc is empty (with no stored column dc_jc may be
    // null and is never read).
    int dcsc;
    const int32_t* dc_jc;
    const int32_t* dc_aux;
    int32_t dc_shift;
    const int32_t* x_idx;
    const void* x_val;
    int xmode;
    int32_t f_host;          // used when f_dev == nullptr
    const int32_t* f_dev;    // device frontier length (BFS)
    Ctrl* ctrl;
    int32_t* cstart;         // [fnz] first entry of each non-empty column
    int32_t* coff;           // [fnz+1] exclusive prefix of lengths
    uint32_t* cxv;           // [fnz] x value bits
    int32_t* chunk_col;      // [nchunks] first column of each product chunk
    int chunk_log2;          // products per chunk = 2^chunk_log2
    uint64_t* lb1;           // look-back words of this phase (zero on entry):
                             // [lb1_n] product sums, then [lb1_n] column counts
    int32_t lb1_n;
    int64_t nnz;             // products above this mean duplicate x indices
    int64_t chunk_n;         // entries of chunk_col
    int32_t* cursor;         // bucket fill counters, cleared here for scatter
    uint64_t* lb3;           // merge look-back words, cleared here
    int32_t nb;              // buckets of the current schedule
    int bump_level;          // BFS: advance ctrl->level when f > 0
    int wide;                // 1: tiles of kScanItemsWide items per thread (large or device-known f)
    // Direction-switching BFS with the pull direction: 1 heuristic, 2
    // selector (weights in sel), 0 otherwise.  After a pull level the scan
    // decides the direction itself and builds no tables for a pull level; on
    // a push level it clears the x bits that pull level left.
    int chain;
    const float* sel;
    int has_pull;
    uint32_t* xbits;
    const int64_t* chain_part;   // [2 * chain_nparts] the previous emit's per-workgroup column sums
    int32_t chain_nparts;
    // Batched calls: x is the concatenation of nbatch vectors, vector b at
    // positions [xoff[b], xoff[b+1]); xoff[nbatch] (read on the device) is the
    // total length and must not exceed f_cap.
    const int64_t* xoff;     // nullable: single-vector call
    int32_t nbatch;
    int64_t f_cap;
    int32_t* cxid;           // [fnz] vector of each non-empty column
    int32_t* kcount;         // [nb+1] per-key product counts, cleared here
};

// Scatter phase: products -> row-range buckets.
struct ScatterArgs {
    const int32_t* rowids;
    const float* values;     // nullable (pattern)
    Ctrl* ctrl;
    const int32_t* cstart;
    const int32_t* coff;
    const uint32_t* cxv;
    const int32_t* chunk_col;
    int chunk_log2;
    int tile_log2;
    int32_t nb;
    int32_t m;
    const int32_t* rcp;      // [m+1] prefix of row counts of A = bucket bases
    int32_t* cursor;         // [nb]
    // Batched calls: key = vector * nbx + (row >> tile_log2); bases come from
    // an exact count pass (kcount, then its exclusive scan kbase).
    const int32_t* cxid;
    int32_t* kcount;         // [nb] count pass output
    const int32_t* kbase;    // [nb+1] bucket bases of the batched scatter
    int32_t nbx;             // buckets per vector
    int32_t mask_words;      // words per vector in a batched mask
    int64_t xstride;         // > 0: fixed bases, key (x, b) owns slots x * xstride + [rcp[bT], rcp[(b+1)T])
                             // (no counting pass; needs bucket storage of nbatch * nnz)
    uint2* buckets;          // [nnz] (row, value bits)
    const uint32_t* mask;    // nullable row bitmap: drop rows whose bit is set (mask_keep = 0, the BFS
                             // visited set) or whose bit is clear (mask_keep = 1, a GraphBLAS mask)
    int mask_keep;
    uint64_t* lb1;           // scan look-back words to clear (two halves of lb1_n)
    int32_t lb1_n;
    int32_t lb1_clear;       // how many of each half to clear
    int32_t f_host;
    const int32_t* f_dev;
    int gate;                // 1: skip the work when ctrl->dir selects pull
};

// Merge + compaction phase: one workgroup per bucket.
struct MergeArgs {
    Ctrl* ctrl;
    const int32_t* cursor;
    const uint2* buckets;
    const int32_t* rcp;
    int32_t m;
    int tile_log2;
    int32_t nb;
    uint64_t* lb3;
    int32_t* y_idx;
    void* y_val;             // nullable
    int64_t y_cap;
    int64_t* d_nnz_y;        // nullable
    uint32_t* visited;       // BFS: visited bitmap, updated with new vertices
    int set_f;               // BFS: publish nnz(y) as the next frontier length
    int gate;                // 1: skip when ctrl->dir selects pull
    // Batched calls (key = vector * nbx + bucket)
    const int32_t* kbase;    // [nb+1] (counted bases), unused when xstride > 0
    int64_t xstride;         // > 0: fixed bases as in ScatterArgs
    int32_t nbx;
    int32_t nbatch;
    int64_t* yoff;           // [nbatch+1] out: start of each vector's y
    int64_t n_stride;        // BFS: level / parent entries per vector
    int32_t mask_words;      // BFS: visited words per vector
    // Merge through the HBM sparse accumulator (merge variant 1): dense
    // cells for every row, empty between calls (plus-times fp64 at -0.0,
    // min-select2nd int32 at INT32_MAX, or-and value bits clear) and the
    // touched-row bitmap (clear between calls).
    double* h_f64;
    int32_t* h_i32;
    uint32_t* h_orbits;
    uint32_t* h_touched;
    int32_t h_split;         // workgroups per bucket in the accumulation
    // bitvector output (single calls, not BFS or batched): every word of y's
    // bitmap is written from the tiles' touched-row bitmaps; nullable
    uint32_t* y_bits;
};
// Merge variant 1: rows per output tile of the in-order walk.
constexpr int kHTileRows = 65536;
inline int64_t hmerge_tiles(int64_t m) { return (m + kHTileRows - 1) / kHTileRows; }
// Accumulate every bucket entry into the HBM cells, then walk the touched
// rows in order, writing y (and the BFS outputs) and emptying the cells.
// Uses lb3[0, hmerge_tiles(m)) as look-back words (zero on entry).
hipError_t launch_hbm_merge(const MergeArgs& a, int semiring, bool bfs, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t count, hipStream_t s);

// Pull (matrix-driven) direction over the CSR form of A.
struct PullArgs {
    Ctrl* ctrl;
    int32_t m, n;
    int64_t nnz;
    const int32_t* rowptr;   // [m+1]
    const uint32_t* colids;  // [nnz]
    const float* values;     // [nnz] CSR values, nullable
    const int32_t* part;     // [pull_blocks+1] merge-path partition
    int pull_blocks;
    const int32_t* x_idx;
    const void* x_val;
    int32_t f_host;
    const int32_t* f_dev;
    uint32_t* xbits;         // [n/32] zero between calls
    uint32_t* xdense;        // [n]
    uint32_t* ybits;         // [m/32] zero between calls
    uint32_t* ydense;        // [m] semiring identity between calls
    const uint32_t* mask;    // nullable: rows to skip (BFS visited)
    uint64_t* lbp;           // [emit_blocks] look-back words
    int emit_blocks;
    int32_t* y_idx;
    void* y_val;
    int64_t y_cap;
    int64_t* d_nnz_y;
    uint32_t* visited;
    int set_f;
    int bump_level;
    int gate;                // 1: skip when ctrl->dir selects push
    // BFS level of a direction-switching BFS: the emit writes the next
    // frontier's bitmap over xbits and sums its column lengths (colptr) for
    // the next decision; prep leaves xbits as the previous emit wrote them.
    int chain;
    const int32_t* colptr;
    int64_t* chain_part;     // [2 * emit_blocks]: per workgroup, stored entries and (longest << 32 | non-empty)
    int x_index;             // x value = vertex id: read j instead of xdense[j]
};

constexpr int kPullBlock = 256;
constexpr int kPullItems = 8;
constexpr int kPullChunk = kPullBlock * kPullItems;

// rowwise: one thread per unmasked row with first-hit exit (the bottom-up BFS
// step; min-select2nd and or-and only) instead of the merge-path kernel.
hipError_t launch_pull(const PullArgs& a, int semiring, int xmode, bool bfs, bool early, bool rowwise,
                       hipStream_t s);
hipError_t launch_pull_setup(const int32_t* colptr, const int32_t* rowids, const float* values, int32_t m,
                             int32_t n, int64_t nnz, const int32_t* rowptr, int32_t* cursor, int32_t* colids,
                             float* tvalues, int32_t* part, uint32_t* unsorted, hipStream_t s);
hipError_t launch_clear_u64(uint64_t* p, int n, hipStream_t s);
hipError_t launch_fill_ident(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
int pull_emit_blocks(int32_t m);
int pull_blocks(int32_t m, int64_t nnz);

size_t merge_lds_bytes(int tile_log2, int semiring);
size_t scatter_lds_bytes(int nb, int chunk, bool batch = false);
// Scatter workgroups resident per compute unit (registers, LDS, threads).
int scatter_resident(int semiring, int block, int items, int nb, bool batch);
constexpr int kMaxBatch = 1024;    // vectors per batched call
hipError_t launch_scatter_batch(const ScatterArgs& a, int semiring, int block, int items, int grid, bool count,
                                hipStream_t s);
// Masked multiply with accumulate / replace: row bitmap of a mask list, and
// the merge of the masked product t with the accumulation input w.  The
// list is first set into a byte map (plain byte stores), which is then
// packed into the bitmap and cleared, so `bytes` (at least 32 * ceil(m / 32)
// bytes) is all zero before and after.
hipError_t launch_mask_bits(const int32_t* idx, const uint8_t* val, int64_t count, int32_t m, uint8_t* bytes,
                            uint32_t* bits, uint32_t* err, hipStream_t s);
struct CombineArgs {
    const int32_t* t_idx;    // masked product, ascending
    const void* t_val;
    const int64_t* d_nt;     // its length (device)
    const int32_t* w_idx;    // accumulation input, ascending
    const void* w_val;
    int64_t nw;
    const uint32_t* mbits;   // nullable: mask row bitmap
    int complement, replace, accum;
    int32_t* y_idx;
    void* y_val;
    int64_t y_cap;
    int64_t* d_nnz_y;        // nullable
    Ctrl* ctrl;
    uint64_t* lb;            // look-back words, zero on entry
    int32_t lb_n;
};
constexpr int kCombineTile = 2048;   // merged entries per workgroup tile
hipError_t launch_combine(const CombineArgs& a, int semiring, int grid, hipStream_t s);
// Deterministic plus-times multiply (det_kernels.hip): the product list in
// product order, stably sorted by row, folded per row in that order.
constexpr int kDetBlock = 256;
constexpr int kDetItems = 16;
constexpr int kDetTile = kDetBlock * kDetItems;   // list entries per radix block
constexpr int kDetMaxDigitBits = 11;
constexpr int kDetShortRun = 128;   // a run longer than this continues in the wave-wide fold
constexpr int kDetLongPerBlock = kDetTile / kDetShortRun;   // long runs starting in one radix block, at most
// Groups of radix tiles in the count matrix's column scan, at most (the
// kernels size the groups from the call's tile count).
constexpr int kDetMaxGroups = 32;
// int32 entries of the group totals (gt[group][digit])
constexpr int64_t kDetGroupEntries = int64_t(kDetMaxGroups) << kDetMaxDigitBits;
struct DetArgs {
    Ctrl* ctrl;
    int32_t m;               // rows of the operand; m itself marks a masked-out product
    const int32_t* rowids;
    const float* values;     // nullable (pattern)
    const int32_t* cstart;   // the scan's column tables
    const int32_t* coff;
    const uint32_t* cxv;
    const int32_t* chunk_col;
    int chunk_log2;
    const uint32_t* mask;    // nullable: row bitmap, a product is kept when its bit == mask_keep
    int mask_keep;
    uint64_t* lb1;           // the scan's look-back words: the first lb1_clear of each half are
    int32_t lb1_n;           // cleared for the next call (the bucket scatter's task otherwise)
    int32_t lb1_clear;
    // Per radix tile of kDetTile list entries; the call's tile count,
    // ceil(W / kDetTile) (at least one), is taken from W on the device.
    int32_t* counts;         // radix passes: [tiles][2^digit_bits] per-(tile, digit) counts, tile rows
                             // contiguous; the fold: [tiles + 1] heads per tile, scanned in place
    int4* long_runs;         // [tiles * kDetLongPerBlock] runs longer than kDetShortRun, in the order the
                             // fold appends them: (row, acc bits, next entry, y position)
    int32_t* long_count;     // [1] long runs in the list (cleared by the gather)
    int32_t* y_idx;
    float* y_val;
    int64_t y_cap;
    int64_t* d_nnz_y;
};
// The launches take any grid (>= 1): each workgroup loops over chunks or
// tiles, whose count comes from W on the device.
// Products -> (row, RN32(a * x)) at their product index, by chunks of
// 2^chunk_log2 products.
hipError_t launch_det_gather(const DetArgs& a, uint2* list, int grid, hipStream_t s);
// One stable pass on bits [shift, shift + digit_bits) of the row; `partials`
// holds kDetGroupEntries int32 (the count matrix's group totals).
hipError_t launch_det_pass(const DetArgs& a, const uint2* in, uint2* out, int shift, int digit_bits,
                           int32_t* partials, int grid, hipStream_t s);
// Fold each row's run of the sorted list and write y ascending.
hipError_t launch_det_fold(const DetArgs& a, const uint2* list, int grid, hipStream_t s);
hipError_t launch_merge_batch(const MergeArgs& a, int semiring, int block, bool bfs, hipStream_t s);
// Multi-source BFS in the pull direction (msbfs_kernels.hip): frontier and
// seen masks with one bit per source, G = ceil(nsrc / 64) 64-bit words per
// vertex (vertex-major).
constexpr int kMsLong = 64;   // rows longer than this are scanned by a whole wave
struct MsArgs {
    int32_t n;
    int G;
    int nsrc;
    const int32_t* rowptr;   // row form: in-neighbours of each vertex, ascending
    const uint32_t* colids;
    const uint64_t* fcur;    // [n * G] frontier masks of the current level
    uint64_t* fnext;         // [n * G] next level's (every word written)
    uint64_t* seen;          // [n * G]
    int32_t* level;          // [nsrc][n]
    int32_t* parent;         // [nsrc][n], nullable
    int32_t lvl;             // level of the vertices found now
    const int32_t* long_rows;
    const int32_t* long_count;
    unsigned long long* found_total;   // += bits set in fnext
};
hipError_t launch_ms_long_rows(const int32_t* rowptr, int32_t n, int32_t* rows, int32_t* count, hipStream_t s);
hipError_t launch_ms_to_pull(const MsArgs& a, const uint32_t* visited, int32_t mask_words, const int32_t* front,
                             const int64_t* xoff, uint64_t* fm, hipStream_t s);
hipError_t launch_ms_pull(const MsArgs& a, bool parent, int num_cu, hipStream_t s);
hipError_t launch_ms_degsum(const int32_t* front, const int64_t* xoff, int nsrc, const int32_t* colptr, int32_t n,
                            unsigned long long* out, hipStream_t s);
hipError_t launch_msbfs_init(int32_t n, int nsrc, const int32_t* roots, int32_t* level, int32_t* parent,
                             uint32_t* visited, int32_t mask_words, int32_t* frontier, int64_t* xoff, Ctrl* ctrl,
                             hipStream_t s);
bool scatter_shape_supported(int block, int items);

// Optional timing of one launch: the events take the kernel's own start and
// end timestamps (no marker packets around it).
struct LaunchEvents {
    hipEvent_t start, stop;
};
hipError_t launch_scan(const ScanArgs& a, int grid, hipStream_t s, const LaunchEvents* ev = nullptr);
hipError_t launch_scatter(const ScatterArgs& a, int semiring, int block, int items, int grid, hipStream_t s,
                          const LaunchEvents* ev = nullptr);
hipError_t launch_merge(const MergeArgs& a, int semiring, int block, bool bfs, hipStream_t s,
                        const LaunchEvents* ev = nullptr);

constexpr int kScanBlock = 256;
constexpr int kScanItems = 2;         // host-known f: one tile per workgroup
constexpr int kScanItemsWide = 8;     // device-known f or batched: looping grid
constexpr int kScanTile = kScanBlock * kScanItems;   // smallest tile (sizes look-back arrays)
constexpr int kMergeItems = 8;
constexpr int kMergeList = 8192;   // rows staged per round of the in-order bitmap walk (largest tiles)
constexpr int kTileLog2Cap = 15;   // widest merge tile (2^15 rows of 4-byte cells) the LDS holds
constexpr int kTileLog2Wide = 14;  // widest plus-times tile (2^14 rows of 8-byte fp64 cells)
// Rows the merge's LDS list holds: the whole tile while its cells take at
// most 64 KB, else kMergeList per round of the walk.
__host__ __device__ inline int merge_list_cap(int tile_log2, bool wide) {
    return tile_log2 + (wide ? 3 : 2) <= 16 ? (1 << tile_log2) : kMergeList;
}
// Tile of a call: plus-times merges in fp64 cells, so at most 2^14 rows.
__host__ __device__ inline int tile_for(int tile_log2, int semiring) {
    return semiring == SR_PLUS_TIMES && tile_log2 > kTileLog2Wide ? kTileLog2Wide : tile_log2;
}

// One-launch multiply (k_fused): scan, bucketing and merge of one y <- A x
// in a single cooperative launch of one workgroup per compute unit.
constexpr int kFBlock = 1024;                  // threads per workgroup
constexpr int kFItems = 8;                     // products per thread per chunk
constexpr int kFChunk = kFBlock * kFItems;     // largest chunk of products a workgroup bucket-sorts at once
constexpr int kFSamples = 64;                  // local offsets each source list publishes
constexpr int kFMaxF = 4096;                   // x entries per source workgroup (f <= grid * kFMaxF)
constexpr int kFMaxNb = 1024;                  // buckets
constexpr int kFMaxGrid = 1024;                // workgroups
constexpr int kFRunGroup = 1024;               // chunk runs a merge workgroup indexes at once
// Tagged exchange words (64-bit, call tag in bits 63:44), one array each:
constexpr int kXA = 0;                          // per source: column and product counts (its lists are written)
constexpr int kXM = kFMaxGrid;                  // per source: longest column
constexpr int kXD = 2 * kFMaxGrid;              // per workgroup: its chunk runs are written
constexpr int kXG = 3 * kFMaxGrid;              // per workgroup: every run is written (set by workgroup 0)
constexpr int kXU = 4 * kFMaxGrid;              // per bucket: unique rows
constexpr int kXY = 4 * kFMaxGrid + kFMaxNb;    // per bucket: offset in y (set by workgroup 0)
constexpr int kXWords = 4 * kFMaxGrid + 2 * kFMaxNb;
struct FusedArgs {
    const int32_t* colptr;
    const int32_t* rowids;
    const float* values;     // nullable (pattern)
    int32_t m, n;
    int64_t nnz;
    const int32_t* x_idx;
    const void* x_val;
    int xmode;
    int32_t f;
    int tile_log2;
    int32_t nb;
    const uint32_t* mask;    // nullable: drop rows whose bit is set
    Ctrl* ctrl;
    int32_t* lstart;         // [grid * F] per-source lists of non-empty columns: first entry,
    int32_t* loff;           //   local exclusive product offset,
    uint32_t* lxv;           //   x value bits
    int32_t* samples;        // [grid][kFSamples] local offsets at evenly spaced list positions
    uint64_t* xw;            // [kXWords] tagged exchange words
    uint64_t* xrec;          // [2 * rows_cap] tagged chunk records: W, and the chunk's first and last source
    int64_t* gpoff;          // [kFMaxGrid + 1] product prefix of each source, its column count in bits 60:48
    int32_t* roff;           // [rows_cap][nb + 1] per-chunk bucket offsets
    int64_t rows_cap;
    uint2* buckets;          // [nnz + 1] (row, value bits), chunk k at k * chunk
    int32_t* y_idx;
    void* y_val;             // nullable
    int64_t y_cap;
    int64_t* d_nnz_y;        // nullable
};
size_t fused_lds_bytes(int tile_log2, int semiring, int nb);
int fused_grid(int num_cu, size_t lds_bytes);
hipError_t launch_fused(const FusedArgs& a, int semiring, int grid, hipStream_t s, const LaunchEvents* ev = nullptr);

// Persistent BFS levels for small frontiers on low-degree graphs.
constexpr int kTinyFrontier = 65536;   // vertices per frontier handled by the persistent kernel
constexpr int kPersistMaxDeg = 64;     // largest column length it accepts (lanes walk lists together)
struct PersistArgs {
    Ctrl* ctrl;
    const int32_t* colptr;
    const int32_t* rowids;
    int32_t n;               // vertices (square A): the length of every list and bitmap below
    int32_t* front[3];       // [n] each: frontier lists of three consecutive levels; front[0] on entry and exit
    uint32_t* visited;
    uint32_t* disc[3];       // [n/32] each: discovered-at-that-level bitmaps (min-select2nd), zero between launches
    int32_t* pmin;           // [n] smallest frontier in-neighbour (min-select2nd), INT32_MAX between launches
    uint32_t* bar;           // [160]: arrivals, three append counters, generation, 32 words apart; zero at launch
};
int persistent_grid(int num_cu);
hipError_t launch_bfs_persistent(const PersistArgs& a, bool min_semiring, int grid, hipStream_t s);

// Set-up kernels (spmspv_create, bfs_run).
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s);
// Evenly spaced samples of a device array (first and last included), K >= 2.
hipError_t launch_sample_i32(const int32_t* a, int64_t count, int32_t* out, int32_t K, hipStream_t s);
hipError_t launch_row_counts(const int32_t* rowids, int64_t nnz, int32_t m, int32_t* counts, Ctrl* ctrl,
                             hipStream_t s);
hipError_t launch_exclusive_scan_i32(int32_t* data, int64_t count, int32_t* partials, hipStream_t s);
hipError_t launch_validate_colptr(const int32_t* colptr, int32_t n, int64_t nnz, Ctrl* ctrl, int32_t* maxout,
                                 hipStream_t s);

// Format variants (format_kernels.hip).
// DCSC column index: aux[c] = first k with jc[k] >= c << shift, c in [0, nchunk].
hipError_t launch_dcsc_aux(const int32_t* jc, int32_t nzc, int32_t shift, int32_t nchunk, int32_t* aux,
                           hipStream_t s);
// ERR_CSC unless jc is strictly ascending inside [0, n).
hipError_t launch_validate_jc(const int32_t* jc, int32_t nzc, int32_t n, Ctrl* ctrl, hipStream_t s);
// Bitmap of n bits -> ascending index list out[], its length to *count
// (ERR_X_RANGE if a bit at or past n is set; such bits are ignored).
// tile_counts: bits_tiles(n) ints of scratch.
int64_t bits_tiles(int64_t n);
hipError_t launch_bits_to_list(const uint32_t* bits, int32_t n, int32_t* out, int32_t* count, int32_t* tile_counts,
                               Ctrl* ctrl, hipStream_t s);
hipError_t launch_decide(Ctrl* ctrl, int32_t n, int64_t nnz, hipStream_t s);
hipError_t launch_pr_init(int32_t n, const int32_t* colptr, float d, float* rank, int32_t* x_idx, float* x_val,
                          Ctrl* ctrl, hipStream_t s);
hipError_t launch_pr_update(int32_t n, const int32_t* colptr, float d, float tol, float* rank, const int32_t* y_idx,
                            const float* y_val, int32_t* x_idx, float* x_val, Ctrl* ctrl, hipStream_t s);
hipError_t launch_gen_x(int32_t n, double density, uint64_t seed, int32_t* x_idx, float* x_val, Ctrl* ctrl,
                        hipStream_t s);
hipError_t launch_cc_init(int32_t n, const int32_t* colptr, int32_t* label, int32_t* x_idx, int32_t* x_val,
                          Ctrl* ctrl, hipStream_t s);
hipError_t launch_cc_update(int32_t n, const int32_t* colptr, int32_t* label, const int32_t* y_idx,
                            const int32_t* y_val, int32_t* x_idx, int32_t* x_val, Ctrl* ctrl, hipStream_t s);

// Schedule-selector MLP (6 -> 64 -> 64 -> 10).
constexpr int kMlpIn = 6, kMlpH1 = 64, kMlpH2 = 64, kMlpOut = 10;
constexpr int kMlpParams = kMlpH1 * kMlpIn + kMlpH1 + kMlpH2 * kMlpH1 + kMlpH2 + kMlpOut * kMlpH2 + kMlpOut;
constexpr int kMlpBatchMax = 128;
hipError_t launch_mlp_forward(const float* p, const float* X, int B, float* logits, hipStream_t s);
hipError_t launch_mlp_train_step(float* p, float* am, float* av, int step, float lr, const float* X,
                                 const int32_t* labels, int B, float* grad_out, float* loss_out, hipStream_t s);
// set_dir: also write the level's direction (1 = pull when the class is pull
// and the handle has a row form) for gated BFS kernels.
hipError_t launch_select(Ctrl* ctrl, const float* sel, int32_t n, int64_t nnz, int has_pull, int set_dir,
                         int forced, hipStream_t s);
hipError_t launch_bfs_init(int32_t n, int32_t root, int32_t* level, int32_t* parent, uint32_t* visited,
                           uint32_t* xbits, int32_t* frontier, Ctrl* ctrl, int64_t nnz, int policy, hipStream_t s);

}  // namespace spv
