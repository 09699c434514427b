// C ABI of the SpMSpV library (include/spmspv.h): handle, workspace layout,
// schedule, validation and the per-call launch sequence.

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <atomic>
#include <mutex>
#include <algorithm>
#include <cmath>
#include <vector>
#include <fstream>
#include <sstream>

#include "spmspv.h"
#include "internal.h"

using namespace spv;

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t e, const char* where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return SPMSPV_EHIP;
}

#define HIP_TRY(expr)                                      \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);  \
    } while (0)

constexpr int kTileLog2Min = 8;
constexpr int kTileLog2Max = 15;
constexpr int kTileLog2MaxHbm = 30;   // merge variant 1: any bucket width
constexpr int kChunkMin = 256;
constexpr size_t kAlign = 256;
constexpr int kProfileSlots = 1024;
constexpr int kGraphLevels = 8;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline int ceil_log2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

// Offsets of every region inside the caller's workspace.
struct Layout {
    size_t ctrl, rcp, partials, cstart, coff, cxv, chunk_col, lb1, cursor, lb3, xw, xrec, buckets, visited, front0,
        front1, front2, disc, pmin, bar, samples, gpoff, roff, gb_lb, gb_bytes, bv_idx, bv_val, bv_tiles, dc_aux, det_list,
        det_counts, det_partials, det_long, det_long_count, h_f64, h_i32, h_orbits, h_touched, total;
    // pull direction (present with SPMSPV_WITH_TRANSPOSE or SPMSPV_SYMMETRIC)
    size_t p_xbits, p_xdense, p_ybits, p_ydense, p_lbp, p_part, p_chain, t_colids, t_values, selector;
    bool pull, transpose, det;
    int64_t nb_max, lb1_n, chunk_n;
    int32_t det_nblk_max;   // deterministic mode: radix blocks of the longest product list
    int64_t h_rows;         // merge variant 1: rows of the HBM accumulator
    int64_t rows_cap;   // one-launch multiply: chunk rows of run offsets
    int32_t fnb;        // one-launch multiply: buckets per row of run offsets
};

inline int64_t gb_lb_words(int64_t m) { return (2 * m + kCombineTile - 1) / kCombineTile + 2; }

Layout make_layout(int64_t m, int64_t n, int64_t nnz, int flags = 0, int64_t dc_chunks = 0) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + (bytes ? bytes : 1));
        return at;
    };
    // Left multiplication runs A^T (m and n swapped) through the same
    // regions, so with the transpose present the regions sized by the
    // output length (mr) or by the x length (nc) take max(m, n).
    const int64_t mx = std::max(m, n);
    const bool tr = (flags & (SPMSPV_WITH_TRANSPOSE | SPMSPV_SYMMETRIC)) != 0;
    const int64_t mr = tr ? mx : m, nc = tr ? mx : n;
    L.nb_max = (mr + (1 << kTileLog2Min) - 1) >> kTileLog2Min;
    // one-launch multiply: chunks of at most kFChunk products, at least one per workgroup
    L.rows_cap = std::max<int64_t>(kFMaxGrid, (nnz + kFChunk) / kFChunk) + 1;
    L.fnb = (int32_t)std::min<int64_t>(kFMaxNb, L.nb_max);
    L.lb1_n = (nc + kScanTile - 1) / kScanTile + 1;
    L.chunk_n = nnz / kChunkMin + 2;
    L.ctrl = take(sizeof(Ctrl));
    L.rcp = take(size_t(m + 1) * 4);
    L.partials = take(size_t((m + 1) / 4096 + 2) * 4);
    // column tables; the one-launch multiply keeps its per-workgroup column
    // lists here too (up to kFMaxGrid - 1 slots past n)
    L.cstart = take(size_t(nc + kFMaxGrid + 1) * 4);
    L.coff = take(size_t(nc + kFMaxGrid + 1) * 4);
    L.cxv = take(size_t(nc + kFMaxGrid + 1) * 4);
    L.chunk_col = take(size_t(L.chunk_n) * 4);
    L.lb1 = take(size_t(L.lb1_n) * 16);
    L.cursor = take(size_t(L.nb_max) * 4);
    L.lb3 = take(size_t(L.nb_max) * 8);
    // one-launch multiply: tagged exchange words and chunk records (zeroed
    // at create with everything before the buckets; tags are never zero)
    L.xw = take(size_t(kXWords) * 8);
    L.xrec = take(size_t(2 * L.rows_cap) * 8);
    L.buckets = take(size_t(nnz + 1) * 8);
    L.visited = take(size_t((mr + 31) / 32) * 4);
    L.front0 = take(size_t(m) * 4);
    L.front1 = take(size_t(m) * 4);
    L.front2 = take(size_t(m) * 4);
    L.disc = take(size_t((m + 31) / 32) * 4 * 3);
    L.pmin = take(size_t(m) * 4);
    L.bar = take(160 * 4);
    L.selector = take(size_t(kMlpParams + 2 * kMlpIn) * 4);
    // one-launch multiply: list samples, source prefix and per-chunk bucket offsets
    L.samples = take(size_t(kFMaxGrid) * kFSamples * 4);
    L.gpoff = take(size_t(kFMaxGrid + 1) * 8);
    L.roff = take(size_t(L.rows_cap) * size_t(L.fnb + 1) * 4);
    // masked multiply: look-back words of the combine (t and w each hold at most m rows)
    L.gb_lb = take(size_t(gb_lb_words(mr)) * 8);
    // masked multiply: byte map of the mask list (zero between calls)
    L.gb_bytes = take(size_t((mr + 31) / 32) * 32);
    // bitvector calls (x list, then y list) and the masked multiply's
    // product t: lists of up to max(m, n) entries
    L.bv_idx = take(size_t(mx) * 4);
    L.bv_val = take(size_t(mx) * 4);
    L.bv_tiles = take(size_t(bits_tiles(mx)) * 4);
    // DCSC: column index over the stored column ids
    L.dc_aux = dc_chunks > 0 ? take(size_t(dc_chunks + 1) * 4) : 0;
    // merge variant 1: the HBM sparse accumulator over every row
    L.h_f64 = take(size_t(mr) * 8);
    L.h_i32 = take(size_t(mr) * 4);
    L.h_orbits = take(size_t((mr + 31) / 32) * 4);
    L.h_touched = take(size_t((mr + 31) / 32) * 4);
    L.h_rows = mr;
    // deterministic plus-times: a second product list (the buckets are the
    // first) and the radix passes' count matrix with its scan partials
    L.det = (flags & SPMSPV_DETERMINISTIC) != 0;
    if (L.det) {
        L.det_nblk_max = (int32_t)(nnz / kDetTile + 2);
        const int64_t ncounts = (int64_t(1) << kDetMaxDigitBits) * L.det_nblk_max + 1;
        L.det_list = take(size_t(nnz + 1) * 8);
        L.det_counts = take(size_t(ncounts) * 4);
        L.det_partials = take(size_t(kDetGroupEntries) * 4);
        L.det_long = take(size_t(L.det_nblk_max) * kDetLongPerBlock * 16);
        L.det_long_count = take(4);
    }
    L.pull = (flags & (SPMSPV_WITH_TRANSPOSE | SPMSPV_SYMMETRIC)) != 0;
    L.transpose = (flags & SPMSPV_WITH_TRANSPOSE) != 0;
    if (L.pull) {
        L.p_xbits = take(size_t((n + 31) / 32) * 4);
        L.p_xdense = take(size_t(n) * 4);
        L.p_ybits = take(size_t((m + 31) / 32) * 4);
        L.p_ydense = take(size_t(m) * 4);
        L.p_lbp = take(size_t(pull_emit_blocks((int32_t)m) + 1) * 8);
        L.p_part = take(size_t(pull_blocks((int32_t)m, nnz) + 2) * 4);
        L.p_chain = take(size_t(pull_emit_blocks((int32_t)m)) * 16);
    }
    if (L.transpose) {
        L.t_colids = take(size_t(nnz + 1) * 4);
        L.t_values = take(size_t(nnz + 1) * 4);
    }
    L.total = o;
    return L;
}

// Batched calls: caller-provided second workspace.
constexpr int kMaxKeys = 8192;   // (vector, bucket) keys per batched call

struct BatchLayout {
    size_t cstart, coff, cxid, cxv, chunk_col, lb1, kcount, partials, cursor, lb3, buckets, visited, front0, front1,
        xoff0, xoff1, roots, ms_f0, ms_f1, ms_seen, ms_long, ms_cnt, total;
    int64_t max_f, max_products, chunk_n, lb1_n;
    int32_t mask_words;
    int32_t ms_groups;   // multi-source pull: 64-bit mask words per vertex
};

BatchLayout make_batch_layout(int64_t m, int64_t n, int64_t nnz, int max_batch, int64_t max_f,
                              int64_t max_products, bool bfs) {
    BatchLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + (bytes ? bytes : 1));
        return at;
    };
    if (bfs) {
        // every source's frontier holds at most n vertices and one level at
        // most nnz products per source
        max_f = (int64_t)max_batch * n;
        if (max_products <= 0) max_products = (int64_t)max_batch * nnz;
    }
    if (max_products > INT32_MAX - 1) max_products = INT32_MAX - 1;
    L.max_f = max_f;
    L.max_products = max_products;
    L.chunk_n = max_products / kChunkMin + 2;
    L.lb1_n = (max_f + kScanTile - 1) / kScanTile + 1;
    L.mask_words = (int32_t)((m + 31) / 32);
    L.cstart = take(size_t(max_f + 1) * 4);
    L.coff = take(size_t(max_f + 1) * 4);
    L.cxid = take(size_t(max_f + 1) * 4);
    L.cxv = take(size_t(max_f + 1) * 4);
    L.chunk_col = take(size_t(L.chunk_n) * 4);
    L.lb1 = take(size_t(L.lb1_n) * 16);
    L.kcount = take(size_t(kMaxKeys + 1) * 4);
    L.partials = take(size_t(kMaxKeys / 4096 + 2) * 4);
    L.cursor = take(size_t(kMaxKeys) * 4);
    L.lb3 = take(size_t(kMaxKeys) * 8);
    L.buckets = take(size_t(max_products + 1) * 8);
    if (bfs) {
        L.visited = take(size_t(max_batch) * L.mask_words * 4);
        L.front0 = take(size_t(max_f) * 4);
        L.front1 = take(size_t(max_f) * 4);
        L.xoff0 = take(size_t(max_batch + 1) * 8);
        L.xoff1 = take(size_t(max_batch + 1) * 8);
        L.roots = take(size_t(max_batch) * 4);
        // pull levels (SPMSPV_DIRECTION_OPT): frontier masks (two levels) and
        // seen masks, one bit per source; the list of long rows; counters
        L.ms_groups = (max_batch + 63) / 64;
        L.ms_f0 = take(size_t(n) * L.ms_groups * 8);
        L.ms_f1 = take(size_t(n) * L.ms_groups * 8);
        L.ms_seen = take(size_t(n) * L.ms_groups * 8);
        L.ms_long = take(size_t(nnz / kMsLong + 2) * 4);
        L.ms_cnt = take(64);
    }
    L.total = o;
    return L;
}

struct BatchCtx {
    bool bound = false;
    bool bfs = false;
    bool fixed_last = false;   // the last batched call used fixed slices (no counting pass)
    bool ms_long_ready = false;   // the long-row list of the pull levels is built
    int max_batch = 0;
    BatchLayout L{};
    char* ws = nullptr;
};

}  // namespace

struct spmspv_matrix {
    int64_t m = 0, n = 0, nnz = 0;
    const int32_t* colptr = nullptr;
    const int32_t* rowids = nullptr;
    const float* values = nullptr;
    Layout L{};
    char* ws = nullptr;
    Ctrl* ctrl = nullptr;
    int32_t* rcp = nullptr;
    int32_t* cstart = nullptr;
    int32_t* coff = nullptr;
    uint32_t* cxv = nullptr;
    int32_t* chunk_col = nullptr;
    uint64_t* lb1 = nullptr;
    int32_t* cursor = nullptr;
    uint64_t* lb3 = nullptr;
    uint2* buckets = nullptr;
    uint32_t* visited = nullptr;
    uint32_t* disc = nullptr;           // persistent BFS: three discovered-at-level bitmaps of m/32 words
    int32_t* pmin = nullptr;            // persistent BFS: smallest frontier in-neighbour
    uint32_t* bar = nullptr;            // persistent BFS: grid barrier words
    int persist_grid = -1;              // co-resident workgroups of the persistent kernel (0 = unavailable)
    int fused_grid = -1;                // workgroups of the one-launch multiply (0 = unavailable)
    int32_t* front[2] = {nullptr, nullptr};
    int32_t* front2 = nullptr;          // persistent BFS: third frontier list
    int32_t maxdeg = 0;
    int device = 0;
    int num_cu = 256;
    size_t lds_max = 65536;
    spmspv_schedule sched{};
    // profiling ring
    std::vector<hipEvent_t> prof_ev;
    int prof_used = 0;
    bool sched_default = true;          // no schedule set by the caller: size the scatter chunk per call
    // BFS graph cache
    hipGraphExec_t graph = nullptr;
    int graph_key = -1;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    // pull direction
    bool pull = false;
    bool rows_sorted = false;           // CSR rows have ascending column ids
    const int32_t* rowptr = nullptr;
    const uint32_t* colids = nullptr;
    const float* rvalues = nullptr;
    uint32_t* p_xbits = nullptr;
    uint32_t* p_xdense = nullptr;
    uint32_t* p_ybits = nullptr;
    uint32_t* p_ydense = nullptr;
    int64_t* p_chain = nullptr;         // direction-switching BFS: the pull emit's per-workgroup column sums
    uint64_t* p_lbp = nullptr;
    int32_t* p_part = nullptr;
    uint32_t ydense_ident = 0;
    // schedule selector: MLP parameters, then feature mean[6] and std[6]
    float* selector = nullptr;
    bool selector_loaded = false;
    std::vector<int> level_classes;     // classes the selector chose in the last BFS
    BatchCtx batch;                     // second workspace for batched calls
    spmspv_schedule batch_sched{};      // batched-call schedule (tile_log2 0 = derive)
    std::vector<spmspv_tune_entry> tuned;   // autotuned schedule per density band
    std::vector<int32_t> forced_classes;    // per-step classes replacing the selector (replay)
    // Left multiplication reads the CSR copy as the CSC of A^T: its row
    // counts are A's column counts (bucket bases colptr) and its longest
    // column is A's longest row.
    int32_t maxrow = 0;
    // DCSC input: colptr holds the nzc + 1 starts of the stored columns
    bool dcsc = false;
    int64_t nzc = 0;
    const int32_t* dc_jc = nullptr;     // ids of the stored columns, ascending
    int32_t* dc_aux = nullptr;          // column index: first stored column of each id chunk
    int32_t dc_shift = 0;               // id chunk = j >> dc_shift
    // list scratch of max(m, n) entries (bitvector calls, masked product t)
    int32_t* bv_idx = nullptr;
    uint32_t* bv_val = nullptr;
    int32_t* bv_tiles = nullptr;
};

namespace {

int default_schedule(const spmspv_matrix* A, spmspv_schedule* s) {
    // Buckets as wide as LDS allows, but at least ~256 of them when the
    // matrix is tall enough (one merge workgroup per bucket).
    int tl = ceil_log2(A->m) - 8;
    if (tl < kTileLog2Min) tl = kTileLog2Min;
    if (tl > kTileLog2Max) tl = kTileLog2Max;
    while (tl > kTileLog2Min && merge_lds_bytes(tl, SR_MIN_SELECT2ND) + 1024 > A->lds_max) --tl;
    s->direction = 0;
    s->tile_log2 = tl;
    s->scatter_block = 1024;
    s->scatter_items = 8;
    s->merge_block = 1024;
    s->merge_variant = 0;
    s->launch = 0;
    const int64_t nb = (A->m + (int64_t(1) << tl) - 1) >> tl;
    if (scatter_lds_bytes((int)nb, 8192) + 1024 > A->lds_max) s->scatter_items = 4;
    return SPMSPV_OK;
}

// Default schedule for one standalone call with f x entries: the scatter
// takes chunks of exactly block x items products, one workgroup per chunk
// at a time, so with few products a large chunk leaves compute units idle.
// Take the largest chunk (at most 4096 products: two workgroups per compute
// unit overlap their phases; measured faster than 8192 at every density on
// R-MAT scale 22) for which the expected product count f * nnz / n still
// gives every compute unit one.
spmspv_schedule sized_for_call(const spmspv_matrix* A, int64_t f) {
    spmspv_schedule s = A->sched;
    const double w_est = A->n > 0 ? (double)f * (double)A->nnz / (double)A->n : 0.0;
    const int64_t nb = (A->m + (int64_t(1) << s.tile_log2) - 1) >> s.tile_log2;
    const int shapes[3][2] = {{512, 8}, {256, 8}, {256, 4}};
    for (const auto& sh : shapes) {
        const int chunk = sh[0] * sh[1];
        if (scatter_lds_bytes((int)nb, chunk) + 1024 > A->lds_max) continue;
        s.scatter_block = sh[0];
        s.scatter_items = sh[1];
        if (w_est >= (double)chunk * A->num_cu) break;
    }
    return s;
}

int check_schedule(const spmspv_matrix* A, const spmspv_schedule* s) {
    if (s->direction != 0 && s->direction != 1) return fail(SPMSPV_EINVAL, "direction must be 0 (push) or 1 (pull)");
    if (s->direction == 1 && !A->pull)
        return fail(SPMSPV_EUNSUPPORTED, "pull needs a handle created with SPMSPV_WITH_TRANSPOSE or SPMSPV_SYMMETRIC");
    if (s->merge_variant != 0 && s->merge_variant != 1)
        return fail(SPMSPV_EINVAL, "merge_variant must be 0 (LDS) or 1 (HBM)");
    const int tmax = s->merge_variant == 1 ? kTileLog2MaxHbm : kTileLog2Max;
    if (s->tile_log2 < kTileLog2Min || s->tile_log2 > tmax)
        return fail(SPMSPV_EINVAL, s->merge_variant == 1 ? "tile_log2 out of [8, 30]" : "tile_log2 out of [8, 15]");
    const int64_t nb = (A->m + (int64_t(1) << s->tile_log2) - 1) >> s->tile_log2;
    const int sb = s->scatter_block, si = s->scatter_items;
    if (!scatter_shape_supported(sb, si)) return fail(SPMSPV_EINVAL, "unsupported scatter_block / scatter_items pair");
    if (s->merge_block != 256 && s->merge_block != 512 && s->merge_block != 1024)
        return fail(SPMSPV_EINVAL, "merge_block must be 256, 512 or 1024");
    if (s->launch < 0 || s->launch > 2) return fail(SPMSPV_EINVAL, "launch must be 0 (auto), 1 (three) or 2 (one)");
    if (s->merge_variant == 0 && merge_lds_bytes(s->tile_log2, SR_MIN_SELECT2ND) + 1024 > A->lds_max)
        return fail(SPMSPV_EINVAL, "tile exceeds LDS");
    if (scatter_lds_bytes((int)nb, sb * si) + 1024 > A->lds_max)
        return fail(SPMSPV_EINVAL, "too many buckets for the scatter LDS histogram");
    return SPMSPV_OK;
}

// Tile one call merges with: the schedule's tile, narrowed for plus-times
// (fp64 cells take twice the LDS of the other semirings' cells).
int call_tile(const spmspv_matrix* A, int tl, int semiring) {
    tl = tile_for(tl, semiring);
    while (tl > kTileLog2Min && merge_lds_bytes(tl, semiring) + 1024 > A->lds_max) --tl;
    return tl;
}

// Bucketing workgroups one compute unit holds at once (registers, LDS and
// threads, as the runtime computes it for the kernel): the scatter grid is at
// most this many per CU, so every workgroup of the grid is resident and short
// chunks overlap their memory round trips across workgroups.  (A grid sized
// by LDS alone once put a third of the workgroups, each with its share of the
// chunks, in a second round: 96 -> 114 us at 10 % density on scale 22.)
int64_t scatter_occupancy(const spmspv_matrix* A, int semiring, int nb, int block, int items, bool batch) {
    const size_t lds = scatter_lds_bytes(nb, block * items, batch) + 1024;
    int64_t by_lds = (int64_t)(A->lds_max / (lds ? lds : 1));
    int64_t occ = scatter_resident(semiring, block, items, nb, batch);
    if (by_lds < occ) occ = by_lds;
    return occ < 1 ? 1 : occ;
}

// Enqueue the three phases of one y <- A x.
// phases: 1 = scan only, 2 = scatter + merge only, 3 = all.  tile_log2 < 0
// uses the handle's schedule.  clear_nb > 0 makes the scan clear that many
// bucket counters (so a later scatter may use a narrower tile).
int enqueue(spmspv_matrix* A, int semiring, int xmode, int64_t f_host, const int32_t* f_dev, const int32_t* x_idx,
            const void* x_val, int32_t* y_idx, void* y_val, int64_t y_cap, int64_t* d_nnz_y, bool bfs,
            const uint32_t* mask, hipStream_t s, hipEvent_t* ev, bool diropt = false, int tile_log2 = -1,
            int phases = 3, int clear_nb = 0, bool learned_gate = false, int mask_keep = 0, bool left = false,
            int variant = -1, uint32_t* y_bits = nullptr) {
    // The operand: A, or for left multiplication A^T through the CSR copy
    // (y' = x'A is y = A^T x; Background, Notation).  The CSR copy's row
    // pointer is A^T's column pointer and A's column pointer is A^T's
    // row-count prefix, which sizes the buckets.
    const int64_t Om = left ? A->n : A->m, On = left ? A->m : A->n;
    const int32_t* Ocolptr = left ? A->rowptr : A->colptr;
    const int32_t* Orowids = left ? reinterpret_cast<const int32_t*>(A->colids) : A->rowids;
    const float* Ovalues = left ? A->rvalues : A->values;
    const int32_t* Orcp = left ? A->colptr : A->rcp;
    const int64_t Omaxdeg = left ? A->maxrow : A->maxdeg;
    spmspv_schedule sc = A->sched;
    if (tile_log2 >= 0) sc.tile_log2 = tile_log2;
    if (variant >= 0) sc.merge_variant = variant;
    // merge variant 1 (HBM accumulator) takes any tile; the LDS merge's is
    // narrowed to what its accumulator holds for this semiring
    const bool hbm = sc.merge_variant == 1;
    if (!hbm) sc.tile_log2 = call_tile(A, sc.tile_log2, semiring);
    const int chunk = sc.scatter_block * sc.scatter_items;
    auto buckets_of = [&](int tl) { return (int)((Om + (int64_t(1) << tl) - 1) >> tl); };
    // A^T of a wide A can have more rows than the schedule's tile covers in
    // one scatter histogram: widen the tile as far as the merge allows.
    while (left && scatter_lds_bytes(buckets_of(sc.tile_log2), chunk) + 1024 > A->lds_max &&
           sc.tile_log2 < (hbm ? kTileLog2MaxHbm : call_tile(A, kTileLog2Max, semiring)))
        ++sc.tile_log2;
    const int nb = buckets_of(sc.tile_log2);
    if (scatter_lds_bytes(nb, chunk) + 1024 > A->lds_max)
        return fail(SPMSPV_EUNSUPPORTED, "too many buckets of 2^" + std::to_string(sc.tile_log2) +
                                             " rows for the scatter LDS histogram");
    const int chunk_log2 = ceil_log2(chunk);
    const int64_t f_bound = f_dev ? On : f_host;

    ScanArgs sa{};
    sa.colptr = Ocolptr;
    sa.n = (int32_t)On;
    if (A->dcsc && !left) {
        sa.dcsc = 1;
        sa.dc_jc = A->dc_jc;
        sa.dc_aux = A->dc_aux;
        sa.dc_shift = A->dc_shift;
    }
    sa.x_idx = x_idx;
    sa.x_val = x_val;
    sa.xmode = xmode;
    sa.f_host = (int32_t)f_host;
    sa.f_dev = f_dev;
    sa.ctrl = A->ctrl;
    sa.cstart = A->cstart;
    sa.coff = A->coff;
    sa.cxv = A->cxv;
    sa.chunk_col = A->chunk_col;
    sa.chunk_log2 = chunk_log2;
    sa.lb1 = A->lb1;
    sa.lb1_n = (int32_t)A->L.lb1_n;
    sa.nnz = A->nnz;
    sa.chunk_n = A->L.chunk_n;
    sa.cursor = A->cursor;
    sa.lb3 = A->lb3;
    sa.nb = clear_nb > nb ? clear_nb : nb;
    if (hbm && sa.nb < hmerge_tiles(Om)) sa.nb = (int32_t)hmerge_tiles(Om);   // its walk's look-back words
    sa.bump_level = bfs ? 1 : 0;
    // A direction-switching BFS level: after a pull level the scan takes the
    // decision itself (see the pull emit's chain mode).
    if (bfs && diropt && A->pull && f_dev) {
        sa.chain = learned_gate ? 2 : 1;
        sa.sel = A->selector;
        sa.has_pull = 1;
        sa.xbits = A->p_xbits;
        sa.chain_part = A->p_chain;
        sa.chain_nparts = pull_emit_blocks((int32_t)A->m);
    }
    // f known on the host: one workgroup per tile, narrow tiles unless that
    // would take more than two workgroups per compute unit.  f on the device
    // (BFS): a fixed grid of wide tiles loops over the frontier.
    sa.wide = (f_dev || f_bound > (int64_t)kScanTile * 2 * A->num_cu) ? 1 : 0;
    const int64_t scan_tile = sa.wide ? (int64_t)kScanBlock * kScanItemsWide : kScanTile;
    int64_t g1 = (f_bound + scan_tile - 1) / scan_tile;
    if (g1 < 1) g1 = 1;
    if (f_dev && g1 > 2 * A->num_cu) g1 = 2 * A->num_cu;

    ScatterArgs ca{};
    ca.rowids = Orowids;
    ca.values = Ovalues;
    ca.ctrl = A->ctrl;
    ca.cstart = A->cstart;
    ca.coff = A->coff;
    ca.cxv = A->cxv;
    ca.chunk_col = A->chunk_col;
    ca.chunk_log2 = chunk_log2;
    ca.tile_log2 = sc.tile_log2;
    ca.nb = nb;
    ca.m = (int32_t)Om;
    ca.rcp = Orcp;
    ca.cursor = A->cursor;
    ca.buckets = A->buckets;
    ca.mask = mask;
    ca.mask_keep = mask_keep;
    ca.lb1 = A->lb1;
    ca.lb1_n = (int32_t)A->L.lb1_n;
    ca.lb1_clear = (int32_t)((f_bound + kScanTile - 1) / kScanTile + 1);
    if (ca.lb1_clear > ca.lb1_n) ca.lb1_clear = ca.lb1_n;
    ca.f_host = (int32_t)f_host;
    ca.f_dev = f_dev;
    ca.gate = diropt ? 1 : 0;
    int64_t wbound = f_dev ? A->nnz : f_host * Omaxdeg;
    if (wbound > A->nnz) wbound = A->nnz;
    int64_t g2 = (wbound + chunk - 1) / chunk;
    if (g2 < 1) g2 = 1;
    const int64_t g2max =
        int64_t(A->num_cu) * scatter_occupancy(A, semiring, nb, sc.scatter_block, sc.scatter_items, false);
    if (g2 > g2max) g2 = g2max;

    MergeArgs ma{};
    ma.ctrl = A->ctrl;
    ma.cursor = A->cursor;
    ma.buckets = A->buckets;
    ma.rcp = Orcp;
    ma.m = (int32_t)Om;
    ma.tile_log2 = sc.tile_log2;
    ma.nb = nb;
    ma.lb3 = A->lb3;
    ma.y_idx = y_idx;
    ma.y_val = y_val;
    ma.y_cap = y_cap;
    ma.d_nnz_y = d_nnz_y;
    ma.visited = A->visited;
    ma.set_f = bfs ? 1 : 0;
    ma.gate = diropt ? 1 : 0;
    ma.h_f64 = reinterpret_cast<double*>(A->ws + A->L.h_f64);
    ma.h_i32 = reinterpret_cast<int32_t*>(A->ws + A->L.h_i32);
    ma.h_orbits = reinterpret_cast<uint32_t*>(A->ws + A->L.h_orbits);
    ma.h_touched = reinterpret_cast<uint32_t*>(A->ws + A->L.h_touched);
    ma.h_split = std::max(1, std::min(1024, 4 * A->num_cu / nb));   // about four workgroups per CU
    ma.y_bits = bfs ? nullptr : y_bits;

    // With profiling, each kernel's own start and end timestamps go to a pair
    // of events (scan, scatter, merge).
    const LaunchEvents le[3] = {{ev ? ev[0] : nullptr, ev ? ev[1] : nullptr},
                                {ev ? ev[2] : nullptr, ev ? ev[3] : nullptr},
                                {ev ? ev[4] : nullptr, ev ? ev[5] : nullptr}};
    if (phases & 1) {
        HIP_TRY(launch_scan(sa, (int)g1, s, ev ? &le[0] : nullptr));
        if (diropt && learned_gate)   // the selector picks the direction on the device
            HIP_TRY(launch_select(A->ctrl, A->selector, (int32_t)A->n, A->nnz, A->pull ? 1 : 0, 1, -1, s));
        else if (diropt)
            HIP_TRY(launch_decide(A->ctrl, (int32_t)A->n, A->nnz, s));
    }
    if (phases & 2) {
        HIP_TRY(launch_scatter(ca, semiring, sc.scatter_block, sc.scatter_items, (int)g2, s, ev ? &le[1] : nullptr));
        if (hbm) {   // two kernels: profile them between plain event markers
            if (ev) HIP_TRY(hipEventRecord(ev[4], s));
            HIP_TRY(launch_hbm_merge(ma, semiring, bfs, s));
            if (ev) HIP_TRY(hipEventRecord(ev[5], s));
        } else {
            HIP_TRY(launch_merge(ma, semiring, sc.merge_block, bfs, s, ev ? &le[2] : nullptr));
        }
    }
    return SPMSPV_OK;
}

// Deterministic plus-times multiply: the scan, then the product list in
// product order, its stable sort by row and the sequential fold per row
// (det_kernels.hip).  y is ascending.
int enqueue_det(spmspv_matrix* A, int xmode, int64_t f, const int32_t* x_idx, const void* x_val, int32_t* y_idx,
                float* y_val, int64_t y_cap, int64_t* d_nnz_y, const uint32_t* mask, int mask_keep, bool left,
                hipStream_t s) {
    const Layout& L = A->L;
    if (!L.det)
        return fail(SPMSPV_EUNSUPPORTED, "SPMSPV_DETERMINISTIC needs a handle whose workspace was sized and "
                                         "created with SPMSPV_DETERMINISTIC");
    const int64_t Om = left ? A->n : A->m;
    // the scan only (phase 1), on the same operand
    int rc = enqueue(A, SR_PLUS_TIMES, xmode, f, nullptr, x_idx, x_val, nullptr, nullptr, 0, nullptr, false,
                     nullptr, s, nullptr, false, -1, 1, 0, false, 0, left);
    if (rc) return rc;
    const int chunk_log2 = ceil_log2(A->sched.scatter_block * A->sched.scatter_items);
    // The kernels size their work by the call's product count W on the
    // device (the scan caps W at nnz) and loop over chunks and radix tiles,
    // so the call needs no host read.  Grids: a workgroup per expected chunk
    // or tile (f * nnz / n products) and a quarter more, at least one per
    // compute unit, never more than the workspace holds; the estimate only
    // sets how many chunks or tiles each workgroup takes.
    const int64_t nx = left ? A->m : A->n;   // x's length
    const int64_t w_est = nx > 0 ? (int64_t)((double)f * (double)A->nnz / (double)nx) : 0;
    auto grid_for = [&](int64_t unit_log2) {
        const int64_t cap = std::max<int64_t>(1, (A->nnz + (int64_t(1) << unit_log2) - 1) >> unit_log2);
        const int64_t est = (w_est >> unit_log2) + 1;
        return (int)std::min<int64_t>(cap, std::max<int64_t>(A->num_cu, est + est / 4));
    };
    static_assert((kDetTile & (kDetTile - 1)) == 0, "radix tiles are a power of two");
    const int tile_grid = grid_for(ceil_log2(kDetTile));
    const int gather_grid = grid_for(chunk_log2);
    DetArgs d{};
    d.ctrl = A->ctrl;
    d.m = (int32_t)Om;
    d.rowids = left ? reinterpret_cast<const int32_t*>(A->colids) : A->rowids;
    d.values = left ? A->rvalues : A->values;
    d.cstart = A->cstart;
    d.coff = A->coff;
    d.cxv = A->cxv;
    d.chunk_col = A->chunk_col;
    d.chunk_log2 = chunk_log2;
    d.mask = mask;
    d.mask_keep = mask_keep;
    d.lb1 = A->lb1;
    d.lb1_n = (int32_t)L.lb1_n;
    d.lb1_clear = (int32_t)std::min<int64_t>(L.lb1_n, (f + kScanTile - 1) / kScanTile + 1);
    d.counts = reinterpret_cast<int32_t*>(A->ws + L.det_counts);
    d.long_runs = reinterpret_cast<int4*>(A->ws + L.det_long);
    d.long_count = reinterpret_cast<int32_t*>(A->ws + L.det_long_count);
    d.y_idx = y_idx;
    d.y_val = y_val;
    d.y_cap = y_cap;
    d.d_nnz_y = d_nnz_y;
    int32_t* partials = reinterpret_cast<int32_t*>(A->ws + L.det_partials);
    uint2* cur = A->buckets;
    uint2* other = reinterpret_cast<uint2*>(A->ws + L.det_list);
    HIP_TRY(launch_det_gather(d, cur, gather_grid, s));
    // stable LSD passes over the bits of the row (m itself included: it marks masked products)
    // bits of the largest key: m - 1, or m itself when a mask marks products with it
    const int64_t top = mask ? Om : Om - 1;
    int bits = 1;
    while ((top >> bits) > 0) ++bits;
    const int passes = (bits + kDetMaxDigitBits - 1) / kDetMaxDigitBits;
    const int dbits = (bits + passes - 1) / passes;
    for (int p = 0; p < passes; ++p) {
        HIP_TRY(launch_det_pass(d, cur, other, p * dbits, dbits, partials, tile_grid, s));
        std::swap(cur, other);
    }
    HIP_TRY(launch_det_fold(d, cur, tile_grid, s));
    return SPMSPV_OK;
}

// One-launch multiply.  Eligible when the device holds one workgroup of it
// per compute unit, every source workgroup's slice of x fits its list
// (f <= kFMaxF per workgroup) and the call's buckets fit one row of run
// offsets.  Returns the grid, or 0 when the call must take three launches.
int fused_eligible(spmspv_matrix* A, int semiring, int64_t f, int* tl_out, int* nb_out) {
    if (A->sched.merge_variant != 0) return 0;   // the one launch merges in LDS only
    const int tl = call_tile(A, A->sched.tile_log2, semiring);
    const int64_t nb = (A->m + (int64_t(1) << tl) - 1) >> tl;
    if (nb > A->L.fnb || nb > kFMaxNb) return 0;
    if (A->fused_grid < 0) {
        size_t lds = 0;
        for (int t = kTileLog2Min; t <= kTileLog2Max; ++t)
            for (int sr = 0; sr < 3; ++sr) {
                if (merge_lds_bytes(tile_for(t, sr), sr) + 1024 > A->lds_max) continue;
                lds = std::max(lds, fused_lds_bytes(tile_for(t, sr), sr, kFMaxNb));
            }
        A->fused_grid = lds + 1024 <= A->lds_max ? fused_grid(A->num_cu, lds) : 0;
        (void)hipGetLastError();   // an unavailable attribute leaves no sticky error behind
    }
    const int G = A->fused_grid;
    if (G < 1 || f > (int64_t)G * kFMaxF) return 0;
    if (fused_lds_bytes(tl, semiring, (int)nb) + 1024 > A->lds_max) return 0;
    *tl_out = tl;
    *nb_out = (int)nb;
    return G;
}

int enqueue_fused(spmspv_matrix* A, int semiring, int xmode, int64_t f, const int32_t* x_idx, const void* x_val,
                  int32_t* y_idx, void* y_val, int64_t y_cap, int64_t* d_nnz_y, const uint32_t* mask, int G, int tl,
                  int nb, hipStream_t s, hipEvent_t* ev) {
    FusedArgs a{};
    a.colptr = A->colptr;
    a.rowids = A->rowids;
    a.values = A->values;
    a.m = (int32_t)A->m;
    a.n = (int32_t)A->n;
    a.nnz = A->nnz;
    a.x_idx = x_idx;
    a.x_val = x_val;
    a.xmode = xmode;
    a.f = (int32_t)f;
    a.tile_log2 = tl;
    a.nb = nb;
    a.mask = mask;
    a.ctrl = A->ctrl;
    a.lstart = A->cstart;
    a.loff = A->coff;
    a.lxv = A->cxv;
    a.samples = reinterpret_cast<int32_t*>(A->ws + A->L.samples);
    a.xw = reinterpret_cast<uint64_t*>(A->ws + A->L.xw);
    a.xrec = reinterpret_cast<uint64_t*>(A->ws + A->L.xrec);
    a.gpoff = reinterpret_cast<int64_t*>(A->ws + A->L.gpoff);
    a.roff = reinterpret_cast<int32_t*>(A->ws + A->L.roff);
    a.rows_cap = A->L.rows_cap;
    a.buckets = A->buckets;
    a.y_idx = y_idx;
    a.y_val = y_val;
    a.y_cap = y_cap;
    a.d_nnz_y = d_nnz_y;
    // the row width of the offsets array is fixed at create
    a.nb = nb;
    if (nb > A->L.fnb) return fail(SPMSPV_EUNSUPPORTED, "too many buckets for the one-launch multiply");
    const LaunchEvents le{ev ? ev[0] : nullptr, ev ? ev[1] : nullptr};
    HIP_TRY(launch_fused(a, semiring, G, s, ev ? &le : nullptr));
    if (ev)
        for (int k = 2; k < 6; ++k) HIP_TRY(hipEventRecord(ev[k], s));   // the scatter and merge phases take no separate time
    return SPMSPV_OK;
}

// The pull direction's dense output holds the semiring's identity between
// calls (every emitted row is reset to it); a change of semiring refills it.
// Called eagerly before a BFS level graph is captured or replayed too, so a
// graph never holds the refill: the host's record of the identity would not
// follow a replay.
int set_ydense_ident(spmspv_matrix* A, int semiring, hipStream_t s) {
    const uint32_t ident = semiring == SR_MIN_SELECT2ND ? 0x7fffffffu : 0u;
    if (A->ydense_ident != ident) {
        HIP_TRY(launch_fill_ident(A->p_ydense, ident, A->m, s));
        A->ydense_ident = ident;
    }
    return SPMSPV_OK;
}

// Enqueue one pull-direction multiply (three launches).
int enqueue_pull(spmspv_matrix* A, int semiring, int xmode, int64_t f_host, const int32_t* f_dev,
                 const int32_t* x_idx, const void* x_val, int32_t* y_idx, void* y_val, int64_t y_cap,
                 int64_t* d_nnz_y, bool bfs, const uint32_t* mask, bool bump, bool gate, hipStream_t s,
                 hipEvent_t* ev, bool rowwise = false) {
    if (const int rc = set_ydense_ident(A, semiring, s)) return rc;
    PullArgs pa{};
    pa.ctrl = A->ctrl;
    pa.m = (int32_t)A->m;
    pa.n = (int32_t)A->n;
    pa.nnz = A->nnz;
    pa.rowptr = A->rowptr;
    pa.colids = A->colids;
    pa.values = A->rvalues;
    pa.part = A->p_part;
    pa.pull_blocks = pull_blocks((int32_t)A->m, A->nnz);
    pa.x_idx = x_idx;
    pa.x_val = x_val;
    pa.f_host = (int32_t)f_host;
    pa.f_dev = f_dev;
    pa.xbits = A->p_xbits;
    pa.xdense = A->p_xdense;
    pa.ybits = A->p_ybits;
    pa.ydense = A->p_ydense;
    pa.mask = mask;
    pa.lbp = A->p_lbp;
    pa.emit_blocks = pull_emit_blocks((int32_t)A->m);
    pa.y_idx = y_idx;
    pa.y_val = y_val;
    pa.y_cap = y_cap;
    pa.d_nnz_y = d_nnz_y;
    pa.visited = A->visited;
    pa.set_f = bfs ? 1 : 0;
    pa.bump_level = bump ? 1 : 0;
    pa.gate = gate ? 1 : 0;
    if (bfs && gate) {   // level of a direction-switching BFS (square A)
        pa.chain = 1;
        pa.colptr = A->colptr;
        pa.chain_part = A->p_chain;
        pa.x_index = xmode == XV_INDEX ? 1 : 0;
    }
    const bool early = semiring == SR_OR_AND || (semiring == SR_MIN_SELECT2ND && xmode == XV_INDEX && A->rows_sorted);
    if (ev) HIP_TRY(hipEventRecord(ev[0], s));
    HIP_TRY(launch_pull(pa, semiring, xmode, bfs, early, bfs || rowwise, s));
    if (ev) {   // the pull launches count as the first phase
        for (int k = 1; k < 6; ++k) HIP_TRY(hipEventRecord(ev[k], s));
    }
    return SPMSPV_OK;
}

int read_ctrl(spmspv_matrix* A, Ctrl* h, hipStream_t s);

// Tile of a selector class c < 9: 2^(c+4) buckets over m rows, clamped to
// what LDS and the scatter histogram can hold.
// Selector class c < 9: push with 2^(c+4) buckets, i.e. the tile
// ceil_log2(m) - (c + 4) (at least 2^8 rows, widened while the scatter's
// bucket histogram would not fit LDS), merged in LDS: a tile wider than the
// semiring's LDS accumulator runs as the widest one it holds.  (The HBM
// merge would realise the wider tiles, but its global atomics made those
// classes several times slower than the widest LDS tile on the scale-24
// graph -- 1.2 ms against 0.22 ms on a 2,290-vertex frontier -- and a
// network trained on smaller graphs, where the same classes were LDS tiles,
// cannot foresee that; it stays a schedule the caller or the autotuner
// chooses.)
int class_tile(const spmspv_matrix* A, int c) {
    int tl = ceil_log2(A->m) - (c + 4);
    if (tl < kTileLog2Min) tl = kTileLog2Min;
    if (tl > kTileLog2Max) tl = kTileLog2Max;
    while (tl < kTileLog2Max && scatter_lds_bytes((int)((A->m + (int64_t(1) << tl) - 1) >> tl),
                                                 A->sched.scatter_block * A->sched.scatter_items) + 1024 >
                                   A->lds_max)
        ++tl;
    return tl;
}


// One multiply whose schedule the selector MLP picks: scan, selector
// inference on the device, one host read of the class, then the chosen
// push tile or the pull direction.  Returns the class in *cls.
int run_selected(spmspv_matrix* A, int semiring, int xmode, int64_t f_host, const int32_t* f_dev,
                 const int32_t* x_idx, const void* x_val, int32_t* y_idx, void* y_val, int64_t y_cap,
                 int64_t* d_nnz_y, bool bfs, const uint32_t* mask, hipStream_t s, int* cls, int32_t* f_now,
                 int forced = -1) {
    const int clear_nb = (int)((A->m + (int64_t(1) << kTileLog2Min) - 1) >> kTileLog2Min);
    int rc = enqueue(A, semiring, xmode, f_host, f_dev, x_idx, x_val, y_idx, y_val, y_cap, d_nnz_y, bfs, mask, s,
                     nullptr, false, -1, 1, clear_nb);
    if (rc) return rc;
    HIP_TRY(launch_select(A->ctrl, A->selector, (int32_t)A->n, A->nnz, A->pull ? 1 : 0, 0, forced, s));
    Ctrl h{};
    rc = read_ctrl(A, &h, s);
    if (rc) return rc;
    *cls = h.cls;
    if (f_now) *f_now = h.f;
    if (h.cls == 9 && A->pull && h.f > 0) {
        // the scatter that normally clears the scan's look-back words is skipped
        HIP_TRY(launch_clear_u64(A->lb1, (int)A->L.lb1_n * 2, s));
        return enqueue_pull(A, semiring, xmode, f_host, f_dev, x_idx, x_val, y_idx, y_val, y_cap, d_nnz_y, bfs,
                            mask, false, false, s, nullptr);
    }
    const int c = h.cls < 9 ? h.cls : 8;
    return enqueue(A, semiring, xmode, f_host, f_dev, x_idx, x_val, y_idx, y_val, y_cap, d_nnz_y, bfs, mask, s,
                   nullptr, false, class_tile(A, c), 2, 0, false, 0, false, 0);
}

// Shape of a batched call: the narrowest tile at or above the handle's whose
// nbatch * buckets keys fit the key limit and whose scatter histogram fits
// LDS with one of the candidate workgroup shapes.
int batch_shape(const spmspv_matrix* A, int nbatch, int semiring, spmspv_schedule* out) {
    spmspv_schedule sc = A->sched;
    if (A->batch_sched.tile_log2 > 0) sc = A->batch_sched;
    const int shapes[4][2] = {{sc.scatter_block, sc.scatter_items}, {1024, 4}, {512, 4}, {256, 4}};
    for (int tl = call_tile(A, sc.tile_log2, semiring); tl <= kTileLog2Max; ++tl) {
        if (merge_lds_bytes(tl, semiring) + 1024 > A->lds_max) break;
        const int64_t nbx = (A->m + (int64_t(1) << tl) - 1) >> tl;
        const int64_t K = nbx * nbatch;
        if (K > kMaxKeys) continue;
        for (const auto& sh : shapes) {
            if (!scatter_shape_supported(sh[0], sh[1])) continue;
            if (scatter_lds_bytes((int)K, sh[0] * sh[1], true) + 1024 > A->lds_max) continue;
            *out = sc;
            out->tile_log2 = tl;
            out->merge_variant = 0;   // batched keys merge in LDS
            out->scatter_block = sh[0];
            out->scatter_items = sh[1];
            return SPMSPV_OK;
        }
    }
    return fail(SPMSPV_EUNSUPPORTED, "batch too large for the key limit: nbatch * ceil(m / 2^15) must be <= " +
                                         std::to_string(kMaxKeys));
}

int enqueue_batch(spmspv_matrix* A, int semiring, int xmode, int nbatch, const int64_t* x_off, const int32_t* x_idx,
                  const void* x_val, int64_t* y_off, int32_t* y_idx, void* y_val, int64_t y_cap, bool bfs,
                  hipStream_t s) {
    BatchCtx& B = A->batch;
    char* w = B.ws;
    const BatchLayout& L = B.L;
    spmspv_schedule sc{};
    int rc = batch_shape(A, nbatch, semiring, &sc);
    if (rc) return rc;
    const int tl = sc.tile_log2;
    const int nbx = (int)((A->m + (int64_t(1) << tl) - 1) >> tl);
    const int K = nbx * nbatch;
    const int chunk = sc.scatter_block * sc.scatter_items;
    const int chunk_log2 = ceil_log2(chunk);
    auto i32 = [&](size_t off) { return reinterpret_cast<int32_t*>(w + off); };
    int32_t* kcount = i32(L.kcount);
    uint32_t* visited = bfs ? reinterpret_cast<uint32_t*>(w + L.visited) : nullptr;

    ScanArgs sa{};
    sa.colptr = A->colptr;
    if (A->dcsc) {
        sa.dcsc = 1;
        sa.dc_jc = A->dc_jc;
        sa.dc_aux = A->dc_aux;
        sa.dc_shift = A->dc_shift;
    }
    sa.n = (int32_t)A->n;
    sa.x_idx = x_idx;
    sa.x_val = x_val;
    sa.xmode = xmode;
    sa.ctrl = A->ctrl;
    sa.cstart = i32(L.cstart);
    sa.coff = i32(L.coff);
    sa.cxv = reinterpret_cast<uint32_t*>(w + L.cxv);
    sa.chunk_col = i32(L.chunk_col);
    sa.chunk_log2 = chunk_log2;
    sa.lb1 = reinterpret_cast<uint64_t*>(w + L.lb1);
    sa.lb1_n = (int32_t)L.lb1_n;
    sa.nnz = L.max_products;
    sa.chunk_n = L.chunk_n;
    sa.cursor = i32(L.cursor);
    sa.lb3 = reinterpret_cast<uint64_t*>(w + L.lb3);
    sa.nb = K;
    sa.bump_level = bfs ? 1 : 0;
    sa.xoff = x_off;
    sa.nbatch = nbatch;
    sa.f_cap = L.max_f;
    sa.cxid = i32(L.cxid);
    sa.kcount = kcount;
    int64_t g1 = (L.max_f + kScanTile - 1) / kScanTile;
    if (g1 < 1) g1 = 1;
    if (g1 > 2 * A->num_cu) g1 = 2 * A->num_cu;   // co-resident: look-back waits stay bounded

    ScatterArgs ca{};
    ca.rowids = A->rowids;
    ca.values = A->values;
    ca.ctrl = A->ctrl;
    ca.cstart = sa.cstart;
    ca.coff = sa.coff;
    ca.cxv = sa.cxv;
    ca.chunk_col = sa.chunk_col;
    ca.chunk_log2 = chunk_log2;
    ca.tile_log2 = tl;
    ca.nb = K;
    ca.m = (int32_t)A->m;
    ca.rcp = A->rcp;
    ca.cursor = sa.cursor;
    ca.buckets = reinterpret_cast<uint2*>(w + L.buckets);
    ca.mask = visited;
    ca.lb1 = sa.lb1;
    ca.lb1_n = sa.lb1_n;
    ca.lb1_clear = (int32_t)L.lb1_n;
    ca.cxid = sa.cxid;
    ca.kcount = kcount;
    ca.kbase = kcount;   // scanned in place between the two passes
    ca.nbx = nbx;
    ca.mask_words = L.mask_words;
    int64_t g2 = (L.max_products + chunk - 1) / chunk;
    if (g2 < 1) g2 = 1;
    const int64_t g2max =
        int64_t(A->num_cu) * scatter_occupancy(A, semiring, K, sc.scatter_block, sc.scatter_items, true);
    if (g2 > g2max) g2 = g2max;

    MergeArgs ma{};
    ma.ctrl = A->ctrl;
    ma.cursor = sa.cursor;
    ma.buckets = ca.buckets;
    ma.rcp = A->rcp;
    ma.m = (int32_t)A->m;
    ma.tile_log2 = tl;
    ma.nb = K;
    ma.lb3 = sa.lb3;
    ma.y_idx = y_idx;
    ma.y_val = y_val;
    ma.y_cap = y_cap;
    ma.d_nnz_y = nullptr;
    ma.visited = visited;
    ma.set_f = bfs ? 1 : 0;
    ma.kbase = kcount;
    ma.nbx = nbx;
    ma.nbatch = nbatch;
    ma.yoff = y_off;
    ma.n_stride = A->n;
    ma.mask_words = L.mask_words;

    // With distinct indices inside each vector (a precondition of every
    // multiply; multi-source BFS frontiers are sets), vector x puts at most
    // one product per stored entry of A into bucket b, so bucket b's share
    // is bounded by its rows' entry count rcp[(b+1)T] - rcp[bT] exactly as
    // in a single call.  When the workspace holds nnz slots per vector, key
    // (x, b) owns the fixed slice x * nnz + [rcp[bT], rcp[(b+1)T]) and the
    // counting pass is not needed.  A repeated index can overflow a slice:
    // the scatter then drops the run and raises an error bit.
    const bool fixed = L.max_products >= (int64_t)nbatch * A->nnz && A->nnz > 0;
    A->batch.fixed_last = fixed;
    if (fixed) {
        ca.xstride = A->nnz;
        ma.xstride = A->nnz;
        ca.lb1_clear = (int32_t)L.lb1_n;   // the counting pass normally clears these
    }
    HIP_TRY(launch_scan(sa, (int)g1, s));
    if (!fixed) {
        HIP_TRY(launch_scatter_batch(ca, semiring, sc.scatter_block, sc.scatter_items, (int)g2, true, s));
        HIP_TRY(launch_exclusive_scan_i32(kcount, K + 1, i32(L.partials), s));
    }
    HIP_TRY(launch_scatter_batch(ca, semiring, sc.scatter_block, sc.scatter_items, (int)g2, false, s));
    HIP_TRY(launch_merge_batch(ma, semiring, sc.merge_block, bfs, s));
    return SPMSPV_OK;
}

// Schedule of the autotuned band nearest (in log density) to f / n.
const spmspv_schedule* tuned_for(const spmspv_matrix* A, int64_t f) {
    if (A->tuned.empty()) return nullptr;
    const double d = std::log(std::max(1.0, (double)f) / (double)A->n);
    const spmspv_tune_entry* best = &A->tuned[0];
    for (const auto& e : A->tuned)
        if (std::fabs(std::log(e.density) - d) < std::fabs(std::log(best->density) - d)) best = &e;
    return &best->sched;
}

// Average device time of `reps` calls under schedule `sc` (two untimed
// calls first), on stream s.
int time_schedule(spmspv_matrix* A, const spmspv_schedule& sc, int semiring, int xmode, int64_t f,
                  const int32_t* x_idx, const void* x_val, int32_t* y_idx, void* y_val, int reps, hipStream_t s,
                  double* us) {
    const spmspv_schedule keep = A->sched;
    A->sched = sc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SPMSPV_OK;
    auto once = [&]() {
        return sc.direction == 1 ? enqueue_pull(A, semiring, xmode, f, nullptr, x_idx, x_val, y_idx, y_val, A->m,
                                                nullptr, false, nullptr, false, false, s, nullptr)
                                 : enqueue(A, semiring, xmode, f, nullptr, x_idx, x_val, y_idx, y_val, A->m, nullptr,
                                           false, nullptr, s, nullptr);
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(SPMSPV_EHIP, "event");
    for (int k = 0; k < 2 && !rc; ++k) rc = once();
    if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = fail(SPMSPV_EHIP, "event record");
    for (int k = 0; k < reps && !rc; ++k) rc = once();
    if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = fail(SPMSPV_EHIP, "event record");
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(SPMSPV_EHIP, "event sync");
    float ms = 0.f;
    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(SPMSPV_EHIP, "event time");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    A->sched = keep;
    if (!rc) *us = 1e3 * ms / reps;
    return rc;
}

hipEvent_t* profile_slot(spmspv_matrix* A) {
    if (A->prof_ev.empty()) {
        A->prof_ev.resize(size_t(kProfileSlots) * 6);
        for (auto& e : A->prof_ev)
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
    }
    if (A->prof_used >= kProfileSlots) return nullptr;
    return &A->prof_ev[size_t(A->prof_used++) * 6];
}

// Point a handle at matrix arrays and a workspace laid out by make_layout.
void bind_workspace(spmspv_matrix* A, int64_t m, int64_t n, int64_t nnz, const int32_t* colptr,
                    const int32_t* rowids, const float* values, char* ws, int flags, int64_t dc_chunks = 0) {
    A->m = m;
    A->n = n;
    A->nnz = nnz;
    A->colptr = colptr;
    A->rowids = rowids;
    A->values = values;
    A->L = make_layout(m, n, nnz, flags, dc_chunks);
    A->ws = ws;
    const Layout& L = A->L;
    A->ctrl = reinterpret_cast<Ctrl*>(A->ws + L.ctrl);
    A->rcp = reinterpret_cast<int32_t*>(A->ws + L.rcp);
    A->cstart = reinterpret_cast<int32_t*>(A->ws + L.cstart);
    A->coff = reinterpret_cast<int32_t*>(A->ws + L.coff);
    A->cxv = reinterpret_cast<uint32_t*>(A->ws + L.cxv);
    A->chunk_col = reinterpret_cast<int32_t*>(A->ws + L.chunk_col);
    A->lb1 = reinterpret_cast<uint64_t*>(A->ws + L.lb1);
    A->cursor = reinterpret_cast<int32_t*>(A->ws + L.cursor);
    A->lb3 = reinterpret_cast<uint64_t*>(A->ws + L.lb3);
    A->buckets = reinterpret_cast<uint2*>(A->ws + L.buckets);
    A->visited = reinterpret_cast<uint32_t*>(A->ws + L.visited);
    A->front[0] = reinterpret_cast<int32_t*>(A->ws + L.front0);
    A->front[1] = reinterpret_cast<int32_t*>(A->ws + L.front1);
    A->front2 = reinterpret_cast<int32_t*>(A->ws + L.front2);
    A->disc = reinterpret_cast<uint32_t*>(A->ws + L.disc);
    A->pmin = reinterpret_cast<int32_t*>(A->ws + L.pmin);
    A->bar = reinterpret_cast<uint32_t*>(A->ws + L.bar);
    A->selector = reinterpret_cast<float*>(A->ws + L.selector);
    A->bv_idx = reinterpret_cast<int32_t*>(A->ws + L.bv_idx);
    A->bv_val = reinterpret_cast<uint32_t*>(A->ws + L.bv_val);
    A->bv_tiles = reinterpret_cast<int32_t*>(A->ws + L.bv_tiles);
    A->dc_aux = dc_chunks > 0 ? reinterpret_cast<int32_t*>(A->ws + L.dc_aux) : nullptr;
}

int read_ctrl(spmspv_matrix* A, Ctrl* h, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(h, A->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SPMSPV_OK;
}

// Persistent BFS scratch between launches: bitmaps clear, pmin at INT32_MAX.
hipError_t reset_persistent_state(spmspv_matrix* A, hipStream_t s) {
    hipError_t e = launch_fill_u32(A->disc, 0u, 3 * ((A->m + 31) / 32), s);
    if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t*>(A->pmin), 0x7fffffffu, A->m, s);
    return e;
}

// Clears the sticky error bits, and the persistent BFS scratch, which a
// launch that gave up at a barrier leaves as it was.
int clear_err(spmspv_matrix* A, hipStream_t s) {
    HIP_TRY(launch_fill_u32(&A->ctrl->err, 0u, 1, s));
    HIP_TRY(reset_persistent_state(A, s));
    return SPMSPV_OK;
}

}  // namespace

// Allocation-free multiply (spmspv_run_static): the workspace a handle's
// workspace argument would bring in lives in this file-scope array instead,
// one copy per device, held until the process ends.  In host code the
// array's name is only a stand-in: its device address is looked up once per
// device with hipGetSymbolAddress and every launch takes that address.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kStaticMaxDevices = 64;

struct StaticDevice {
    std::atomic<void*> ptr{nullptr};   // device address of `scratch` on this device
    int num_cu = 0;
    size_t lds_max = 0;
};
StaticDevice g_static[kStaticMaxDevices];
std::mutex g_static_mu;

// Address of this device's scratch array (and its unit count and LDS size),
// found once per device with that device current.
int static_scratch(int* dev_out, void** ptr_out, StaticDevice** info_out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(SPMSPV_EUNSUPPORTED, "device index beyond the static table");
    StaticDevice& d = g_static[dev];
    void* p = d.ptr.load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        p = d.ptr.load(std::memory_order_relaxed);
        if (!p) {
            int v = 0;
            d.num_cu = (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
                           ? v : 256;
            d.lds_max = (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
                         v > 0) ? (size_t)v : 65536;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                       "hipGetSymbolAddress(scratch)");
            d.ptr.store(p, std::memory_order_release);
        }
    }
    *dev_out = dev;
    *ptr_out = p;
    *info_out = &d;
    return SPMSPV_OK;
}

}  // namespace

extern "C" {

const char* spmspv_status_string(int status) {
    switch (status) {
        case SPMSPV_OK: return "ok";
        case SPMSPV_EINVAL: return "invalid argument or input";
        case SPMSPV_ENOMEM: return "workspace too small";
        case SPMSPV_ECAPACITY: return "output capacity too small";
        case SPMSPV_EHIP: return "HIP runtime error";
        case SPMSPV_EUNSUPPORTED: return "unsupported request";
        case SPMSPV_EDEVICE: return "device reported an error";
        default: return "unknown status";
    }
}

const char* spmspv_last_error(void) { return g_last_error.c_str(); }

int spmspv_workspace_size(int64_t m, int64_t n, int64_t nnz, int flags, size_t* h_bytes) {
    (void)flags;
    if (!h_bytes) return fail(SPMSPV_EINVAL, "h_bytes is NULL");
    if (m < 1 || n < 1 || nnz < 0 || nnz >= (int64_t(1) << 31) || m >= (int64_t(1) << 31) ||
        n >= (int64_t(1) << 31))
        return fail(SPMSPV_EINVAL, "sizes out of range (need 1 <= m, n < 2^31, 0 <= nnz < 2^31)");
    if ((flags & SPMSPV_SYMMETRIC) && m != n) return fail(SPMSPV_EINVAL, "SPMSPV_SYMMETRIC needs m == n");
    *h_bytes = make_layout(m, n, nnz, flags).total;
    return SPMSPV_OK;
}

namespace {

// DCSC column index: chunks of 2^shift column ids, about one stored column
// per chunk (at most 2 nzc + 1 chunks).
int dcsc_shift(int64_t n, int64_t nzc) {
    int sh = 0;
    while ((n >> sh) > std::max<int64_t>(nzc, 1)) ++sh;
    return sh;
}
int64_t dcsc_chunks(int64_t n, int64_t nzc) { return ((n - 1) >> dcsc_shift(n, nzc)) + 1; }

// spmspv_create and spmspv_create_dcsc.  CSC: jc == nullptr and colptr has
// n + 1 entries; DCSC: colptr has nzc + 1 entries, the starts of the stored
// columns jc[0..nzc).
int create_impl(spmspv_handle* h_out, int64_t m, int64_t n, int64_t nnz, int64_t nzc, const int32_t* jc,
                const int32_t* colptr, const int32_t* rowids, const float* values, void* workspace, size_t ws_bytes,
                int flags, void* stream) {
    if (!h_out) return fail(SPMSPV_EINVAL, "h_out is NULL");
    *h_out = nullptr;
    const bool dcsc = nzc >= 0;
    size_t need = 0;
    int rc = dcsc ? spmspv_dcsc_workspace_size(m, n, nzc, nnz, flags, &need)
                  : spmspv_workspace_size(m, n, nnz, flags, &need);
    if (rc) return rc;
    if (!colptr || (nnz > 0 && !rowids) || !workspace || (dcsc && nzc > 0 && !jc))
        return fail(SPMSPV_EINVAL, "NULL matrix or workspace");
    if (ws_bytes < need) return fail(SPMSPV_ENOMEM, "workspace smaller than the workspace size call's");
    if ((reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
        return fail(SPMSPV_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);

    auto* A = new spmspv_matrix();
    bind_workspace(A, m, n, nnz, colptr, rowids, values, static_cast<char*>(workspace), flags,
                   dcsc ? dcsc_chunks(n, nzc) : 0);
    const Layout& L = A->L;
    if (dcsc) {
        A->dcsc = true;
        A->nzc = nzc;
        A->dc_jc = jc;
        A->dc_shift = dcsc_shift(n, nzc);
    }

    auto bail = [&](int status) {
        delete A;
        return status;
    };
    hipError_t e = hipGetDevice(&A->device);
    if (e != hipSuccess) return bail(hip_fail(e, "hipGetDevice"));
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, A->device) == hipSuccess && v > 0)
        A->num_cu = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, A->device) == hipSuccess && v > 0)
        A->lds_max = (size_t)v;

    // Zero the control block and the per-call look-back / counter state.
    const size_t zero_end = L.buckets;
    if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(A->ws), 0u, int64_t(zero_end / 4), s)) != hipSuccess)
        return bail(hip_fail(e, "zero workspace"));
    if ((e = launch_validate_colptr(colptr, (int32_t)(dcsc ? nzc : n), nnz, A->ctrl, &A->ctrl->maxdeg, s)) !=
        hipSuccess)
        return bail(hip_fail(e, "validate colptr"));
    if (dcsc) {
        if ((e = launch_validate_jc(jc, (int32_t)nzc, (int32_t)n, A->ctrl, s)) != hipSuccess)
            return bail(hip_fail(e, "validate column ids"));
        if ((e = launch_dcsc_aux(jc, (int32_t)nzc, A->dc_shift, (int32_t)dcsc_chunks(n, nzc), A->dc_aux, s)) !=
            hipSuccess)
            return bail(hip_fail(e, "DCSC column index"));
    }
    if ((e = launch_row_counts(rowids, nnz, (int32_t)m, A->rcp, A->ctrl, s)) != hipSuccess)
        return bail(hip_fail(e, "row counts"));
    if ((e = launch_exclusive_scan_i32(A->rcp, m + 1, reinterpret_cast<int32_t*>(A->ws + L.partials), s)) !=
        hipSuccess)
        return bail(hip_fail(e, "row count scan"));
    if ((e = reset_persistent_state(A, s)) != hipSuccess || (e = launch_fill_u32(A->bar, 0u, 160, s)) != hipSuccess)
        return bail(hip_fail(e, "persistent BFS state"));
    // the HBM accumulator starts (and is left after every call) empty
    if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(A->ws + L.h_f64), 0x8000000000000000ull, L.h_rows, s)) !=
            hipSuccess ||
        (e = launch_fill_u32(reinterpret_cast<uint32_t*>(A->ws + L.h_i32), 0x7fffffffu, L.h_rows, s)) != hipSuccess ||
        (e = launch_fill_u32(reinterpret_cast<uint32_t*>(A->ws + L.h_orbits), 0u, (L.h_rows + 31) / 32, s)) !=
            hipSuccess ||
        (e = launch_fill_u32(reinterpret_cast<uint32_t*>(A->ws + L.h_touched), 0u, (L.h_rows + 31) / 32, s)) !=
            hipSuccess)
        return bail(hip_fail(e, "HBM accumulator"));
    if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(A->ws + L.gb_bytes), 0u, (L.h_rows + 31) / 32 * 8, s)) !=
        hipSuccess)
        return bail(hip_fail(e, "mask byte map"));
    if (L.pull) {
        A->pull = true;
        A->p_xbits = reinterpret_cast<uint32_t*>(A->ws + L.p_xbits);
        A->p_xdense = reinterpret_cast<uint32_t*>(A->ws + L.p_xdense);
        A->p_ybits = reinterpret_cast<uint32_t*>(A->ws + L.p_ybits);
        A->p_ydense = reinterpret_cast<uint32_t*>(A->ws + L.p_ydense);
        A->p_lbp = reinterpret_cast<uint64_t*>(A->ws + L.p_lbp);
        A->p_part = reinterpret_cast<int32_t*>(A->ws + L.p_part);
        A->p_chain = reinterpret_cast<int64_t*>(A->ws + L.p_chain);
        // every pull region up to the transpose starts at zero (ydense = identity of + and or)
        const size_t zb = L.p_xbits, ze = L.transpose ? L.t_colids : L.total;
        if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(A->ws + zb), 0u, int64_t((ze - zb) / 4), s)) != hipSuccess)
            return bail(hip_fail(e, "zero pull buffers"));
        A->ydense_ident = 0;
        int32_t* colids_t = nullptr;
        float* tvalues = nullptr;
        if (L.transpose) {
            colids_t = reinterpret_cast<int32_t*>(A->ws + L.t_colids);
            tvalues = values ? reinterpret_cast<float*>(A->ws + L.t_values) : nullptr;
            if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(A->front[0]), 0u, m, s)) != hipSuccess)
                return bail(hip_fail(e, "zero transpose cursors"));
            A->rowptr = A->rcp;
            A->colids = reinterpret_cast<const uint32_t*>(colids_t);
            A->rvalues = tvalues;
        } else {
            A->rowptr = colptr;
            A->colids = reinterpret_cast<const uint32_t*>(rowids);
            A->rvalues = values;
        }
        if ((e = launch_pull_setup(colptr, rowids, values, (int32_t)m, (int32_t)n, nnz, A->rowptr, A->front[0],
                                   colids_t, tvalues, A->p_part, L.transpose ? nullptr : &A->ctrl->unsorted, s)) !=
            hipSuccess)
            return bail(hip_fail(e, "pull set-up"));
        // longest row: bounds the products of a left multiplication
        if ((e = launch_validate_colptr(A->rowptr, (int32_t)m, nnz, A->ctrl, &A->ctrl->maxrow, s)) != hipSuccess)
            return bail(hip_fail(e, "row lengths"));
    }
    Ctrl h{};
    if ((e = hipMemcpyAsync(&h, A->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return bail(hip_fail(e, "read control block"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return bail(hip_fail(e, "create sync"));
    if (h.err & (ERR_CSC | ERR_ROW_RANGE)) {
        if (flags & SPMSPV_VALIDATE) return bail(fail(SPMSPV_EINVAL, "invalid CSC (colptr or row ids)"));
        // Without validation an invalid matrix is still refused: bucket
        // sizing depends on it.
        return bail(fail(SPMSPV_EINVAL, "invalid CSC detected while sizing buckets"));
    }
    A->maxdeg = h.maxdeg;
    A->maxrow = h.maxrow;
    A->rows_sorted = A->pull && !L.transpose && h.unsorted == 0;
    default_schedule(A, &A->sched);
    if (check_schedule(A, &A->sched) != SPMSPV_OK)
        return bail(fail(SPMSPV_EUNSUPPORTED, "matrix too tall for the LDS bucket layout"));
    *h_out = A;
    return SPMSPV_OK;
}

}  // namespace

int spmspv_create(spmspv_handle* h_out, int64_t m, int64_t n, int64_t nnz, const int32_t* colptr,
                  const int32_t* rowids, const float* values, void* workspace, size_t ws_bytes, int flags,
                  void* stream) {
    return create_impl(h_out, m, n, nnz, -1, nullptr, colptr, rowids, values, workspace, ws_bytes, flags, stream);
}

int spmspv_dcsc_workspace_size(int64_t m, int64_t n, int64_t nzc, int64_t nnz, int flags, size_t* h_bytes) {
    if (!h_bytes) return fail(SPMSPV_EINVAL, "h_bytes is NULL");
    if (flags & ~(SPMSPV_VALIDATE | SPMSPV_DETERMINISTIC))
        return fail(SPMSPV_EINVAL, "a DCSC handle takes only SPMSPV_VALIDATE and SPMSPV_DETERMINISTIC");
    if (nzc < 0 || nzc > n || (nzc == 0 && nnz != 0) || nnz < nzc)
        return fail(SPMSPV_EINVAL, "need 0 <= nzc <= min(n, nnz), nnz == 0 when nzc == 0");
    const int rc = spmspv_workspace_size(m, n, nnz, flags, h_bytes);
    if (rc) return rc;
    *h_bytes = make_layout(m, n, nnz, flags, dcsc_chunks(n, nzc)).total;
    return SPMSPV_OK;
}

int spmspv_create_dcsc(spmspv_handle* h_out, int64_t m, int64_t n, int64_t nzc, int64_t nnz, const int32_t* jc,
                       const int32_t* cp, const int32_t* rowids, const float* values, void* workspace,
                       size_t ws_bytes, int flags, void* stream) {
    if (nzc < 0) return fail(SPMSPV_EINVAL, "nzc must be >= 0");
    return create_impl(h_out, m, n, nnz, nzc, jc, cp, rowids, values, workspace, ws_bytes, flags, stream);
}

int spmspv_get_schedule(spmspv_handle A, spmspv_schedule* h_sched) {
    if (!A || !h_sched) return fail(SPMSPV_EINVAL, "NULL argument");
    *h_sched = A->sched;
    return SPMSPV_OK;
}

int spmspv_effective_schedule(spmspv_handle A, int semiring, int64_t f, int flags, spmspv_schedule* h_sched) {
    if (!A || !h_sched) return fail(SPMSPV_EINVAL, "NULL argument");
    if (semiring < 0 || semiring > 2) return fail(SPMSPV_EINVAL, "unknown semiring");
    if (f < 0 || f > A->n) return fail(SPMSPV_EINVAL, "f must be in [0, n]");
    const spmspv_schedule keep = A->sched;
    const spmspv_schedule* tuned = (flags & SPMSPV_AUTO_SCHEDULE) ? tuned_for(A, f) : nullptr;
    if (tuned) A->sched = *tuned;
    else if (A->sched_default) A->sched = sized_for_call(A, f);
    spmspv_schedule e = A->sched;
    if (e.direction == 0) {
        if (e.merge_variant == 0) e.tile_log2 = call_tile(A, e.tile_log2, semiring);
        e.launch = e.launch == 2 ? 2 : 1;
    }
    A->sched = keep;
    *h_sched = e;
    return SPMSPV_OK;
}

int spmspv_set_schedule(spmspv_handle A, const spmspv_schedule* h_sched) {
    if (!A) return fail(SPMSPV_EINVAL, "NULL handle");
    spmspv_schedule s{};
    if (h_sched) s = *h_sched;
    else default_schedule(A, &s);
    const int rc = check_schedule(A, &s);
    if (rc) return rc;
    A->sched = s;
    A->sched_default = h_sched == nullptr;
    if (A->graph) {
        (void)hipGraphExecDestroy(A->graph);
        A->graph = nullptr;
        A->graph_key = -1;
    }
    return SPMSPV_OK;
}

int spmspv_run(spmspv_handle A, int semiring, int flags, int64_t f, const int32_t* x_idx, const void* x_val,
               int32_t* y_idx, void* y_val, int64_t y_capacity, int64_t* d_nnz_y, int64_t* h_nnz_y, void* stream) {
    return spmspv_run_masked(A, semiring, flags, f, x_idx, x_val, nullptr, y_idx, y_val, y_capacity, d_nnz_y, h_nnz_y,
                             stream);
}

int spmspv_run_masked(spmspv_handle A, int semiring, int flags, int64_t f, const int32_t* x_idx, const void* x_val,
                      const uint32_t* mask, int32_t* y_idx, void* y_val, int64_t y_capacity, int64_t* d_nnz_y,
                      int64_t* h_nnz_y, void* stream) {
    if (!A) return fail(SPMSPV_EINVAL, "NULL handle");
    if (semiring < 0 || semiring > 2) return fail(SPMSPV_EINVAL, "unknown semiring");
    const bool left = (flags & SPMSPV_LEFT) != 0;
    const int64_t xlen = left ? A->m : A->n;
    if (f < 0 || f > xlen) return fail(SPMSPV_EINVAL, left ? "f must be in [0, m]" : "f must be in [0, n]");
    if (f > 0 && !x_idx) return fail(SPMSPV_EINVAL, "x_idx is NULL");
    if (y_capacity < 0 || (y_capacity > 0 && !y_idx)) return fail(SPMSPV_EINVAL, "bad y buffer");
    int xmode = XV_BITS32;
    if (semiring == SR_MIN_SELECT2ND && (flags & SPMSPV_X_VAL_IS_INDEX)) xmode = XV_INDEX;
    else if (semiring == SR_OR_AND) xmode = (flags & SPMSPV_X_ALL_TRUE) ? XV_TRUE : XV_U8;
    if (f > 0 && !x_val && (xmode == XV_BITS32 || xmode == XV_U8)) return fail(SPMSPV_EINVAL, "x_val is NULL");
    if ((flags & SPMSPV_PULL_ROWWISE) && semiring == SR_PLUS_TIMES)
        return fail(SPMSPV_EINVAL, "SPMSPV_PULL_ROWWISE is for min-select2nd and or-and");
    if (left && !A->pull)
        return fail(SPMSPV_EUNSUPPORTED, "SPMSPV_LEFT needs a handle created with SPMSPV_WITH_TRANSPOSE or "
                                         "SPMSPV_SYMMETRIC");
    if (left && (flags & (SPMSPV_USE_SELECTOR | SPMSPV_PULL_ROWWISE | SPMSPV_AUTO_SCHEDULE)))
        return fail(SPMSPV_EINVAL, "SPMSPV_LEFT runs the push multiply only (no selector, pull or tuned schedule)");
    if (A->dcsc && (flags & SPMSPV_USE_SELECTOR))
        return fail(SPMSPV_EUNSUPPORTED, "the selector needs a CSC handle");
    hipStream_t s = static_cast<hipStream_t>(stream);

    if (flags & SPMSPV_VALIDATE) {
        std::vector<int32_t> hx((size_t)f);
        if (f) HIP_TRY(hipMemcpyAsync(hx.data(), x_idx, size_t(f) * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        std::vector<uint8_t> seen((size_t)xlen, 0);
        for (int64_t p = 0; p < f; ++p) {
            const int32_t j = hx[(size_t)p];
            if (j < 0 || j >= xlen) return fail(SPMSPV_EINVAL, "x index out of range");
            if (seen[(size_t)j]) return fail(SPMSPV_EINVAL, "duplicate x index");
            seen[(size_t)j] = 1;
        }
    }
    hipEvent_t* ev = (flags & SPMSPV_PROFILE) ? profile_slot(A) : nullptr;
    int rc;
    if ((flags & SPMSPV_DETERMINISTIC) && semiring == SR_PLUS_TIMES) {
        // min and or are order-free: only plus-times takes the ordered fold
        if (flags & (SPMSPV_USE_SELECTOR | SPMSPV_PULL_ROWWISE))
            return fail(SPMSPV_EINVAL, "SPMSPV_DETERMINISTIC runs the push multiply only");
        const spmspv_schedule keep = A->sched;
        if (A->sched_default && !left) A->sched = sized_for_call(A, f);
        rc = enqueue_det(A, xmode, f, x_idx, x_val, y_idx, static_cast<float*>(y_val), y_capacity, d_nnz_y, mask, 0,
                         left, s);
        A->sched = keep;
    } else if (left) {
        const spmspv_schedule keep = A->sched;
        A->sched.direction = 0;
        rc = enqueue(A, semiring, xmode, f, nullptr, x_idx, x_val, y_idx, y_val, y_capacity, d_nnz_y, false, mask, s,
                     ev, false, -1, 3, 0, false, 0, true);
        A->sched = keep;
    } else if (flags & SPMSPV_USE_SELECTOR) {
        if (!A->selector_loaded) return fail(SPMSPV_EINVAL, "no selector weights loaded");
        int cls = 0;
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(&A->ctrl->bfs_mode), 0u, 1, s));
        rc = run_selected(A, semiring, xmode, f, nullptr, x_idx, x_val, y_idx, y_val, y_capacity, d_nnz_y, false,
                          mask, s, &cls, nullptr);
    } else {
        const spmspv_schedule keep = A->sched;
        const spmspv_schedule* tuned = (flags & SPMSPV_AUTO_SCHEDULE) ? tuned_for(A, f) : nullptr;
        if (tuned) A->sched = *tuned;
        else if (A->sched_default) A->sched = sized_for_call(A, f);
        int G = 0, ftl = 0, fnb = 0;
        if (A->sched.direction == 0 && A->sched.launch == 2) {
            G = A->dcsc ? 0 : fused_eligible(A, semiring, f, &ftl, &fnb);
            if (G == 0) {
                A->sched = keep;
                return fail(SPMSPV_EUNSUPPORTED, "this call cannot run as one launch (f > 4096 per compute unit, "
                                                 "more than 1024 buckets, or no co-resident grid)");
            }
        }
        if (A->sched.direction == 1)
            rc = enqueue_pull(A, semiring, xmode, f, nullptr, x_idx, x_val, y_idx, y_val, y_capacity, d_nnz_y, false,
                              mask, false, false, s, ev, (flags & SPMSPV_PULL_ROWWISE) != 0);
        else if (G > 0)
            rc = enqueue_fused(A, semiring, xmode, f, x_idx, x_val, y_idx, y_val, y_capacity, d_nnz_y, mask, G, ftl,
                               fnb, s, ev);
        else
            rc = enqueue(A, semiring, xmode, f, nullptr, x_idx, x_val, y_idx, y_val, y_capacity, d_nnz_y, false, mask,
                         s, ev);
        A->sched = keep;
    }
    if (rc) return rc;
    if (h_nnz_y) {
        Ctrl h{};
        rc = read_ctrl(A, &h, s);
        if (rc) return rc;
        *h_nnz_y = h.nnz_y;
        if (h.err) {
            clear_err(A, s);
            return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err) +
                                            " (1 = x index range, 2 = duplicate x index, 4 = look-back bound)");
        }
        if (h.nnz_y > y_capacity) return fail(SPMSPV_ECAPACITY, "nnz(y) exceeds y_capacity");
    }
    return SPMSPV_OK;
}

int spmspv_run_bitvector(spmspv_handle A, int semiring, int flags, const uint32_t* x_bits, const void* x_val,
                         uint32_t* y_bits, void* y_val, int64_t y_capacity, int64_t* d_nnz_y, int64_t* h_nnz_y,
                         void* stream) {
    if (!A) return fail(SPMSPV_EINVAL, "NULL handle");
    if (semiring < 0 || semiring > 2) return fail(SPMSPV_EINVAL, "unknown semiring");
    if (flags & ~(SPMSPV_SORTED_OUTPUT | SPMSPV_X_VAL_IS_INDEX | SPMSPV_X_ALL_TRUE | SPMSPV_LEFT))
        return fail(SPMSPV_EINVAL, "spmspv_run_bitvector takes SORTED_OUTPUT, X_VAL_IS_INDEX, X_ALL_TRUE, LEFT");
    const bool left = (flags & SPMSPV_LEFT) != 0;
    if (left && !A->pull)
        return fail(SPMSPV_EUNSUPPORTED, "SPMSPV_LEFT needs a handle created with SPMSPV_WITH_TRANSPOSE or "
                                         "SPMSPV_SYMMETRIC");
    if (!x_bits || !y_bits || y_capacity < 0) return fail(SPMSPV_EINVAL, "NULL bitmap or negative capacity");
    int xmode = XV_BITS32;
    if (semiring == SR_MIN_SELECT2ND && (flags & SPMSPV_X_VAL_IS_INDEX)) xmode = XV_INDEX;
    else if (semiring == SR_OR_AND) xmode = (flags & SPMSPV_X_ALL_TRUE) ? XV_TRUE : XV_U8;
    if (!x_val && (xmode == XV_BITS32 || xmode == XV_U8)) return fail(SPMSPV_EINVAL, "x_val is NULL");
    const int64_t xlen = left ? A->m : A->n, ylen = left ? A->n : A->m;
    const int64_t y_cap = y_val ? std::min(y_capacity, ylen) : ylen;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // (1) x's bitmap -> its ascending index list (the values are already in
    // that order); its length stays on the device
    HIP_TRY(launch_bits_to_list(x_bits, (int32_t)xlen, A->bv_idx, &A->ctrl->bv_f, A->bv_tiles, A->ctrl, s));
    // (2) the multiply on the lists, y's bitmap written by the merge from its
    // tiles' touched-row bitmaps (every word, so no clearing pass); y's index
    // list goes to x's storage (the scan has copied what it needs from x
    // before the merge writes y)
    const spmspv_schedule keep = A->sched;
    A->sched.direction = 0;
    const int rc = enqueue(A, semiring, xmode, 0, &A->ctrl->bv_f, A->bv_idx, x_val, A->bv_idx, y_val, y_cap, d_nnz_y,
                           false, nullptr, s, nullptr, false, -1, 3, 0, false, 0, left, -1, y_bits);
    A->sched = keep;
    if (rc) return rc;
    if (h_nnz_y) {
        Ctrl h{};
        const int r = read_ctrl(A, &h, s);
        if (r) return r;
        *h_nnz_y = h.nnz_y;
        if (h.err) {
            clear_err(A, s);
            return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err) +
                                            " (1 = x bit set past the vector length)");
        }
        if (h.nnz_y > y_capacity) return fail(SPMSPV_ECAPACITY, "nnz(y) exceeds y_capacity");
    }
    return SPMSPV_OK;
}

int spmspv_run_graphblas(spmspv_handle A, int semiring, int flags, int64_t f, const int32_t* x_idx,
                         const void* x_val, const int32_t* mask_idx, const uint8_t* mask_val, int64_t mask_count,
                         int mask_flags, int accum, const int32_t* w_idx, const void* w_val, int64_t w_count,
                         int32_t* y_idx, void* y_val, int64_t y_capacity, int64_t* d_nnz_y, int64_t* h_nnz_y,
                         void* stream) {
    if (!A) return fail(SPMSPV_EINVAL, "NULL handle");
    if (semiring < 0 || semiring > 2) return fail(SPMSPV_EINVAL, "unknown semiring");
    // left multiplication: x over A's rows, mask / w / y over its columns
    const bool left = (flags & SPMSPV_LEFT) != 0;
    if (left && !A->pull)
        return fail(SPMSPV_EUNSUPPORTED, "SPMSPV_LEFT needs a handle created with SPMSPV_WITH_TRANSPOSE or "
                                         "SPMSPV_SYMMETRIC");
    const int64_t xlen = left ? A->m : A->n, ylen = left ? A->n : A->m;
    if (f < 0 || f > xlen) return fail(SPMSPV_EINVAL, "f exceeds the length of x");
    if (f > 0 && !x_idx) return fail(SPMSPV_EINVAL, "x_idx is NULL");
    if (mask_count < 0 || (mask_count > 0 && !mask_idx)) return fail(SPMSPV_EINVAL, "bad mask list");
    if (mask_count > ylen) return fail(SPMSPV_EINVAL, "mask longer than y");
    if (mask_flags & ~(SPMSPV_MASK_COMPLEMENT | SPMSPV_MASK_REPLACE)) return fail(SPMSPV_EINVAL, "unknown mask flag");
    if (accum < SPMSPV_ACCUM_NONE || accum > SPMSPV_ACCUM_SECOND) return fail(SPMSPV_EINVAL, "unknown accumulate");
    if (w_count < 0 || w_count > ylen || (w_count > 0 && (!w_idx || !w_val)))
        return fail(SPMSPV_EINVAL, "bad accumulation input w");
    if (y_capacity < 0 || (y_capacity > 0 && !y_idx)) return fail(SPMSPV_EINVAL, "bad y buffer");
    if (flags & ~(SPMSPV_VALIDATE | SPMSPV_SORTED_OUTPUT | SPMSPV_X_VAL_IS_INDEX | SPMSPV_X_ALL_TRUE | SPMSPV_LEFT))
        return fail(SPMSPV_EINVAL,
                    "spmspv_run_graphblas takes VALIDATE, SORTED_OUTPUT, X_VAL_IS_INDEX, X_ALL_TRUE, LEFT");
    int xmode = XV_BITS32;
    if (semiring == SR_MIN_SELECT2ND && (flags & SPMSPV_X_VAL_IS_INDEX)) xmode = XV_INDEX;
    else if (semiring == SR_OR_AND) xmode = (flags & SPMSPV_X_ALL_TRUE) ? XV_TRUE : XV_U8;
    if (f > 0 && !x_val && (xmode == XV_BITS32 || xmode == XV_U8)) return fail(SPMSPV_EINVAL, "x_val is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool complement = (mask_flags & SPMSPV_MASK_COMPLEMENT) != 0;
    const bool replace = (mask_flags & SPMSPV_MASK_REPLACE) != 0;
    const bool has_mask = mask_idx != nullptr;

    if (flags & SPMSPV_VALIDATE) {
        // x: distinct, in range; mask: distinct rows in range; w: strictly ascending rows in range
        std::vector<int32_t> hx((size_t)f), hm((size_t)mask_count), hw((size_t)w_count);
        if (f) HIP_TRY(hipMemcpyAsync(hx.data(), x_idx, size_t(f) * 4, hipMemcpyDeviceToHost, s));
        if (mask_count) HIP_TRY(hipMemcpyAsync(hm.data(), mask_idx, size_t(mask_count) * 4, hipMemcpyDeviceToHost, s));
        if (w_count) HIP_TRY(hipMemcpyAsync(hw.data(), w_idx, size_t(w_count) * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        std::vector<uint8_t> seen((size_t)std::max(A->n, A->m), 0);
        for (int32_t j : hx) {
            if (j < 0 || j >= xlen) return fail(SPMSPV_EINVAL, "x index out of range");
            if (seen[(size_t)j]) return fail(SPMSPV_EINVAL, "duplicate x index");
            seen[(size_t)j] = 1;
        }
        std::fill(seen.begin(), seen.end(), 0);
        for (int32_t i : hm) {
            if (i < 0 || i >= ylen) return fail(SPMSPV_EINVAL, "mask index out of range");
            if (seen[(size_t)i]) return fail(SPMSPV_EINVAL, "duplicate mask index");
            seen[(size_t)i] = 1;
        }
        for (size_t r = 0; r < hw.size(); ++r) {
            if (hw[r] < 0 || hw[r] >= ylen) return fail(SPMSPV_EINVAL, "w index out of range");
            if (r > 0 && hw[r] <= hw[r - 1]) return fail(SPMSPV_EINVAL, "w indices must be strictly ascending");
        }
    }

    // (1) the mask's rows as a bitmap (the BFS visited bitmap's storage)
    uint32_t* bits = nullptr;
    if (has_mask) {
        bits = A->visited;
        HIP_TRY(launch_mask_bits(mask_idx, mask_val, mask_count, (int32_t)ylen,
                                 reinterpret_cast<uint8_t*>(A->ws + A->L.gb_bytes), bits, &A->ctrl->err, s));
    }
    // (2) t = A x restricted to the mask, ascending; straight into y when
    // there is nothing to accumulate into (then the result is t: rows
    // outside the mask have no w to keep)
    const bool direct = w_count == 0;
    int32_t* t_idx = direct ? y_idx : A->bv_idx;
    void* t_val = direct ? y_val : static_cast<void*>(A->bv_val);
    const int64_t t_cap = direct ? y_capacity : ylen;
    int64_t* t_count = direct ? d_nnz_y : &A->ctrl->aux_count;
    const spmspv_schedule keep = A->sched;
    if (A->sched_default && !left) A->sched = sized_for_call(A, f);
    A->sched.direction = 0;
    int rc;
    if (!has_mask && complement) {
        // no row is in the mask: t is empty
        rc = enqueue(A, semiring, xmode, 0, nullptr, x_idx, x_val, t_idx, t_val, t_cap, t_count, false, nullptr, s,
                     nullptr, false, -1, 3, 0, false, 0, left);
    } else {
        rc = enqueue(A, semiring, xmode, f, nullptr, x_idx, x_val, t_idx, t_val, t_cap, t_count, false, bits, s,
                     nullptr, false, -1, 3, 0, false, complement ? 0 : 1, left);
    }
    A->sched = keep;
    if (rc) return rc;
    // (3) merge t with w under the accumulate and replace rules
    if (!direct) {
        CombineArgs ca{};
        ca.t_idx = A->bv_idx;
        ca.t_val = A->bv_val;
        ca.d_nt = &A->ctrl->aux_count;
        ca.w_idx = w_idx;
        ca.w_val = w_val;
        ca.nw = w_count;
        ca.mbits = bits;
        ca.complement = complement ? 1 : 0;
        ca.replace = replace ? 1 : 0;
        ca.accum = accum;
        ca.y_idx = y_idx;
        ca.y_val = y_val;
        ca.y_cap = y_capacity;
        ca.d_nnz_y = d_nnz_y;
        ca.ctrl = A->ctrl;
        ca.lb = reinterpret_cast<uint64_t*>(A->ws + A->L.gb_lb);
        ca.lb_n = (int32_t)gb_lb_words(ylen);
        HIP_TRY(launch_clear_u64(ca.lb, ca.lb_n, s));
        int64_t grid = (ylen + w_count + kCombineTile - 1) / kCombineTile;
        if (grid < 1) grid = 1;
        // co-resident (four 33 KB workgroups fit one compute unit's LDS):
        // look-back waits stay bounded
        if (grid > 4 * A->num_cu) grid = 4 * A->num_cu;
        HIP_TRY(launch_combine(ca, semiring, (int)grid, s));
    }
    if (h_nnz_y) {
        Ctrl h{};
        rc = read_ctrl(A, &h, s);
        if (rc) return rc;
        *h_nnz_y = h.nnz_y;
        if (h.err) {
            clear_err(A, s);
            return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err) +
                                            " (1 = x index range, 2 = duplicate x index, 4 = look-back bound, "
                                            "32 = mask or w index range, 64 = w not ascending)");
        }
        if (h.nnz_y > y_capacity) return fail(SPMSPV_ECAPACITY, "nnz(y) exceeds y_capacity");
    }
    return SPMSPV_OK;
}

int spmspv_run_static(int64_t m, int64_t n, int64_t nnz, const int32_t* colptr, const int32_t* rowids,
                      const float* values, int semiring, int flags, int64_t f, const int32_t* x_idx,
                      const void* x_val, int32_t* y_idx, void* y_val, int64_t y_capacity, int64_t* d_nnz_y,
                      int64_t* h_nnz_y, size_t* h_scratch_bytes, void* stream) {
    size_t need = 0;
    int rc = spmspv_workspace_size(m, n, nnz, 0, &need);
    if (rc) return rc;
    if (h_scratch_bytes) *h_scratch_bytes = need;
    if (need > kStaticScratchBytes)
        return fail(SPMSPV_EINVAL, "matrix needs " + std::to_string(need) + " bytes of scratch; the static scratch "
                                   "holds " + std::to_string(kStaticScratchBytes) + " (use spmspv_create)");
    if (!colptr || (nnz > 0 && !rowids)) return fail(SPMSPV_EINVAL, "NULL matrix");
    if (semiring < 0 || semiring > 2) return fail(SPMSPV_EINVAL, "unknown semiring");
    if (f < 0 || f > n) return fail(SPMSPV_EINVAL, "f must be in [0, n]");
    if (f > 0 && !x_idx) return fail(SPMSPV_EINVAL, "x_idx is NULL");
    if (y_capacity < 0 || (y_capacity > 0 && !y_idx)) return fail(SPMSPV_EINVAL, "bad y buffer");
    if (flags & ~(SPMSPV_SORTED_OUTPUT | SPMSPV_X_VAL_IS_INDEX | SPMSPV_X_ALL_TRUE))
        return fail(SPMSPV_EINVAL, "spmspv_run_static takes only SORTED_OUTPUT, X_VAL_IS_INDEX and X_ALL_TRUE");
    int xmode = XV_BITS32;
    if (semiring == SR_MIN_SELECT2ND && (flags & SPMSPV_X_VAL_IS_INDEX)) xmode = XV_INDEX;
    else if (semiring == SR_OR_AND) xmode = (flags & SPMSPV_X_ALL_TRUE) ? XV_TRUE : XV_U8;
    if (f > 0 && !x_val && (xmode == XV_BITS32 || xmode == XV_U8)) return fail(SPMSPV_EINVAL, "x_val is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    void* ws = nullptr;
    StaticDevice* info = nullptr;
    if ((rc = static_scratch(&dev, &ws, &info))) return rc;

    // A handle on the stack over the scratch (no allocation: its host
    // containers stay empty), set up as spmspv_create sets one up, without
    // the host read of the longest column (the bucketing grid is sized from
    // nnz instead).
    spmspv_matrix M;
    bind_workspace(&M, m, n, nnz, colptr, rowids, values, static_cast<char*>(ws), 0);
    M.device = dev;
    M.num_cu = info->num_cu;
    M.lds_max = info->lds_max;
    M.maxdeg = nnz > INT32_MAX ? INT32_MAX : (int32_t)nnz;
    default_schedule(&M, &M.sched);
    if ((rc = check_schedule(&M, &M.sched))) return fail(SPMSPV_EUNSUPPORTED, "matrix too tall for the LDS bucket layout");
    M.sched = sized_for_call(&M, f);
    const Layout& L = M.L;
    // The scratch keeps the previous call's contents: clear the control block,
    // counters and look-back words (a fill kernel, not a memset).
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(M.ws), 0u, int64_t(L.buckets / 4), s));
    HIP_TRY(launch_validate_colptr(colptr, (int32_t)n, nnz, M.ctrl, &M.ctrl->maxdeg, s));
    HIP_TRY(launch_row_counts(rowids, nnz, (int32_t)m, M.rcp, M.ctrl, s));
    HIP_TRY(launch_exclusive_scan_i32(M.rcp, m + 1, reinterpret_cast<int32_t*>(M.ws + L.partials), s));
    rc = enqueue(&M, semiring, xmode, f, nullptr, x_idx, x_val, y_idx, y_val, y_capacity, d_nnz_y, false, nullptr, s,
                 nullptr);
    if (rc) return rc;
    if (h_nnz_y) {
        Ctrl h{};
        if ((rc = read_ctrl(&M, &h, s))) return rc;
        *h_nnz_y = h.nnz_y;
        if (h.err & (ERR_CSC | ERR_ROW_RANGE)) return fail(SPMSPV_EINVAL, "invalid CSC (colptr or row ids)");
        if (h.err)
            return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err) +
                                            " (1 = x index range, 2 = duplicate x index, 4 = look-back bound)");
        if (h.nnz_y > y_capacity) return fail(SPMSPV_ECAPACITY, "nnz(y) exceeds y_capacity");
    }
    return SPMSPV_OK;
}

int bfs_run(spmspv_handle A, int semiring, int32_t root, int flags, int32_t* level, int32_t* parent,
            int32_t* h_num_levels, void* stream) {
    if (!A) return fail(SPMSPV_EINVAL, "NULL handle");
    if (A->m != A->n) return fail(SPMSPV_EINVAL, "BFS needs a square matrix");
    if (semiring != SR_MIN_SELECT2ND && semiring != SR_OR_AND)
        return fail(SPMSPV_EINVAL, "BFS semiring must be MIN_SELECT2ND_I32 or OR_AND_BOOL");
    if (semiring == SR_OR_AND && parent) return fail(SPMSPV_EINVAL, "OR_AND BFS has no parents");
    if (!level) return fail(SPMSPV_EINVAL, "level is NULL");
    if (root < 0 || root >= A->n) return fail(SPMSPV_EINVAL, "root out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int xmode = semiring == SR_MIN_SELECT2ND ? XV_INDEX : XV_TRUE;
    const bool selector = (flags & SPMSPV_USE_SELECTOR) != 0;
    // With a captured level graph and a row form, the selector's decision is
    // consumed on the device: it sets the level's direction and the gated
    // push / pull kernels follow it (the push tile stays the handle's).
    const bool learned_gate = selector && (flags & SPMSPV_USE_GRAPH) && A->pull && A->forced_classes.empty();
    const bool diropt = (flags & SPMSPV_DIRECTION_OPT) != 0 || learned_gate;
    if (selector && !A->selector_loaded && A->forced_classes.empty())
        return fail(SPMSPV_EINVAL, "no selector weights loaded");
    if (diropt && !A->pull)
        return fail(SPMSPV_EUNSUPPORTED, "SPMSPV_DIRECTION_OPT needs SPMSPV_WITH_TRANSPOSE or SPMSPV_SYMMETRIC");
    if (A->dcsc && (flags & (SPMSPV_PERSISTENT | SPMSPV_USE_SELECTOR)))
        return fail(SPMSPV_EUNSUPPORTED, "a DCSC handle runs BFS with the bucketing levels only");


    auto enqueue_levels = [&](int count, hipStream_t st) -> int {
        for (int l = 0; l < count; ++l) {
            int32_t* x = A->front[l & 1];
            int32_t* y = A->front[(l + 1) & 1];
            int rc = enqueue(A, semiring, xmode, 0, &A->ctrl->f, x, nullptr, y, nullptr, A->m, nullptr, true,
                             A->visited, st, nullptr, diropt, -1, 3, 0, learned_gate);
            if (rc) return rc;
            if (diropt) {
                // pull kernels for the same level; they run only when k_decide chose pull
                rc = enqueue_pull(A, semiring, xmode, 0, &A->ctrl->f, x, nullptr, y, nullptr, A->m, nullptr, true,
                                  A->visited, false, true, st, nullptr);
                if (rc) return rc;
            }
        }
        return SPMSPV_OK;
    };

    if (selector && !learned_gate) {
        // One host read per level: scan, device-side inference, chosen path.
        HIP_TRY(launch_bfs_init((int32_t)A->n, root, level, parent, A->visited, A->p_xbits, A->front[0], A->ctrl,
                                A->nnz, 0, s));
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(&A->ctrl->bfs_mode), 1u, 1, s));
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(&A->ctrl->seen), 0u, 2, s));
        A->level_classes.clear();
        for (int64_t l = 0;; ++l) {
            if (l > A->n + 1) return fail(SPMSPV_EDEVICE, "BFS did not terminate");
            int cls = 0;
            int32_t fnow = 0;
            const int forced = l < (int64_t)A->forced_classes.size() ? A->forced_classes[(size_t)l] : -1;
            const int rc = run_selected(A, semiring, xmode, 0, &A->ctrl->f, A->front[l & 1], nullptr,
                                        A->front[(l + 1) & 1], nullptr, A->m, nullptr, true, A->visited, s, &cls,
                                        &fnow, forced);
            if (rc) return rc;
            if (fnow == 0) break;
            A->level_classes.push_back(cls);
        }
        Ctrl h{};
        int rc = read_ctrl(A, &h, s);
        if (rc) return rc;
        if (h.err) {
            clear_err(A, s);
            return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err));
        }
        if (h_num_levels) *h_num_levels = h.level;
        return SPMSPV_OK;
    }
    const bool use_graph = (flags & SPMSPV_USE_GRAPH) != 0;
    if (use_graph && A->pull) {
        const int rc = set_ydense_ident(A, semiring, s);
        if (rc) return rc;
    }
    const int key = semiring + 1 + (diropt ? 8 : 0) + (learned_gate ? 16 : 0);
    if (use_graph && (A->graph == nullptr || A->graph_key != key)) {
        if (A->graph) {
            (void)hipGraphExecDestroy(A->graph);
            A->graph = nullptr;
        }
        // Capture on a private stream (the caller's may be the null stream,
        // which cannot be captured); the graph is then launched on `s`.
        if (!A->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&A->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(A->cap_stream, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_levels(kGraphLevels, A->cap_stream);
        hipError_t e = hipStreamEndCapture(A->cap_stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&A->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            A->graph = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        A->graph_key = key;
    }
    HIP_TRY(launch_bfs_init((int32_t)A->n, root, level, parent, A->visited, A->p_xbits, A->front[0], A->ctrl, A->nnz,
                            diropt ? 1 : 0, s));
    // Small frontiers of a low-degree graph run in the persistent kernel;
    // larger ones in batches of the bucketing levels below.
    bool persist = (flags & SPMSPV_PERSISTENT) && !diropt && A->maxdeg <= kPersistMaxDeg;
    if (persist && A->persist_grid < 0) A->persist_grid = persistent_grid(A->num_cu);
    persist = persist && A->persist_grid > 0;
    PersistArgs pa{};
    if (persist) {
        pa.ctrl = A->ctrl;
        pa.colptr = A->colptr;
        pa.rowids = A->rowids;
        pa.n = (int32_t)A->m;
        pa.front[0] = A->front[0];
        pa.front[1] = A->front[1];
        pa.front[2] = A->front2;
        pa.visited = A->visited;
        for (int k = 0; k < 3; ++k) pa.disc[k] = A->disc + k * ((A->m + 31) / 32);
        pa.pmin = A->pmin;
        pa.bar = A->bar;
    }
    if (learned_gate) {
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(&A->ctrl->bfs_mode), 1u, 1, s));
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(&A->ctrl->seen), 0u, 2, s));
    }
    // Level loop: kGraphLevels levels per batch, then one host check of the
    // frontier length.  Levels after the frontier empties are no-ops.
    // Each host check reads the whole control block, so the last one also
    // gives the level count and error bits.
    Ctrl h{};
    h.f = 1;
    for (int64_t batch = 0; h.f > 0; ++batch) {
        if (batch * kGraphLevels > A->n + kGraphLevels) return fail(SPMSPV_EDEVICE, "BFS did not terminate");
        if (persist) {
            HIP_TRY(launch_fill_u32(A->bar, 0u, 160, s));   // arrivals, append counters, barrier count
            HIP_TRY(launch_bfs_persistent(pa, semiring == SR_MIN_SELECT2ND, A->persist_grid, s));
            const int rc = read_ctrl(A, &h, s);
            if (rc) return rc;
            if (h.f == 0) break;
        }
        if (use_graph) HIP_TRY(hipGraphLaunch(A->graph, s));
        else {
            const int rc = enqueue_levels(kGraphLevels, s);
            if (rc) return rc;
        }
        const int rc = read_ctrl(A, &h, s);
        if (rc) return rc;
    }
    if (h.err) {
        clear_err(A, s);
        return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err));
    }
    if (h_num_levels) *h_num_levels = h.level;
    return SPMSPV_OK;
}

int spmspv_last_stats(spmspv_handle A, int64_t* h_out, void* stream) {
    if (!A || !h_out) return fail(SPMSPV_EINVAL, "NULL argument");
    Ctrl h{};
    const int rc = read_ctrl(A, &h, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    h_out[0] = h.W_last;
    h_out[1] = h.nnz_y;
    h_out[2] = h.fnz_last;
    h_out[3] = h.maxlen_last;
    h_out[4] = h.err;
    h_out[5] = h.cls;
    return SPMSPV_OK;
}

int spmspv_selector_load(spmspv_handle A, const float* h_params, const float* h_mean, const float* h_std,
                         void* stream) {
    if (!A || !h_params || !h_mean || !h_std) return fail(SPMSPV_EINVAL, "NULL argument");
    std::vector<float> buf((size_t)kMlpParams + 2 * kMlpIn);
    for (int q = 0; q < kMlpParams; ++q) {
        if (!(h_params[q] == h_params[q]) || h_params[q] > 1e30f || h_params[q] < -1e30f) {
            A->selector_loaded = false;
            return fail(SPMSPV_EINVAL, "selector weights are not finite; selector disabled");
        }
        buf[(size_t)q] = h_params[q];
    }
    for (int c = 0; c < kMlpIn; ++c) {
        if (!(h_std[c] > 0.f)) {
            A->selector_loaded = false;
            return fail(SPMSPV_EINVAL, "feature std must be positive; selector disabled");
        }
        buf[(size_t)kMlpParams + c] = h_mean[c];
        buf[(size_t)kMlpParams + kMlpIn + c] = h_std[c];
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(A->selector, buf.data(), buf.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    A->selector_loaded = true;
    return SPMSPV_OK;
}

int spmspv_selector_classes(spmspv_handle A, int32_t* h_out, int32_t cap, int32_t* h_count) {
    if (!A || !h_count) return fail(SPMSPV_EINVAL, "NULL argument");
    *h_count = (int32_t)A->level_classes.size();
    for (int32_t k = 0; k < cap && k < *h_count; ++k) h_out[k] = A->level_classes[(size_t)k];
    return SPMSPV_OK;
}

int spmspv_force_classes(spmspv_handle A, const int32_t* h_classes, int32_t count) {
    if (!A || count < 0 || (count > 0 && !h_classes)) return fail(SPMSPV_EINVAL, "bad argument");
    for (int32_t k = 0; k < count; ++k)
        if (h_classes[k] < 0 || h_classes[k] > 9) return fail(SPMSPV_EINVAL, "classes must be in [0, 9]");
    A->forced_classes.assign(h_classes, h_classes + count);
    return SPMSPV_OK;
}

int spmspv_selector_features(spmspv_handle A, float* h_out, void* stream) {
    if (!A || !h_out) return fail(SPMSPV_EINVAL, "NULL argument");
    Ctrl h{};
    const int rc = read_ctrl(A, &h, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    for (int c = 0; c < kMlpIn; ++c) h_out[c] = h.features[c];
    return SPMSPV_OK;
}

int spmspv_class_schedule(spmspv_handle A, int semiring, int cls, spmspv_schedule* h_sched) {
    if (!A || !h_sched) return fail(SPMSPV_EINVAL, "NULL argument");
    if (cls < 0 || cls > 9) return fail(SPMSPV_EINVAL, "class must be in [0, 9]");
    if (semiring < 0 || semiring > 2) return fail(SPMSPV_EINVAL, "unknown semiring");
    spmspv_schedule e = A->sched;
    if (cls == 9) {
        if (!A->pull) return fail(SPMSPV_EUNSUPPORTED, "pull needs a handle with a row form");
        e.direction = 1;
    } else {
        e.direction = 0;
        e.merge_variant = 0;
        e.tile_log2 = call_tile(A, class_tile(A, cls), semiring);
    }
    e.launch = 1;
    *h_sched = e;
    return SPMSPV_OK;
}

int spmspv_class_tile(spmspv_handle A, int cls, int32_t* h_tile_log2) {
    if (!A || !h_tile_log2 || cls < 0 || cls > 9) return fail(SPMSPV_EINVAL, "bad argument");
    *h_tile_log2 = cls == 9 ? -1 : class_tile(A, cls);
    return SPMSPV_OK;
}

int spmspv_batch_workspace_size(spmspv_handle A, int max_batch, int64_t max_f, int64_t max_products, int flags,
                                size_t* h_bytes) {
    if (!A || !h_bytes) return fail(SPMSPV_EINVAL, "NULL argument");
    if (max_batch < 1 || max_batch > kMaxBatch) return fail(SPMSPV_EINVAL, "max_batch must be in [1, 1024]");
    const bool bfs = (flags & SPMSPV_MSBFS) != 0;
    if (bfs && A->m != A->n) return fail(SPMSPV_EINVAL, "multi-source BFS needs a square matrix");
    if (bfs && (int64_t)max_batch * A->n >= INT32_MAX)
        return fail(SPMSPV_EUNSUPPORTED, "max_batch * n must stay below 2^31");
    if (!bfs && (max_f < 0 || max_f >= INT32_MAX || max_products < 0))
        return fail(SPMSPV_EINVAL, "max_f must be in [0, 2^31) and max_products >= 0");
    *h_bytes = make_batch_layout(A->m, A->n, A->nnz, max_batch, max_f, max_products, bfs).total;
    return SPMSPV_OK;
}

int spmspv_batch_attach(spmspv_handle A, int max_batch, int64_t max_f, int64_t max_products, int flags,
                        void* workspace, size_t ws_bytes, void* stream) {
    size_t need = 0;
    const int rc = spmspv_batch_workspace_size(A, max_batch, max_f, max_products, flags, &need);
    if (rc) return rc;
    if (!workspace) return fail(SPMSPV_EINVAL, "NULL workspace");
    if (ws_bytes < need) return fail(SPMSPV_ENOMEM, "batch workspace needs " + std::to_string(need) + " bytes");
    const bool bfs = (flags & SPMSPV_MSBFS) != 0;
    A->batch.bound = true;
    A->batch.bfs = bfs;
    A->batch.max_batch = max_batch;
    A->batch.L = make_batch_layout(A->m, A->n, A->nnz, max_batch, max_f, max_products, bfs);
    A->batch.ws = static_cast<char*>(workspace);
    A->batch.ms_long_ready = false;
    // The first scan looks back over these words; later calls clear them in
    // their first bucketing pass.  (The counters and merge look-back words
    // are cleared by every scan.)
    const hipError_t e = launch_clear_u64(reinterpret_cast<uint64_t*>(A->batch.ws + A->batch.L.lb1),
                                          (int)A->batch.L.lb1_n * 2, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        A->batch.bound = false;
        return hip_fail(e, "clear batch look-back words");
    }
    return SPMSPV_OK;
}

int spmspv_set_batch_schedule(spmspv_handle A, const spmspv_schedule* h_sched) {
    if (!A) return fail(SPMSPV_EINVAL, "NULL handle");
    if (!h_sched) {
        A->batch_sched = spmspv_schedule{};
        return SPMSPV_OK;
    }
    const int rc = check_schedule(A, h_sched);
    if (rc) return rc;
    if (h_sched->direction != 0) return fail(SPMSPV_EINVAL, "batched calls run the push direction");
    A->batch_sched = *h_sched;
    return SPMSPV_OK;
}

int spmspv_get_batch_schedule(spmspv_handle A, int semiring, int nbatch, spmspv_schedule* h_sched) {
    if (!A || !h_sched) return fail(SPMSPV_EINVAL, "NULL argument");
    if (semiring < 0 || semiring > 2) return fail(SPMSPV_EINVAL, "unknown semiring");
    if (nbatch < 1 || nbatch > kMaxBatch) return fail(SPMSPV_EINVAL, "nbatch must be in [1, 1024]");
    return batch_shape(A, nbatch, semiring, h_sched);
}

namespace {
int batch_status(spmspv_matrix* A, hipStream_t s, int64_t* total) {
    Ctrl h{};
    int rc = read_ctrl(A, &h, s);
    if (rc) return rc;
    if (h.err) {
        clear_err(A, s);
        if (h.err & ERR_X_RANGE) return fail(SPMSPV_EINVAL, "x index or vector offset out of range");
        if ((h.err & ERR_BUCKET_OVERFLOW) && A->batch.fixed_last)
            return fail(SPMSPV_EDEVICE, "a bucket slice overflowed: repeated x index within a vector");
        if (h.err & ERR_BUCKET_OVERFLOW)
            return fail(SPMSPV_ECAPACITY, "products exceed the batch workspace's max_products");
        return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err));
    }
    if (total) *total = h.nnz_y;
    return SPMSPV_OK;
}
}  // namespace

int spmspv_run_batch(spmspv_handle A, int semiring, int flags, int nbatch, const int64_t* x_off,
                     const int32_t* x_idx, const void* x_val, int64_t* y_off, int32_t* y_idx, void* y_val,
                     int64_t y_capacity, int64_t* h_nnz_total, void* stream) {
    if (!A) return fail(SPMSPV_EINVAL, "NULL handle");
    if (!A->batch.bound) return fail(SPMSPV_EINVAL, "no batch workspace attached (spmspv_batch_attach)");
    if (nbatch < 1 || nbatch > A->batch.max_batch) return fail(SPMSPV_EINVAL, "nbatch out of range");
    if (semiring < 0 || semiring > 2) return fail(SPMSPV_EINVAL, "unknown semiring");
    if (!x_off || !y_off || !y_idx || y_capacity < 0) return fail(SPMSPV_EINVAL, "NULL or negative argument");
    int xmode = XV_BITS32;
    if (semiring == SR_MIN_SELECT2ND && (flags & SPMSPV_X_VAL_IS_INDEX)) xmode = XV_INDEX;
    else if (semiring == SR_OR_AND) xmode = (flags & SPMSPV_X_ALL_TRUE) ? XV_TRUE : XV_U8;
    if (xmode != XV_INDEX && xmode != XV_TRUE && !x_val) return fail(SPMSPV_EINVAL, "x_val is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & SPMSPV_VALIDATE) {
        std::vector<int64_t> off((size_t)nbatch + 1);
        HIP_TRY(hipMemcpyAsync(off.data(), x_off, off.size() * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (off[0] != 0) return fail(SPMSPV_EINVAL, "x_off[0] must be 0");
        for (int b = 0; b < nbatch; ++b)
            if (off[(size_t)b + 1] < off[(size_t)b]) return fail(SPMSPV_EINVAL, "x_off must be non-decreasing");
        if (off[(size_t)nbatch] > A->batch.L.max_f) return fail(SPMSPV_EINVAL, "total x length exceeds max_f");
        std::vector<int32_t> xi((size_t)off[(size_t)nbatch]);
        if (!xi.empty()) {
            if (!x_idx) return fail(SPMSPV_EINVAL, "x_idx is NULL");
            HIP_TRY(hipMemcpyAsync(xi.data(), x_idx, xi.size() * 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        std::vector<int32_t> stamp((size_t)A->n, -1);
        for (int b = 0; b < nbatch; ++b)
            for (int64_t p = off[(size_t)b]; p < off[(size_t)b + 1]; ++p) {
                const int32_t j = xi[(size_t)p];
                if (j < 0 || j >= A->n) return fail(SPMSPV_EINVAL, "x index out of range");
                if (stamp[(size_t)j] == b) return fail(SPMSPV_EINVAL, "duplicate x index within a vector");
                stamp[(size_t)j] = b;
            }
    }
    const int rc = enqueue_batch(A, semiring, xmode, nbatch, x_off, x_idx, x_val, y_off, y_idx, y_val, y_capacity,
                                 false, s);
    if (rc) return rc;
    if (h_nnz_total) {
        int64_t total = 0;
        const int st = batch_status(A, s, &total);
        if (st) return st;
        *h_nnz_total = total;
        if (total > y_capacity)
            return fail(SPMSPV_ECAPACITY, "nnz(y) total " + std::to_string(total) + " exceeds y_capacity");
    }
    return SPMSPV_OK;
}

// Multi-source BFS with the direction chosen per level for all sources
// together, by the frontier-edge rule summed over the sources: push (the
// batched SpMSpV) while the frontiers' column lengths m_f stay below the
// sources' unexplored edges m_u / alpha, then pull levels on one-bit-per-
// source masks until every frontier is empty.  The searches stay pull once
// switched: late levels cost one read of the seen masks, less than the
// batched push launches.  One host read per level (the switch test, the
// frontier total); the state starts as k_msbfs_init left it.
int msbfs_diropt(spmspv_matrix* A, int semiring, int nsrc, int32_t* level, int32_t* parent, int32_t* h_num_levels,
                 hipStream_t s) {
    BatchCtx& B = A->batch;
    const BatchLayout& L = B.L;
    int32_t* front[2] = {reinterpret_cast<int32_t*>(B.ws + L.front0), reinterpret_cast<int32_t*>(B.ws + L.front1)};
    int64_t* xoff[2] = {reinterpret_cast<int64_t*>(B.ws + L.xoff0), reinterpret_cast<int64_t*>(B.ws + L.xoff1)};
    uint64_t* fm[2] = {reinterpret_cast<uint64_t*>(B.ws + L.ms_f0), reinterpret_cast<uint64_t*>(B.ws + L.ms_f1)};
    int32_t* long_count = reinterpret_cast<int32_t*>(B.ws + L.ms_cnt);
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(B.ws + L.ms_cnt + 16);
    const int xmode = semiring == SR_MIN_SELECT2ND ? XV_INDEX : XV_TRUE;
    const int G = (nsrc + 63) / 64;
    const double alpha = 14.0;
    if (!B.ms_long_ready) {
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(long_count), 0u, 1, s));
        HIP_TRY(launch_ms_long_rows(A->rowptr, (int32_t)A->n, reinterpret_cast<int32_t*>(B.ws + L.ms_long),
                                    long_count, s));
        B.ms_long_ready = true;
    }
    // push levels while the frontier-edge rule says so
    double m_u = (double)nsrc * (double)A->nnz;
    int32_t hf = nsrc;
    int64_t lv = 0;   // the current frontier's position in the level sequence
    bool pull = false;
    for (;;) {
        if (lv > A->n + 1) return fail(SPMSPV_EDEVICE, "BFS did not terminate");
        HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(counter), 0ull, 1, s));
        HIP_TRY(launch_ms_degsum(front[lv & 1], xoff[lv & 1], nsrc, A->colptr, (int32_t)A->n, counter, s));
        unsigned long long mf = 0;
        HIP_TRY(hipMemcpyAsync(&mf, counter, sizeof(mf), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&hf, &A->ctrl->f, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hf <= 0) break;
        m_u -= (double)mf;
        if ((double)mf * alpha > m_u) {
            pull = true;
            break;
        }
        const int rc = enqueue_batch(A, semiring, xmode, nsrc, xoff[lv & 1], front[lv & 1], nullptr,
                                     xoff[(lv + 1) & 1], front[(lv + 1) & 1], nullptr, L.max_f, true, s);
        if (rc) return rc;
        ++lv;
    }
    Ctrl h{};
    int rc = read_ctrl(A, &h, s);
    if (rc) return rc;
    int32_t levels = h.level;
    if (pull && hf > 0) {
        // level of the current frontier: the scans have counted the push levels
        int32_t cur = h.level;
        MsArgs ma{};
        ma.n = (int32_t)A->n;
        ma.G = G;
        ma.nsrc = nsrc;
        ma.rowptr = A->rowptr;
        ma.colids = A->colids;
        ma.level = level;
        ma.parent = semiring == SR_MIN_SELECT2ND ? parent : nullptr;
        ma.long_rows = reinterpret_cast<const int32_t*>(B.ws + L.ms_long);
        ma.long_count = long_count;
        ma.found_total = counter;
        ma.seen = reinterpret_cast<uint64_t*>(B.ws + L.ms_seen);
        int cf = 0;
        ma.fcur = fm[cf];
        HIP_TRY(launch_fill_u64(fm[cf], 0ull, A->n * G, s));
        HIP_TRY(launch_ms_to_pull(ma, reinterpret_cast<const uint32_t*>(B.ws + L.visited), L.mask_words, front[lv & 1],
                                  xoff[lv & 1], fm[cf], s));
        for (int64_t step = 0;; ++step) {
            if (step > A->n + 1) return fail(SPMSPV_EDEVICE, "BFS did not terminate");
            ma.fcur = fm[cf];
            ma.fnext = fm[cf ^ 1];
            ma.lvl = cur + 1;
            HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(counter), 0ull, 1, s));
            HIP_TRY(launch_ms_pull(ma, ma.parent != nullptr, A->num_cu, s));
            unsigned long long found = 0;
            HIP_TRY(hipMemcpyAsync(&found, counter, sizeof(found), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            ++cur;   // the frontier was not empty
            if (found == 0) break;
            cf ^= 1;
        }
        levels = cur;
    }
    if (h.err) {
        clear_err(A, s);
        if (h.err & ERR_BUCKET_OVERFLOW)
            return fail(SPMSPV_ECAPACITY, "a level's products exceed the batch workspace's max_products");
        return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err));
    }
    if (h_num_levels) *h_num_levels = levels;
    return SPMSPV_OK;
}

int msbfs_run(spmspv_handle A, int semiring, int nsrc, const int32_t* h_roots, int flags, int32_t* level,
              int32_t* parent, int32_t* h_num_levels, void* stream) {
    if (!A) return fail(SPMSPV_EINVAL, "NULL handle");
    if (!A->batch.bound || !A->batch.bfs)
        return fail(SPMSPV_EINVAL, "no batch workspace attached with SPMSPV_MSBFS");
    if (A->m != A->n) return fail(SPMSPV_EINVAL, "BFS needs a square matrix");
    if (semiring != SR_MIN_SELECT2ND && semiring != SR_OR_AND)
        return fail(SPMSPV_EINVAL, "BFS semiring must be MIN_SELECT2ND_I32 or OR_AND_BOOL");
    if (semiring == SR_OR_AND && parent) return fail(SPMSPV_EINVAL, "OR_AND BFS has no parents");
    if (nsrc < 1 || nsrc > A->batch.max_batch) return fail(SPMSPV_EINVAL, "nsrc out of range");
    if (!h_roots || !level) return fail(SPMSPV_EINVAL, "NULL argument");
    for (int x = 0; x < nsrc; ++x)
        if (h_roots[x] < 0 || h_roots[x] >= A->n) return fail(SPMSPV_EINVAL, "root out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    BatchCtx& B = A->batch;
    const BatchLayout& L = B.L;
    spmspv_schedule sc{};
    int rc = batch_shape(A, nsrc, semiring, &sc);
    if (rc) return rc;
    int32_t* roots = reinterpret_cast<int32_t*>(B.ws + L.roots);
    int32_t* front[2] = {reinterpret_cast<int32_t*>(B.ws + L.front0), reinterpret_cast<int32_t*>(B.ws + L.front1)};
    int64_t* xoff[2] = {reinterpret_cast<int64_t*>(B.ws + L.xoff0), reinterpret_cast<int64_t*>(B.ws + L.xoff1)};
    HIP_TRY(hipMemcpyAsync(roots, h_roots, size_t(nsrc) * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_msbfs_init((int32_t)A->n, nsrc, roots, level, parent, reinterpret_cast<uint32_t*>(B.ws + L.visited),
                              L.mask_words, front[0], xoff[0], A->ctrl, s));
    const int xmode = semiring == SR_MIN_SELECT2ND ? XV_INDEX : XV_TRUE;
    // Direction switching needs the row form, and for parents ascending rows
    // (the first frontier in-neighbour found is then the smallest).
    if ((flags & SPMSPV_DIRECTION_OPT) && A->pull && (semiring == SR_OR_AND || A->rows_sorted))
        return msbfs_diropt(A, semiring, nsrc, level, parent, h_num_levels, s);
    // Levels are enqueued kGraphLevels at a time; levels after the frontiers
    // empty are no-ops.  One host check of the total frontier per batch.
    int32_t hf = nsrc;
    for (int64_t l = 0; hf > 0; l += kGraphLevels) {
        if (l > A->n + kGraphLevels) return fail(SPMSPV_EDEVICE, "BFS did not terminate");
        for (int k = 0; k < kGraphLevels; ++k) {
            const int64_t lv = l + k;
            rc = enqueue_batch(A, semiring, xmode, nsrc, xoff[lv & 1], front[lv & 1], nullptr, xoff[(lv + 1) & 1],
                               front[(lv + 1) & 1], nullptr, L.max_f, true, s);
            if (rc) return rc;
        }
        HIP_TRY(hipMemcpyAsync(&hf, &A->ctrl->f, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    Ctrl h{};
    rc = read_ctrl(A, &h, s);
    if (rc) return rc;
    if (h.err) {
        clear_err(A, s);
        if (h.err & ERR_BUCKET_OVERFLOW)
            return fail(SPMSPV_ECAPACITY, "a level's products exceed the batch workspace's max_products");
        return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err));
    }
    if (h_num_levels) *h_num_levels = h.level;
    return SPMSPV_OK;
}

int spmspv_autotune(spmspv_handle A, int semiring, const double* h_densities, int ndens, int reps, int32_t* x_idx,
                    void* x_val, int32_t* y_idx, void* y_val, spmspv_tune_entry* h_out, void* stream) {
    if (!A || !h_densities || ndens < 1 || ndens > 64 || reps < 1 || !x_idx || !y_idx || !y_val)
        return fail(SPMSPV_EINVAL, "bad argument");
    if (semiring < 0 || semiring > 2) return fail(SPMSPV_EINVAL, "unknown semiring");
    if (semiring == SR_PLUS_TIMES && !x_val) return fail(SPMSPV_EINVAL, "plus-times tuning needs x_val");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int xmode = semiring == SR_PLUS_TIMES ? XV_BITS32 : (semiring == SR_MIN_SELECT2ND ? XV_INDEX : XV_TRUE);
    spmspv_schedule dflt{};
    default_schedule(A, &dflt);
    std::vector<spmspv_tune_entry> table;
    for (int d = 0; d < ndens; ++d) {
        const double dens = h_densities[d];
        if (!(dens > 0.0 && dens <= 1.0)) return fail(SPMSPV_EINVAL, "densities must be in (0, 1]");
        HIP_TRY(launch_gen_x((int32_t)A->n, dens, 0x5eed0000ull + (uint64_t)d, x_idx,
                             semiring == SR_PLUS_TIMES ? static_cast<float*>(x_val) : nullptr, A->ctrl, s));
        Ctrl h{};
        int rc = read_ctrl(A, &h, s);
        if (rc) return rc;
        const int64_t f = h.gen_count;
        const void* xv = semiring == SR_PLUS_TIMES ? x_val : nullptr;
        auto cost = [&](const spmspv_schedule& sc, double* us) {
            return time_schedule(A, sc, semiring, xmode, f, x_idx, xv, y_idx, y_val, reps, s, us);
        };
        spmspv_tune_entry e{};
        e.density = dens;
        e.f = f;
        rc = cost(dflt, &e.default_us);
        if (rc) return rc;
        spmspv_schedule best = dflt;
        double best_us = e.default_us;
        auto consider = [&](spmspv_schedule c) -> int {
            if (check_schedule(A, &c) != SPMSPV_OK) {
                g_last_error.clear();
                return SPMSPV_OK;
            }
            double us = 0;
            const int r = cost(c, &us);
            if (r) return r;
            if (us < best_us) {
                best_us = us;
                best = c;
            }
            return SPMSPV_OK;
        };
        // Coordinate descent over the push schedule, twice, then the pull direction.
        const int shapes[7][2] = {{256, 4}, {256, 8}, {256, 16}, {512, 4}, {512, 8}, {1024, 4}, {1024, 8}};
        const int merges[3] = {256, 512, 1024};
        for (int pass = 0; pass < 2; ++pass) {
            for (int tl = kTileLog2Min; tl <= kTileLog2Max; ++tl) {
                spmspv_schedule c = best;
                c.direction = 0;
                c.tile_log2 = tl;
                c.merge_variant = 0;
                if ((rc = consider(c))) return rc;
            }
            for (const auto& sh : shapes) {
                spmspv_schedule c = best;
                c.direction = 0;
                c.scatter_block = sh[0];
                c.scatter_items = sh[1];
                if ((rc = consider(c))) return rc;
            }
            for (int mb : merges) {
                spmspv_schedule c = best;
                c.direction = 0;
                c.merge_block = mb;
                if ((rc = consider(c))) return rc;
            }
        }
        // wide buckets through the HBM accumulator (16 to 1024 buckets)
        for (int tl = std::max(kTileLog2Max + 1, ceil_log2(A->m) - 10); tl <= ceil_log2(A->m) - 4; ++tl) {
            spmspv_schedule c = best;
            c.direction = 0;
            c.tile_log2 = tl;
            c.merge_variant = 1;
            if ((rc = consider(c))) return rc;
        }
        if (A->pull) {
            spmspv_schedule c = best;
            c.direction = 1;
            if ((rc = consider(c))) return rc;
        }
        e.sched = best;
        e.us = best_us;
        table.push_back(e);
        if (h_out) h_out[d] = e;
    }
    A->tuned = table;
    return SPMSPV_OK;
}

// ---- persisted tuning tables
#ifndef SPMSPV_SOURCE_DIGEST
#define SPMSPV_SOURCE_DIGEST "unknown"
#endif

const char* spmspv_source_digest(void) { return SPMSPV_SOURCE_DIGEST; }

extern "C++" {
namespace {

constexpr int kTuningVersion = 1;
constexpr int kSignatureSamples = 4096;

std::string device_key(const spmspv_matrix* A) {
    hipDeviceProp_t p{};
    if (hipGetDeviceProperties(&p, A->device) != hipSuccess) return "unknown";
    std::string name(p.name);
    for (char& c : name)
        if (c == '\n' || c == '\r') c = ' ';
    return name + "|" + p.gcnArchName + "|" + std::to_string(p.multiProcessorCount);
}

// FNV-1a over m, n, nnz and evenly spaced samples of colptr and rowids.
int graph_signature(spmspv_matrix* A, hipStream_t s, uint64_t* out) {
    const int K = kSignatureSamples;
    // the batch of samples goes through the handle's list scratch (max(m, n) entries)
    const int Kc = (int)std::min<int64_t>(K, std::max<int64_t>(2, std::max(A->m, A->n) / 2));
    int32_t* d = A->bv_idx;
    std::vector<int32_t> h(2 * (size_t)Kc);
    const int64_t ncol = (A->dcsc ? A->nzc : A->n) + 1;
    HIP_TRY(launch_sample_i32(A->colptr, ncol, d, Kc, s));
    HIP_TRY(launch_sample_i32(A->rowids, A->nnz, d + Kc, Kc, s));
    HIP_TRY(hipMemcpyAsync(h.data(), d, h.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            x ^= (v >> (8 * b)) & 0xffu;
            x *= 1099511628211ull;
        }
    };
    mix((uint64_t)A->m);
    mix((uint64_t)A->n);
    mix((uint64_t)A->nnz);
    mix(A->dcsc ? 1u : 0u);
    for (int32_t v : h) mix((uint32_t)v);
    *out = x;
    return SPMSPV_OK;
}

}  // namespace
}  // extern "C++"

int spmspv_tuning_save(spmspv_handle A, const char* path, void* stream) {
    if (!A || !path) return fail(SPMSPV_EINVAL, "NULL argument");
    if (A->tuned.empty()) return fail(SPMSPV_EINVAL, "the handle has not been autotuned");
    uint64_t sig = 0;
    const int rc = graph_signature(A, static_cast<hipStream_t>(stream), &sig);
    if (rc) return rc;
    std::ofstream f(path);
    if (!f) return fail(SPMSPV_EINVAL, std::string("cannot write ") + path);
    char hex[24];
    snprintf(hex, sizeof(hex), "%016llx", (unsigned long long)sig);
    f << "spmspv-tuning " << kTuningVersion << "\n";
    f << "device " << device_key(A) << "\n";
    f << "library " << SPMSPV_SOURCE_DIGEST << "\n";
    f << "graph " << A->m << " " << A->n << " " << A->nnz << " " << hex << "\n";
    f << "entries " << A->tuned.size() << "\n";
    f.precision(17);
    for (const auto& e : A->tuned) {
        const spmspv_schedule& c = e.sched;
        f << e.density << " " << c.direction << " " << c.tile_log2 << " " << c.scatter_block << " "
          << c.scatter_items << " " << c.merge_block << " " << c.merge_variant << " " << c.launch << " " << e.us
          << " " << e.default_us << "\n";
    }
    f.flush();
    if (!f) return fail(SPMSPV_EINVAL, std::string("write failed: ") + path);
    return SPMSPV_OK;
}

int spmspv_tuning_load(spmspv_handle A, const char* path, void* stream) {
    if (!A || !path) return fail(SPMSPV_EINVAL, "NULL argument");
    std::ifstream f(path);
    if (!f) return fail(SPMSPV_EINVAL, std::string("cannot read ") + path);
    std::string line, word;
    auto next = [&](const char* key, std::string* rest) -> bool {
        if (!std::getline(f, line)) return false;
        const std::string k(key);
        if (line.compare(0, k.size() + 1, k + " ") != 0) return false;
        *rest = line.substr(k.size() + 1);
        return true;
    };
    std::string v, dev, lib, graph, count;
    if (!next("spmspv-tuning", &v) || std::atoi(v.c_str()) != kTuningVersion)
        return fail(SPMSPV_EINVAL, "not a tuning table of version " + std::to_string(kTuningVersion));
    if (!next("device", &dev) || !next("library", &lib) || !next("graph", &graph) || !next("entries", &count))
        return fail(SPMSPV_EINVAL, "malformed tuning table header");
    if (dev != device_key(A)) return fail(SPMSPV_EUNSUPPORTED, "tuning table is for another device: " + dev);
    if (lib != SPMSPV_SOURCE_DIGEST)
        return fail(SPMSPV_EUNSUPPORTED, "tuning table was measured on other kernels (" + lib + ")");
    uint64_t sig = 0;
    int rc = graph_signature(A, static_cast<hipStream_t>(stream), &sig);
    if (rc) return rc;
    {
        std::istringstream g(graph);
        long long m = -1, n = -1, nnz = -1;
        std::string hex;
        g >> m >> n >> nnz >> hex;
        if (m != A->m || n != A->n || nnz != A->nnz || std::strtoull(hex.c_str(), nullptr, 16) != sig)
            return fail(SPMSPV_EUNSUPPORTED, "tuning table is for another matrix");
    }
    const int k = std::atoi(count.c_str());
    if (k < 1 || k > 64) return fail(SPMSPV_EINVAL, "bad entry count in tuning table");
    std::vector<spmspv_tune_entry> table;
    for (int i = 0; i < k; ++i) {
        if (!std::getline(f, line)) return fail(SPMSPV_EINVAL, "truncated tuning table");
        std::istringstream r(line);
        spmspv_tune_entry e{};
        spmspv_schedule& c = e.sched;
        if (!(r >> e.density >> c.direction >> c.tile_log2 >> c.scatter_block >> c.scatter_items >> c.merge_block >>
              c.merge_variant >> c.launch >> e.us >> e.default_us))
            return fail(SPMSPV_EINVAL, "malformed tuning table entry");
        if (!(e.density > 0.0 && e.density <= 1.0)) return fail(SPMSPV_EINVAL, "bad density in tuning table");
        if ((rc = check_schedule(A, &c))) return rc;
        table.push_back(e);
    }
    A->tuned = table;
    return SPMSPV_OK;
}

int spmspv_tuned_schedule(spmspv_handle A, int64_t f, spmspv_schedule* h_sched) {
    if (!A || !h_sched) return fail(SPMSPV_EINVAL, "NULL argument");
    const spmspv_schedule* t = tuned_for(A, f);
    if (!t) return fail(SPMSPV_EINVAL, "the handle has not been autotuned");
    *h_sched = *t;
    return SPMSPV_OK;
}

int spmspv_autotune_batch(spmspv_handle A, int semiring, int flags, int nbatch, const int64_t* x_off,
                          const int32_t* x_idx, const void* x_val, int64_t* y_off, int32_t* y_idx, void* y_val,
                          int64_t y_capacity, int reps, spmspv_schedule* h_best, double* h_us, void* stream) {
    if (!A || reps < 1) return fail(SPMSPV_EINVAL, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // A checked call first: rejects bad arguments and sizes the outputs.
    int64_t total = 0;
    int rc = spmspv_run_batch(A, semiring, flags & ~SPMSPV_VALIDATE, nbatch, x_off, x_idx, x_val, y_off, y_idx,
                              y_val, y_capacity, &total, stream);
    if (rc) return rc;
    const spmspv_schedule keep = A->batch_sched;
    auto cost = [&](const spmspv_schedule& c, double* us) -> int {
        A->batch_sched = c;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int r = SPMSPV_OK;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) r = fail(SPMSPV_EHIP, "event");
        for (int k = 0; k < reps + 1 && !r; ++k) {
            if (k == 1 && hipEventRecord(e0, s) != hipSuccess) r = fail(SPMSPV_EHIP, "event record");
            if (!r) r = spmspv_run_batch(A, semiring, flags & ~SPMSPV_VALIDATE, nbatch, x_off, x_idx, x_val, y_off,
                                         y_idx, y_val, y_capacity, nullptr, stream);
        }
        float ms = 0.f;
        if (!r && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                   hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            r = fail(SPMSPV_EHIP, "event timing");
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (!r) *us = 1e3 * ms / reps;
        return r;
    };
    spmspv_schedule best{};
    rc = batch_shape(A, nbatch, semiring, &best);
    if (rc) {
        A->batch_sched = keep;
        return rc;
    }
    double best_us = 0;
    if ((rc = cost(best, &best_us))) {
        A->batch_sched = keep;
        return rc;
    }
    auto consider = [&](spmspv_schedule c) -> int {
        spmspv_schedule eff{};
        A->batch_sched = c;
        if (batch_shape(A, nbatch, semiring, &eff) != SPMSPV_OK || eff.tile_log2 != c.tile_log2 ||
            eff.scatter_block != c.scatter_block || eff.scatter_items != c.scatter_items) {
            g_last_error.clear();
            return SPMSPV_OK;   // infeasible for this batch
        }
        double us = 0;
        const int r = cost(c, &us);
        if (r) return r;
        if (us < best_us) {
            best_us = us;
            best = c;
        }
        return SPMSPV_OK;
    };
    const int shapes[7][2] = {{256, 4}, {256, 8}, {256, 16}, {512, 4}, {512, 8}, {1024, 4}, {1024, 8}};
    const int merges[3] = {256, 512, 1024};
    for (int pass = 0; pass < 2 && !rc; ++pass) {
        for (int tl = kTileLog2Min; tl <= kTileLog2Max && !rc; ++tl) {
            spmspv_schedule c = best;
            c.tile_log2 = tl;
            rc = consider(c);
        }
        for (int k = 0; k < 7 && !rc; ++k) {
            spmspv_schedule c = best;
            c.scatter_block = shapes[k][0];
            c.scatter_items = shapes[k][1];
            rc = consider(c);
        }
        for (int k = 0; k < 3 && !rc; ++k) {
            spmspv_schedule c = best;
            c.merge_block = merges[k];
            rc = consider(c);
        }
    }
    if (rc) {
        A->batch_sched = keep;
        return rc;
    }
    A->batch_sched = best;
    if (h_best) *h_best = best;
    if (h_us) *h_us = best_us;
    return SPMSPV_OK;
}

int pagerank_scratch_size(spmspv_handle A, size_t* h_bytes) {
    if (!A || !h_bytes) return fail(SPMSPV_EINVAL, "NULL argument");
    *h_bytes = size_t(A->n) * 16 + 256;
    return SPMSPV_OK;
}

int pagerank_run(spmspv_handle A, float damping, float tol, int max_iter, int flags, float* rank, void* scratch,
                 size_t scratch_bytes, int32_t* h_iters, void* stream) {
    if (!A) return fail(SPMSPV_EINVAL, "NULL handle");
    if (A->m != A->n) return fail(SPMSPV_EINVAL, "PageRank needs a square matrix");
    if (A->dcsc) return fail(SPMSPV_EUNSUPPORTED, "PageRank needs a CSC handle (column degrees by id)");
    if (A->values) return fail(SPMSPV_EINVAL, "PageRank needs a pattern handle (values NULL)");
    if (!(damping > 0.f && damping < 1.f) || !(tol >= 0.f) || max_iter < 0)
        return fail(SPMSPV_EINVAL, "need 0 < damping < 1, tol >= 0, max_iter >= 0");
    if (!rank || !scratch) return fail(SPMSPV_EINVAL, "NULL argument");
    size_t need = 0;
    pagerank_scratch_size(A, &need);
    if (scratch_bytes < need) return fail(SPMSPV_ENOMEM, "scratch needs " + std::to_string(need) + " bytes");
    const bool selector = (flags & SPMSPV_USE_SELECTOR) != 0;
    if (selector && !A->selector_loaded && A->forced_classes.empty())
        return fail(SPMSPV_EINVAL, "no selector weights loaded");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = A->n;
    char* w = static_cast<char*>(scratch);
    int32_t* x_idx = reinterpret_cast<int32_t*>(w);
    float* x_val = reinterpret_cast<float*>(w + 4 * n);
    int32_t* y_idx = reinterpret_cast<int32_t*>(w + 8 * n);
    float* y_val = reinterpret_cast<float*>(w + 12 * n);
    HIP_TRY(launch_pr_init((int32_t)n, A->colptr, damping, rank, x_idx, x_val, A->ctrl, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(&A->ctrl->bfs_mode), 0u, 1, s));
    A->level_classes.clear();
    int32_t hf = 1;
    int done = 0;
    while (hf > 0 && done < max_iter) {
        // kGraphLevels steps per host check; steps after x empties are no-ops
        // With the selector: one host read per multiply (bucket count and
        // direction), or with SPMSPV_USE_GRAPH the network's direction taken
        // on the device, gating the push and pull kernels, with a host check
        // every kGraphLevels multiplies (as for BFS).  A replayed sequence is
        // always read on the host.
        const bool gated = selector && A->forced_classes.empty() && A->pull && (flags & SPMSPV_USE_GRAPH);
        const int steps = selector && !gated ? 1 : std::min(kGraphLevels, max_iter - done);
        for (int k = 0; k < steps; ++k) {
            int rc;
            if (gated) {
                rc = enqueue(A, SR_PLUS_TIMES, XV_BITS32, 0, &A->ctrl->f, x_idx, x_val, y_idx, y_val, n, nullptr,
                             false, nullptr, s, nullptr, true, -1, 3, 0, true);
                if (!rc)
                    rc = enqueue_pull(A, SR_PLUS_TIMES, XV_BITS32, 0, &A->ctrl->f, x_idx, x_val, y_idx, y_val, n,
                                      nullptr, false, nullptr, false, true, s, nullptr);
            } else if (selector) {
                int cls = 0;
                int32_t fnow = 0;
                const int forced = done + k < (int)A->forced_classes.size() ? A->forced_classes[(size_t)(done + k)]
                                                                              : -1;
                rc = run_selected(A, SR_PLUS_TIMES, XV_BITS32, 0, &A->ctrl->f, x_idx, x_val, y_idx, y_val, n,
                                  nullptr, false, nullptr, s, &cls, &fnow, forced);
                if (!rc && fnow > 0) A->level_classes.push_back(cls);
            } else {
                rc = enqueue(A, SR_PLUS_TIMES, XV_BITS32, 0, &A->ctrl->f, x_idx, x_val, y_idx, y_val, n, nullptr,
                             false, nullptr, s, nullptr);
            }
            if (rc) return rc;
            HIP_TRY(launch_pr_update((int32_t)n, A->colptr, damping, tol, rank, y_idx, y_val, x_idx, x_val, A->ctrl,
                                     s));
        }
        done += steps;
        HIP_TRY(hipMemcpyAsync(&hf, &A->ctrl->f, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    Ctrl h{};
    int rc = read_ctrl(A, &h, s);
    if (rc) return rc;
    if (h.err) {
        clear_err(A, s);
        return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err));
    }
    if (h_iters) *h_iters = h.level;
    return SPMSPV_OK;
}

int cc_run(spmspv_handle A, int flags, int32_t* labels, int32_t* h_iters, void* stream) {
    if (!A) return fail(SPMSPV_EINVAL, "NULL handle");
    if (A->m != A->n) return fail(SPMSPV_EINVAL, "connected components need a square matrix");
    if (A->dcsc) return fail(SPMSPV_EUNSUPPORTED, "connected components need a CSC handle (column degrees by id)");
    if (!labels) return fail(SPMSPV_EINVAL, "labels is NULL");
    if (flags != 0) return fail(SPMSPV_EINVAL, "cc_run takes no flags");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = A->n;
    // x and y lists in the handle's BFS buffers (values are labels, int32)
    int32_t* x_idx = A->front[0];
    int32_t* x_val = A->front[1];
    int32_t* y_idx = A->front2;
    int32_t* y_val = A->pmin;
    HIP_TRY(launch_cc_init((int32_t)n, A->colptr, labels, x_idx, x_val, A->ctrl, s));
    int32_t hf = 1;
    int64_t done = 0;
    while (hf > 0 && done <= n) {
        // kGraphLevels steps per host check; steps after x empties are no-ops
        for (int k = 0; k < kGraphLevels; ++k) {
            const int rc = enqueue(A, SR_MIN_SELECT2ND, XV_BITS32, 0, &A->ctrl->f, x_idx, x_val, y_idx, y_val, n,
                                   nullptr, false, nullptr, s, nullptr);
            if (rc) return rc;
            HIP_TRY(launch_cc_update((int32_t)n, A->colptr, labels, y_idx, y_val, x_idx, x_val, A->ctrl, s));
        }
        done += kGraphLevels;
        HIP_TRY(hipMemcpyAsync(&hf, &A->ctrl->f, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    // the persistent BFS expects its scratch (y values lived in it) reset
    HIP_TRY(reset_persistent_state(A, s));
    Ctrl h{};
    int rc = read_ctrl(A, &h, s);
    if (rc) return rc;
    if (h.err) {
        clear_err(A, s);
        return fail(SPMSPV_EDEVICE, "device error bits " + std::to_string(h.err));
    }
    if (hf > 0) return fail(SPMSPV_EDEVICE, "labels still changing after n steps");
    if (h_iters) *h_iters = h.level;
    return SPMSPV_OK;
}

int spmspv_mlp_param_count(void) { return kMlpParams; }

int spmspv_mlp_forward(const float* params, const float* X, int batch, float* logits, void* stream) {
    if (!params || batch < 0 || (batch > 0 && (!X || !logits))) return fail(SPMSPV_EINVAL, "bad argument");
    HIP_TRY(launch_mlp_forward(params, X, batch, logits, static_cast<hipStream_t>(stream)));
    return SPMSPV_OK;
}

int spmspv_mlp_train_step(float* params, float* adam_m, float* adam_v, int step, float lr, const float* X,
                          const int32_t* labels, int batch, float* grad, float* d_loss, void* stream) {
    if (!params || !X || !labels || batch < 1 || batch > kMlpBatchMax || step < 1 || lr < 0.f ||
        (lr > 0.f && (!adam_m || !adam_v)))
        return fail(SPMSPV_EINVAL, "bad argument (1 <= batch <= 128, step >= 1, lr >= 0)");
    HIP_TRY(launch_mlp_train_step(params, adam_m, adam_v, step, lr, X, labels, batch, grad, d_loss,
                                  static_cast<hipStream_t>(stream)));
    return SPMSPV_OK;
}

int spmspv_profile_read(spmspv_handle A, double* h_ms, int64_t* h_calls) {
    if (!A || !h_ms || !h_calls) return fail(SPMSPV_EINVAL, "NULL argument");
    h_ms[0] = h_ms[1] = h_ms[2] = 0.0;
    for (int c = 0; c < A->prof_used; ++c) {
        hipEvent_t* ev = &A->prof_ev[size_t(c) * 6];
        HIP_TRY(hipEventSynchronize(ev[5]));
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
            h_ms[k] += ms;
        }
    }
    *h_calls = A->prof_used;
    A->prof_used = 0;
    return SPMSPV_OK;
}

int spmspv_destroy(spmspv_handle A) {
    if (!A) return SPMSPV_OK;
    for (auto& e : A->prof_ev) (void)hipEventDestroy(e);
    if (A->graph) (void)hipGraphExecDestroy(A->graph);
    if (A->cap_stream) (void)hipStreamDestroy(A->cap_stream);
    delete A;
    return SPMSPV_OK;
}

}  // extern "C"
