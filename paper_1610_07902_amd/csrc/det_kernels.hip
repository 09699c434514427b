// Deterministic plus-times multiply.  y(i) is the fp32 sum of row i's
// products, each rounded to fp32 (Mult), added one at a time in product
// order: x order, then the column's storage order -- the order in which
// Algorithm 1 forms the products.  Its bits depend on the input alone, not on
// bucket counts, workgroup counts or the timing of atomics.
//   k_det_gather   product w -> (row, RN32(a * x)) at list position w; the
//                  scan's column tables give each product's column.
//   radix passes   a stable LSD sort of that list by row, digits of up to
//                  11 bits: per-tile digit counts (a row of the count
//                  matrix per radix tile of kDetTile entries), their
//                  exclusive scan in digit-major order (Algorithm 2's count
//                  matrix: every (digit, tile) run gets its position) from a
//                  column scan within groups of tiles plus one workgroup of
//                  digit bases, then each tile's entries are written at those
//                  positions, ranked stably (wave ballots, waves in order,
//                  rounds in order).
//   k_det_heads, k_det_scan_small, k_det_fold, k_det_fold_long
//                  every row's products now form one run in product order,
//                  folded sequentially from its first product by one thread
//                  (by one wave past kDetShortRun + 1 products); y is
//                  written at the run's ordinal, so y is ascending.
// A product whose row the mask removes carries row m and sorts after every
// real row; it is never written.

#include "device_ops.h"

namespace spv {

namespace {

constexpr int kGatherBlock = 1024;   // one batch of eight products per thread for 8192-product chunks
constexpr int kMaxDigits = 1 << kDetMaxDigitBits;
constexpr int kDetWaves = kDetBlock / kWave;

// Radix tiles of the call's product list (at least one).  Every kernel over
// tiles takes the count from W on the device and loops over the tiles with
// whatever grid it was given, so the host never reads W back (the scan caps W
// at nnz, which the workspace's tile arrays are sized for).
__device__ __forceinline__ int det_tiles(int W) { return W > 0 ? (W + kDetTile - 1) / kDetTile : 1; }

// Radix tiles per group of the count matrix's column scan: at least 16, and
// enough that there are at most kDetMaxGroups groups.
__device__ __forceinline__ int det_group(int nt) {
    const int g = (nt + kDetMaxGroups - 1) / kDetMaxGroups;
    return g > 16 ? g : 16;
}

// Eight waves per SIMD (at most 64 registers): two 1024-thread workgroups
// per compute unit where the chunk's table fits twice in LDS (4096-product
// chunks); at 66 registers only one fitted.
__global__ __launch_bounds__(kGatherBlock, 8) void k_det_gather(DetArgs a, uint2* list) {
    extern __shared__ int32_t s_off[];   // the chunk's column table, 3 x (chunk + 2) words
    // every word the first chunk's set-up needs, loaded together (the grid is
    // at most the workspace's chunk count, so chunk_col has both entries; they
    // are used only if the chunks exist)
    const int W = ld_ctrl(&a.ctrl->W);
    const int fnz = ld_ctrl(&a.ctrl->fnz);
    const int err = ld_ctrl(reinterpret_cast<const int32_t*>(&a.ctrl->err));
    int col_c = a.chunk_col[blockIdx.x], col_next = a.chunk_col[blockIdx.x + 1];
    // The per-call bookkeeping the bucket scatter does on the other paths:
    // the scan's statistics, and its look-back words cleared for the next
    // call; and this call's list of long runs emptied.
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st_ctrl_u(&a.ctrl->ticket_scan, 0u);
        st_ctrl(&a.ctrl->fnz_last, fnz);
        st_ctrl(&a.ctrl->W_last, W);
        *a.long_count = 0;   // the fold appends this call's long runs
        st_ctrl(&a.ctrl->maxlen_last, atomicExch(&a.ctrl->maxlen, 0));
    }
    for (int i = blockIdx.x * kGatherBlock + threadIdx.x; i < a.lb1_clear; i += gridDim.x * kGatherBlock) {
        a.lb1[i] = 0;
        a.lb1[a.lb1_n + i] = 0;
    }
    // a failed look-back leaves the column tables inconsistent: write
    // nothing (the error is reported with the call's status)
    if (err & (int32_t)ERR_SPIN) return;
    const int64_t chunk = int64_t(1) << a.chunk_log2;
    const int nchunks = (int)((W + chunk - 1) >> a.chunk_log2);
    const int cap = (int)chunk + 2;
    int32_t* s_st = s_off + cap;
    uint32_t* s_xv = reinterpret_cast<uint32_t*>(s_st + cap);
    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t w0 = (int64_t)c << a.chunk_log2;
        const int64_t w1 = w0 + chunk < W ? w0 + chunk : (int64_t)W;
        // chunk_col[k] is the column holding product k * chunk, so the
        // chunk's last product lies in a column no later than chunk_col[k + 1]
        // (the last chunk ends at the last non-empty column)
        if (c != (int)blockIdx.x) {
            col_c = a.chunk_col[c];
            col_next = a.chunk_col[c + 1];   // c + 1 <= nchunks
        }
        const int c_lo = col_c;
        const int c_hi = w1 < W ? col_next : fnz - 1;
        const int ncol = c_hi - c_lo + 1;
        // the chunk's column table in LDS: product offsets, first entries, x values
        for (int i = threadIdx.x; i <= ncol; i += kGatherBlock) {
            s_off[i] = a.coff[c_lo + i];
            if (i < ncol) {
                s_st[i] = a.cstart[c_lo + i];
                s_xv[i] = a.cxv[c_lo + i];
            }
        }
        __syncthreads();
        // products eight per thread at a time: every load unconditional
        // (indices clamped to the chunk's first product), so they are in
        // flight together
        constexpr int B8 = 8;
        const int64_t first = (int64_t)s_st[0] + (w0 - s_off[0]);
        int top = 1;   // the largest power of two <= ncol
        while (top * 2 <= ncol) top *= 2;
        for (int64_t wb = w0 + threadIdx.x; wb < w1; wb += (int64_t)B8 * kGatherBlock) {
            // the last column starting at or before each product: the eight
            // searches advance in lockstep, the same steps for every lane,
            // with clamped reads, so each step's eight LDS reads are in flight
            // together (a search loop per product waits for every read in turn)
            int lo[B8];
#pragma unroll
            for (int u = 0; u < B8; ++u) lo[u] = 0;
            for (int step = top; step > 0; step >>= 1) {
#pragma unroll
                for (int u = 0; u < B8; ++u) {
                    const int64_t w = wb + (int64_t)u * kGatherBlock;
                    const int k = lo[u] + step;
                    const int o = s_off[min(k, ncol - 1)];
                    if (k < ncol && o <= w) lo[u] = k;
                }
            }
            int64_t q[B8];
            uint32_t xv[B8];
#pragma unroll
            for (int u = 0; u < B8; ++u) {
                const int64_t w = wb + (int64_t)u * kGatherBlock;
                q[u] = w < w1 ? (int64_t)s_st[lo[u]] + (w - s_off[lo[u]]) : first;
                xv[u] = s_xv[lo[u]];
            }
            int32_t row[B8];
            float av[B8];
#pragma unroll
            for (int u = 0; u < B8; ++u) row[u] = a.rowids[q[u]];
#pragma unroll
            for (int u = 0; u < B8; ++u) av[u] = a.values ? a.values[q[u]] : 1.0f;
            uint32_t mw[B8];
#pragma unroll
            for (int u = 0; u < B8; ++u) mw[u] = a.mask ? a.mask[row[u] >> 5] : 0u;
#pragma unroll
            for (int u = 0; u < B8; ++u) {
                const int64_t w = wb + (int64_t)u * kGatherBlock;
                if (w < w1) {
                    int32_t r = row[u];
                    const float t = __fmul_rn(av[u], __uint_as_float(xv[u]));
                    if (a.mask && ((mw[u] >> (r & 31)) & 1u) != (uint32_t)a.mask_keep) r = a.m;
                    list[w] = make_uint2((uint32_t)r, __float_as_uint(t));
                }
            }
        }
        __syncthreads();   // the next chunk's table reuses the LDS
    }
}

__global__ __launch_bounds__(kDetBlock) void k_det_hist(DetArgs a, const uint2* in, int shift, int dbits) {
    __shared__ int h[kMaxDigits];
    const int nd = 1 << dbits;
    const int W = ld_ctrl(&a.ctrl->W);
    const int nt = det_tiles(W);
    const int64_t last = W > 0 ? W - 1 : 0;
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        const int64_t base = (int64_t)t * kDetTile;
        // every key loaded first (clamped indices, no branch around a load),
        // so the loads overlap each other and the clearing of the counts
        uint32_t key[kDetItems];
#pragma unroll
        for (int i = 0; i < kDetItems; ++i) key[i] = in[min(base + i * kDetBlock + threadIdx.x, last)].x;
        for (int d = threadIdx.x; d < nd; d += kDetBlock) h[d] = 0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kDetItems; ++i) {
            const int64_t e = base + i * kDetBlock + threadIdx.x;
            if (e < W) atomicAdd(&h[(key[i] >> shift) & (uint32_t)(nd - 1)], 1);
        }
        __syncthreads();
        // the tile's row of the count matrix: contiguous, so the stores coalesce
        for (int d = threadIdx.x; d < nd; d += kDetBlock) a.counts[(int64_t)t * nd + d] = h[d];
        __syncthreads();   // the next tile clears h
    }
}

// Column prefixes of the count matrix within groups of det_group(tiles)
// consecutive tiles: counts[b][d] becomes the digit-d entries of the earlier
// tiles of b's group, gt[g][d] the group's digit-d total.  Thread = digit
// (the loads of a tile row coalesce), grid (kDetMaxGroups, digit slices).
__global__ __launch_bounds__(kDetBlock) void k_det_colscan(DetArgs a, int32_t* gt, int nd) {
    const int nt = det_tiles(ld_ctrl(&a.ctrl->W));
    const int group = det_group(nt);
    const int d = blockIdx.y * kDetBlock + threadIdx.x;
    const int b0 = blockIdx.x * group;
    if (d >= nd || b0 >= nt) return;   // the grid covers kDetMaxGroups groups
    const int b1 = min(b0 + group, nt);
    int run = 0;
    for (int b = b0; b < b1; b += 16) {
        int v[16];
        // clamped, unconditional loads so that all sixteen are in flight
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = a.counts[(int64_t)min(b + u, b1 - 1) * nd + d];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (b + u < b1) {
                a.counts[(int64_t)(b + u) * nd + d] = run;
                run += v[u];
            }
        }
    }
    gt[(int64_t)blockIdx.x * nd + d] = run;
}

// gt[g][d] <- (entries of every digit below d) + (digit-d entries of the
// groups before g): with the in-group prefixes, each (digit, block) run's
// position in the digit-major order of Algorithm 2's count matrix.  One
// block; digit d = p * 1024 + thread, so the loads of a group row coalesce.
// At most kDetMaxGroups groups: all of a thread's totals are loaded at once.
constexpr int kBaseBlock = 1024;
__global__ __launch_bounds__(kBaseBlock) void k_det_digit_base(DetArgs a, int32_t* gt, int nd) {
    __shared__ int s_tmp[kBaseBlock / kWave + 1];
    const int nt = det_tiles(ld_ctrl(&a.ctrl->W));
    const int group = det_group(nt);
    const int ngroups = (nt + group - 1) / group;
    constexpr int P = kMaxDigits / kBaseBlock;
    int v[P][kDetMaxGroups];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int d = p * kBaseBlock + threadIdx.x;
        const int dc = d < nd ? d : 0;
#pragma unroll
        for (int g = 0; g < kDetMaxGroups; ++g) v[p][g] = gt[(int64_t)min(g, ngroups - 1) * nd + dc];
    }
    int carry = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int d = p * kBaseBlock + threadIdx.x;
        int tot = 0;
#pragma unroll
        for (int g = 0; g < kDetMaxGroups; ++g) tot += g < ngroups ? v[p][g] : 0;
        if (d >= nd) tot = 0;
        int total;
        int run = block_exclusive_i32<kBaseBlock>(tot, s_tmp, total) + carry;
        carry += total;
        if (d < nd) {
#pragma unroll
            for (int g = 0; g < kDetMaxGroups; ++g) {
                if (g < ngroups) {
                    gt[(int64_t)g * nd + d] = run;
                    run += v[p][g];
                }
            }
        }
    }
}

// In-place exclusive scan of the tiles' head counts (tiles + 1 values) by
// one block.
__global__ __launch_bounds__(kBaseBlock) void k_det_scan_small(DetArgs a) {
    __shared__ int s_tmp[kBaseBlock / kWave + 1];
    int32_t* data = a.counts;
    const int n = det_tiles(ld_ctrl(&a.ctrl->W)) + 1;
    int carry = 0;
    for (int i0 = 0; i0 < n; i0 += kBaseBlock) {
        const int i = i0 + threadIdx.x;
        const int v = i < n ? data[i] : 0;
        int total;
        const int e = block_exclusive_i32<kBaseBlock>(v, s_tmp, total);
        if (i < n) data[i] = carry + e;
        carry += total;
    }
}

// The scatter's workgroup: more threads over the same tile, so fewer rounds
// of ballots and barriers per tile.
constexpr int kScatBlock = 1024;
constexpr int kScatItems = kDetTile / kScatBlock;
constexpr int kScatWaves = kScatBlock / kWave;

__global__ __launch_bounds__(kScatBlock) void k_det_scatter(DetArgs a, const uint2* in, uint2* out, int shift,
                                                           int dbits, const int32_t* gt) {
    __shared__ int s_run[kMaxDigits];             // next position of each digit's run
    __shared__ uint8_t s_wc[kScatWaves][kMaxDigits];   // this round's count per wave and digit (<= 64)
    const int nd = 1 << dbits;
    const int W = ld_ctrl(&a.ctrl->W);
    const int nt = det_tiles(W);
    const int group = det_group(nt);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        const int64_t base = (int64_t)t * kDetTile;
        if (base >= W) break;   // W == 0: one empty tile
        // the tile's entries into registers first (clamped indices), in
        // flight together with the run-start loads, so the rounds below wait
        // for no memory
        const int64_t last = W - 1;
        uint2 its[kScatItems];
#pragma unroll
        for (int r = 0; r < kScatItems; ++r) its[r] = in[min(base + r * kScatBlock + threadIdx.x, last)];
        const int32_t* grow = gt + (int64_t)(t / group) * nd;
        for (int d = threadIdx.x; d < nd; d += kScatBlock) {
            s_run[d] = a.counts[(int64_t)t * nd + d] + grow[d];
            for (int w = 0; w < kScatWaves; ++w) s_wc[w][d] = 0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kScatItems; ++r) {
            const int64_t e = base + r * kScatBlock + threadIdx.x;
            const bool valid = e < W;
            const uint2 it = its[r];
            const int d = valid ? (int)((it.x >> shift) & (uint32_t)(nd - 1)) : 0;
            // lanes of this wave holding the same digit
            uint64_t peers = __ballot(valid);
            for (int bit = 0; bit < dbits; ++bit) {
                const bool one = (d >> bit) & 1;
                const uint64_t v = __ballot(one);
                peers &= one ? v : ~v;
            }
            const int rank = __popcll(peers & below);
            const bool leader = valid && rank == 0;
            if (leader) s_wc[wave][d] = __popcll(peers);
            __syncthreads();
            if (valid) {
                int off = s_run[d];
                for (int w = 0; w < wave; ++w) off += s_wc[w][d];
                out[off + rank] = it;
            }
            __syncthreads();
            // a wave clears its own entries before (in its program order) it
            // writes the next round's; others read them only after the next
            // round's first barrier
            if (leader) {
                atomicAdd(&s_run[d], __popcll(peers));
                s_wc[wave][d] = 0;
            }
        }
        __syncthreads();   // the next tile sets s_run and s_wc afresh
    }
}

// Eight waves per SIMD (at most 64 registers; 65 allowed seven).
__global__ __launch_bounds__(kDetBlock, 8) void k_det_heads(DetArgs a, const uint2* list) {
    __shared__ int s_tmp[kDetWaves + 1];
    const int W = ld_ctrl(&a.ctrl->W);
    const int nt = det_tiles(W);
    const int64_t last = W > 0 ? W - 1 : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.counts[nt] = 0;
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        const int64_t base = (int64_t)t * kDetTile;
        // every row and its predecessor's first (unconditional loads, clamped
        // indices, all in flight together), then the comparisons
        uint32_t rw[kDetItems], pv[kDetItems];
#pragma unroll
        for (int i = 0; i < kDetItems; ++i) {
            const int64_t e = base + i * kDetBlock + threadIdx.x;
            rw[i] = list[min(e, last)].x;
            pv[i] = list[max(min(e, last) - 1, (int64_t)0)].x;
        }
        int cnt = 0;
#pragma unroll
        for (int i = 0; i < kDetItems; ++i) {
            const int64_t e = base + i * kDetBlock + threadIdx.x;
            if (e < W && rw[i] < (uint32_t)a.m && (e == 0 || pv[i] != rw[i])) ++cnt;
        }
        int total;
        block_exclusive_i32<kDetBlock>(cnt, s_tmp, total);   // ends with a barrier
        if (threadIdx.x == 0) a.counts[t] = total;
    }
}

// The fold's workgroup: twice the radix passes' threads over the same tile,
// so each thread folds half as many runs.
constexpr int kFoldBlock = 512;
constexpr int kFoldItems = kDetTile / kFoldBlock;
constexpr int kFoldWaves = kFoldBlock / kWave;

// A tile's kDetTile entries are staged in LDS with the kDetShortRun + 1
// entries after them (a short fold never reads further).  (1) Row boundaries
// are found with wave ballots; the heads (boundaries of real rows inside the
// tile) are compacted, in entry order, into a list of positions, and the
// first other boundary (in the halo, or where the masked rows begin) ends the
// tile's last run.  (2) Thread t folds heads t, t + kFoldBlock, ...: a run
// ends where the next head starts, so its adds need no row comparisons, and
// consecutive heads -- ordinals, so outputs -- sit in consecutive lanes.
// Past kDetShortRun + 1 entries a run is handed to k_det_fold_long through
// the call's list of long runs.  Workgroups loop over tiles.  (Giving
// each thread the heads among its own items left the wave waiting on the
// lane that held most of them: heads evenly spaced by a power of two all
// fall on one thread.)
__global__ __launch_bounds__(kFoldBlock) void k_det_fold(DetArgs a, const uint2* list) {
    constexpr int kStage = kDetTile + kDetShortRun + 1;
    constexpr int kCells = kFoldItems * kFoldWaves;   // (round, wave) ballots
    static_assert(kCells == kWave, "one lane per ballot in the head-count scan");
    static_assert(kDetTile <= 65536, "head positions are 16-bit");
    __shared__ uint2 s_e[kStage];
    __shared__ uint16_t s_head[kDetTile];
    __shared__ uint64_t s_bal[kCells];   // heads of round r, wave w at r * kFoldWaves + w
    __shared__ int s_pre[kCells + 1];    // heads before each ballot, in entry order
    __shared__ int s_stop, s_nlong, s_nlong_all, s_lbase;
    __shared__ int4 s_long[kDetLongPerBlock];   // the tile's long runs, then copied to the list
    __shared__ uint32_t s_prev;
    __shared__ int64_t s_run0;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int W = ld_ctrl(&a.ctrl->W);
    const int nt = det_tiles(W);
    if (blockIdx.x == 0 && tid == 0) {
        const int64_t total = a.counts[nt];
        __hip_atomic_store(&a.ctrl->nnz_y, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a.d_nnz_y) *a.d_nnz_y = total;
    }
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        const int64_t base = (int64_t)t * kDetTile;
        if (base >= W) {   // W == 0: one empty tile
            continue;
        }
        const int n_in = (int)min((int64_t)kDetTile, (int64_t)W - base);   // this tile's entries
        const int n_st = (int)min((int64_t)kStage, (int64_t)W - base);     // with the halo
        constexpr int kRounds = (kStage + kFoldBlock - 1) / kFoldBlock;
        {
            // every load unconditional (index clamped into range), so all are in
            // flight before the first wait; a guarded load compiles to a branch
            // that waits for its load before the next one is issued
            uint2 st[kRounds];
#pragma unroll
            for (int r = 0; r < kRounds; ++r) st[r] = list[base + min(r * kFoldBlock + tid, n_st - 1)];
            // the row before the tile and the tile's first output position,
            // in the same round trip (clamped index)
            if (tid == 0) {
                const uint32_t before = list[base > 0 ? base - 1 : 0].x;
                s_run0 = a.counts[t];
                s_prev = base > 0 ? before : ~0u;
            }
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
                const int i = r * kFoldBlock + tid;
                if (i < n_st) s_e[i] = st[r];
            }
        }
        if (tid == 0) {
            s_stop = n_st;
            s_nlong = 0;
            s_nlong_all = 0;
        }
        __syncthreads();
        // (1) item r of thread t is entry r * kFoldBlock + t; the rounds past
        // kFoldItems cover the halo, where only the first boundary matters
        const uint64_t lower = (1ull << lane) - 1ull;
        uint32_t heads = 0;   // bit r: item r is a head
        int stop = n_st;
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const int i = r * kFoldBlock + tid;
            const int ic = min(i, n_st - 1);
            const uint32_t row = s_e[ic].x;
            const uint32_t prev = s_e[max(ic - 1, 0)].x;
            const bool bound = i < n_st && (i == 0 ? base == 0 || s_prev != row : prev != row);
            const bool head = bound && i < n_in && row < (uint32_t)a.m;
            if (bound && !head) stop = min(stop, i);
            if (r < kFoldItems) {
                const uint64_t bal = __ballot(head);
                if (lane == 0) s_bal[r * kFoldWaves + wave] = bal;
                heads |= head ? (1u << r) : 0u;
            }
        }
        if (stop < n_st) atomicMin(&s_stop, stop);
        __syncthreads();
        if (wave == 0) {
            // exclusive scan of the 64 ballots' head counts, (round, wave) order
            const int c = __popcll(s_bal[lane]);
            int v = c;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const int u = __shfl_up(v, d);
                if (lane >= d) v += u;
            }
            s_pre[lane] = v - c;
            if (lane == kWave - 1) s_pre[kCells] = v;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kFoldItems; ++r) {
            if ((heads >> r) & 1u) {
                const int cell = r * kFoldWaves + wave;
                s_head[s_pre[cell] + __popcll(s_bal[cell] & lower)] = (uint16_t)(r * kFoldBlock + tid);
            }
        }
        __syncthreads();
        // (2) folds, one add at a time in entry order
        const int H = s_pre[kCells];
        const int last_end = s_stop;
        const int64_t run0 = s_run0;
        // the tile's long runs are counted first, so that their reservation
        // in the call's list is in flight while the runs are folded (the
        // list's order does not matter, each run's fold is its own)
        {
            int nlong_t = 0;
            for (int j = tid; j < H; j += kFoldBlock) {
                const int end = j + 1 < H ? s_head[min(j + 1, H - 1)] : last_end;
                nlong_t += end - s_head[j] > kDetShortRun + 1 ? 1 : 0;
            }
            if (nlong_t > 0) atomicAdd(&s_nlong_all, nlong_t);
        }
        __syncthreads();
        const int nl = min(s_nlong_all, kDetLongPerBlock);
        int lbase = 0;   // thread 0: the tile's first position in the list
        if (tid == 0 && nl > 0) lbase = atomicAdd(a.long_count, nl);
        for (int j = tid; j < H; j += kFoldBlock) {
            const int i = s_head[j];
            const int nxt = s_head[min(j + 1, H - 1)];
            const int end = j + 1 < H ? nxt : last_end;   // the run is entries [i, end)
            const uint2 e0 = s_e[i];
            float acc = __uint_as_float(e0.y);
            const int last = i + min(end - i, kDetShortRun + 1) - 1;   // the last entry folded here
            for (int q = i + 1; q <= last; q += 8) {
                // eight reads ahead of the adds; past the run the pad is -0, which
                // leaves every sum (either zero included) unchanged
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const uint32_t bits = s_e[min(q + u, last)].y;
                    v[u] = q + u <= last ? __uint_as_float(bits) : -0.0f;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = __fadd_rn(acc, v[u]);
            }
            const int64_t p = run0 + j;
            if (end - i > kDetShortRun + 1) {
                // more than kDetShortRun + 1 entries, so at most
                // kDetLongPerBlock runs start in a tile
                const int slot = atomicAdd(&s_nlong, 1);
                if (slot < kDetLongPerBlock)
                    s_long[slot] = make_int4((int)e0.x, (int)__float_as_uint(acc), (int)(base + last + 1), (int)p);
                else
                    atomicOr(&a.ctrl->err, ERR_SPIN);   // not reached (see above)
            } else if (p < a.y_cap) {
                a.y_idx[p] = (int32_t)e0.x;
                if (a.y_val) a.y_val[p] = acc;
            }
        }
        __syncthreads();
        // the tile's long runs join the call's list
        if (nl > 0) {
            if (tid == 0) s_lbase = lbase;
            __syncthreads();
            if (tid < nl) a.long_runs[s_lbase + tid] = s_long[tid];
        }
        __syncthreads();   // the next tile restages the LDS
    }
}

// One wave per long run of the fold's list, so every run starts at once.
// The wave works in trips of kLongDepth steps of 64
// consecutive entries (one coalesced load per step), the next trip's loads
// issued before the current trip's steps; each step's values go to the
// wave's LDS row and one lane adds them in order from there, so the run
// costs its dependent adds and little more.
// (Folding through lane reads cost about 90 cycles per entry, a 16K-entry
// hub row 0.6 ms, and reading the lanes into scalar registers for the adds
// still cost more than this LDS row; one thread per run with sixteen loads
// ahead left the memory latency exposed.)
constexpr int kLongDepth = 8;

__global__ __launch_bounds__(kDetBlock) void k_det_fold_long(DetArgs a, const uint2* list) {
    __shared__ __attribute__((aligned(16))) float s_v[kDetWaves][kWave];
    const int W = ld_ctrl(&a.ctrl->W);
    const int nlong = *a.long_count;   // the fold's list of long runs
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int nwaves = gridDim.x * kDetWaves;
    // clamped, unconditional loads (the end of the list is checked where the
    // rows are compared): a guarded load sits behind a branch, after which the
    // compiler waits for every load in flight, the prefetched ones too
    auto load = [&](int64_t k) { return list[min(k + lane, (int64_t)W - 1)]; };
    for (int pr = blockIdx.x * kDetWaves + wv; pr < nlong; pr += nwaves) {
        const int4 rec = a.long_runs[pr];
        const uint32_t row = (uint32_t)rec.x;
        float acc = __uint_as_float((uint32_t)rec.y);
        int64_t k = rec.z;
        uint2 cur[kLongDepth];
#pragma unroll
        for (int d = 0; d < kLongDepth; ++d) cur[d] = load(k + (int64_t)d * kWave);
        bool more = true;
        while (more) {
            // a trip: issue the next trip's kLongDepth loads, fold this trip's
            // kLongDepth steps, then take the loads over (the only wait for
            // them comes a trip after their issue); steps past the run's end
            // find no entries and add nothing
            uint2 nxt[kLongDepth];
#pragma unroll
            for (int d = 0; d < kLongDepth; ++d) nxt[d] = load(k + (int64_t)(kLongDepth + d) * kWave);
#pragma unroll
            for (int d = 0; d < kLongDepth; ++d) {
                const uint2 v = cur[d];
                const uint64_t match = __ballot(more & (k + lane < W) & (v.x == row));
                // entries of the run in this step: the lanes before the first mismatch
                const int n = (~match == 0ull) ? kWave : __ffsll((unsigned long long)~match) - 1;
                // lanes past the run hold -0, which leaves every sum unchanged,
                // so the 64 adds carry no conditions
                s_v[wv][lane] = lane < n ? __uint_as_float(v.y) : -0.0f;
                __builtin_amdgcn_wave_barrier();
                if (lane == 0 && n > 0) {
                    // all 64 values into registers first, then the dependent adds
                    float4 q[kWave / 4];
#pragma unroll
                    for (int j = 0; j < kWave / 4; ++j) q[j] = *reinterpret_cast<const float4*>(&s_v[wv][4 * j]);
#pragma unroll
                    for (int j = 0; j < kWave / 4; ++j) {
                        acc = __fadd_rn(acc, q[j].x);
                        acc = __fadd_rn(acc, q[j].y);
                        acc = __fadd_rn(acc, q[j].z);
                        acc = __fadd_rn(acc, q[j].w);
                    }
                }
                __builtin_amdgcn_wave_barrier();
                more = more && n == kWave;
                k += kWave;
            }
#pragma unroll
            for (int d = 0; d < kLongDepth; ++d) cur[d] = nxt[d];
        }
        if (lane == 0 && rec.w < a.y_cap) {
            a.y_idx[rec.w] = (int32_t)row;
            if (a.y_val) a.y_val[rec.w] = acc;
        }
    }
}

}  // namespace

hipError_t launch_det_gather(const DetArgs& a, uint2* list, int grid, hipStream_t s) {
    const size_t lds = 3 * ((size_t(1) << a.chunk_log2) + 2) * sizeof(int32_t);
    if (lds > 65536) {   // chunks of 8192 products
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_det_gather),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_det_gather, dim3(grid), dim3(kGatherBlock), lds, s, a, list);
    return hipGetLastError();
}

hipError_t launch_det_pass(const DetArgs& a, const uint2* in, uint2* out, int shift, int digit_bits,
                           int32_t* partials, int grid, hipStream_t s) {
    if (digit_bits < 1 || digit_bits > kDetMaxDigitBits || grid < 1) return hipErrorInvalidValue;
    const int nd = 1 << digit_bits;
    hipLaunchKernelGGL(k_det_hist, dim3(grid), dim3(kDetBlock), 0, s, a, in, shift, digit_bits);
    hipLaunchKernelGGL(k_det_colscan, dim3(kDetMaxGroups, (nd + kDetBlock - 1) / kDetBlock), dim3(kDetBlock), 0, s,
                       a, partials, nd);
    hipLaunchKernelGGL(k_det_digit_base, dim3(1), dim3(kBaseBlock), 0, s, a, partials, nd);
    hipLaunchKernelGGL(k_det_scatter, dim3(grid), dim3(kScatBlock), 0, s, a, in, out, shift, digit_bits, partials);
    return hipGetLastError();
}

hipError_t launch_det_fold(const DetArgs& a, const uint2* list, int grid, hipStream_t s) {
    if (grid < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_det_heads, dim3(grid), dim3(kDetBlock), 0, s, a, list);
    hipLaunchKernelGGL(k_det_scan_small, dim3(1), dim3(kBaseBlock), 0, s, a);
    hipLaunchKernelGGL(k_det_fold, dim3(grid), dim3(kFoldBlock), 0, s, a, list);
    hipLaunchKernelGGL(k_det_fold_long, dim3(2048), dim3(kDetBlock), 0, s, a, list);
    return hipGetLastError();
}

}  // namespace spv
