// Hot-path kernels of SpMSpV-bucket for gfx950 (CDNA4, wave64).
//
// One y <- A x is three launches on one stream:
//   k_scan    (step a) gathers the selected columns' [colptr[j], colptr[j+1])
//             ranges, prefix-sums their lengths with a single-pass
//             decoupled look-back scan, compacts the non-empty columns and
//             records the first column of every fixed-size product chunk.
//             This is the exact work estimate of Algorithm 2
//             (Estimate-Buckets): W = sum of selected column lengths.
//   k_scatter (step b) walks the W products in equal chunks (merge-path
//             over nonzeros: every workgroup gets the same number of
//             products however the column lengths vary), reads row ids and
//             values coalesced, applies Mult, and appends (row, value) to
//             the row-range bucket of the row (Algorithm 1, step 1).  Bucket
//             counts of the chunk are kept in LDS; each bucket's slot range
//             is reserved with one atomic per (chunk, bucket), which plays
//             the role of Algorithm 2's per-thread Boffset prefix.
//   k_merge   (steps c, d) gives each bucket one workgroup and an LDS-resident
//             sparse accumulator over the bucket's rows.  Every cell of the
//             tile is initialised with wide stores (on the GPU cheaper than
//             the first-touch test that Algorithm 1's partial
//             initialisation needs); touched rows are marked in an LDS row
//             bitmap, whose population count is the bucket's number of
//             unique rows.  The per-bucket unique
//             counts are prefix-summed across workgroups by decoupled
//             look-back, and each workgroup writes its rows straight to y
//             (Algorithm 1, step 3), ascending when sorted output is asked
//             for (walk of the row bitmap in order).
//
// Bucket storage: bucket k covers rows [k*T, (k+1)*T) with T = 2^tile_log2.
// Its slots start at rcp[k*T], the number of stored entries of A in rows
// before k*T, and it has rcp[(k+1)*T] - rcp[k*T] slots.  With distinct x
// indices each product (i, j) is a distinct stored entry of A, so a bucket
// never receives more entries than its rows hold: total bucket space is
// nnz(A), the bound of "Performance optimizations / Memory allocation".

#include <hip/hip_ext.h>

#include "decide.h"
#include "device_ops.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

namespace spv {

namespace {

// ------------------------------------------------------------------ step (a)
// Two look-back chains per tile, one for the product count (sum of column
// lengths) and one for the number of non-empty columns, each with a 62-bit
// value: no input, valid or not, can make one overflow into the other.
template <int BLOCK, int ITEMS, int XMODE, bool BATCH, bool CHAIN>
__global__ __launch_bounds__(BLOCK) void k_scan(ScanArgs a) {
    constexpr int TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_tmp[BLOCK / kWave + 1];
    __shared__ uint64_t s_excl_sum, s_excl_cnt;
    __shared__ int s_max;
    __shared__ int64_t s_xoff[BATCH ? kMaxBatch + 1 : 1];
    const int tid = threadIdx.x;
    int f;
    if constexpr (BATCH) {
        // Vector offsets come from the caller or the previous BFS level.
        for (int i = tid; i <= a.nbatch; i += BLOCK)
            s_xoff[i] = __hip_atomic_load(&a.xoff[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int64_t F = s_xoff[a.nbatch];
        const bool ok = F >= 0 && F <= a.f_cap && s_xoff[0] == 0;
        if (!ok && blockIdx.x == 0 && tid == 0) atomicOr(&a.ctrl->err, ERR_X_RANGE);
        f = ok ? (int)F : 0;
    } else {
        f = a.f_dev ? ld_ctrl(a.f_dev) : a.f_host;
    }
    // issued with the frontier length so the two round trips overlap
    uint32_t chain_ready = 0;
    if constexpr (CHAIN)
        chain_ready = a.chain ? __hip_atomic_load(&a.ctrl->chain_ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
    uint64_t* lb_sum = a.lb1;
    uint64_t* lb_cnt = a.lb1 + a.lb1_n;

    // Clear the scatter counters and merge look-back words of this call.
    for (int i = blockIdx.x * BLOCK + tid; i < a.nb; i += gridDim.x * BLOCK) {
        a.cursor[i] = 0;
        a.lb3[i] = 0;
    }
    if constexpr (BATCH)
        for (int i = blockIdx.x * BLOCK + tid; i <= a.nb; i += gridDim.x * BLOCK) a.kcount[i] = 0;
    if (blockIdx.x == 0 && tid == 0) {
        st_ctrl_u(&a.ctrl->ticket_merge, 0u);
        if (!BATCH && !a.f_dev) st_ctrl(&a.ctrl->f, f);   // the selector reads f from here
        if (a.bump_level && f > 0) st_ctrl(&a.ctrl->level, ld_ctrl(&a.ctrl->level) + 1);
        if (f <= 0) {
            st_ctrl(&a.ctrl->W, 0);
            st_ctrl(&a.ctrl->fnz, 0);
            a.coff[0] = 0;
        }
    }
    if (tid == 0) s_max = 0;
    bool clear_x = false;   // push level after a pull level: clear the x bits that level left
    if constexpr (CHAIN) {
        // Direction-switching BFS after a pull level: that level's emit left
        // per-workgroup sums of this frontier's column lengths, so the
        // decision is taken here (workgroup 0 adds them up and publishes the
        // direction in one word) and a level that stays pull needs no column
        // tables.
        if (chain_ready) {
            __shared__ int s_dir;
            if (blockIdx.x == 0) {
                // the frontier's column sums from the emit's per-workgroup partials
                int64_t ws = 0;
                int32_t wm = 0, wz = 0;
                for (int b = tid; b < a.chain_nparts; b += BLOCK) {
                    ws += a.chain_part[2 * b];
                    const int64_t mz = a.chain_part[2 * b + 1];
                    wm = max(wm, (int32_t)(mz >> 32));
                    wz += (int32_t)(uint32_t)mz;
                }
                __shared__ int64_t s_ws[BLOCK / kWave];
                __shared__ int32_t s_wm[BLOCK / kWave], s_wz[BLOCK / kWave];
#pragma unroll
                for (int d = kWave / 2; d >= 1; d >>= 1) {
                    ws += __shfl_xor(ws, d, kWave);
                    wm = max(wm, __shfl_xor(wm, d, kWave));
                    wz += __shfl_xor(wz, d, kWave);
                }
                if ((tid & (kWave - 1)) == 0) {
                    s_ws[tid / kWave] = ws;
                    s_wm[tid / kWave] = wm;
                    s_wz[tid / kWave] = wz;
                }
                __syncthreads();
                int64_t Wt = 0;
                int32_t mx = 0, nz = 0;
                for (int w = 0; w < BLOCK / kWave; ++w) {
                    Wt += s_ws[w];
                    mx = max(mx, s_wm[w]);
                    nz += s_wz[w];
                }
                const int32_t W = (int32_t)Wt;
                int dir;
                if (a.chain == 2) {
                    dir = select_step(a.ctrl, a.sel, a.n, a.nnz, a.has_pull, 1, -1, f, W, mx, nz);
                } else {
                    if (tid == 0) s_dir = heuristic_step(a.ctrl, a.n, f, W);
                    __syncthreads();
                    dir = s_dir;
                }
                if (tid == 0) {
                    st_ctrl(&a.ctrl->W, W);
                    st_ctrl(&a.ctrl->fnz, nz);
                    st_ctrl_u(&a.ctrl->chain_word, 2u | (uint32_t)dir);
                    s_dir = dir;
                }
            } else if (tid == 0) {
                uint32_t w;
                int spins = 0;
                while (!((w = __hip_atomic_load(&a.ctrl->chain_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) &
                         2u)) {
                    if (++spins > kSpinMax) {
                        atomicOr(&a.ctrl->err, ERR_SPIN);
                        w = 3u;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                s_dir = (int)(w & 1u);
            }
            __syncthreads();
            if (s_dir) return;
            clear_x = true;
        }
    }
    const int ntiles = (f + TILE - 1) / TILE;
    const int64_t chunk = 1ll << a.chunk_log2;
    int lmax = 0;
    // Tiles are taken in blockIdx order (tile = blockIdx.x + k * gridDim.x), so
    // every tile's predecessors belong to workgroups dispatched no later than
    // its own; the look-back wait is bounded in any case.
    for (int tile = blockIdx.x;; tile += gridDim.x) {
        if (tile >= ntiles) break;
        const int p0 = tile * TILE + tid * ITEMS;
        int32_t st[ITEMS], ln[ITEMS], jj[ITEMS];
        uint32_t xv[ITEMS];
        uint64_t lsum = 0, lcnt = 0;
        // Independent loads first (x indices, then both colptr ends, then x
        // values) so every thread has all its gathers in flight at once.
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) jj[i] = (p0 + i < f) ? a.x_idx[p0 + i] : -1;
        if (CHAIN && clear_x) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i)
                if (jj[i] >= 0 && jj[i] < a.n) a.xbits[jj[i] >> 5] = 0u;
        }
        bool bad = false;
        int32_t b0[ITEMS], b1[ITEMS];
        if (a.dcsc) {
            // DCSC: find column j among the stored ones through its chunk of
            // the column index (a few candidates), else it is empty.
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                b0[i] = b1[i] = 0;
                if (p0 + i >= f || jj[i] < 0 || jj[i] >= a.n) continue;
                const int c = jj[i] >> a.dc_shift;
                int32_t lo = a.dc_aux[c];
                const int32_t end = a.dc_aux[c + 1];
                int32_t hi = end;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (a.dc_jc[mid] < jj[i]) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < end && a.dc_jc[lo] == jj[i]) {
                    b0[i] = a.colptr[lo];
                    b1[i] = a.colptr[lo + 1];
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                // Clamp to a valid column so all gathers issue unconditionally.
                const int32_t jc = (jj[i] >= 0 && jj[i] < a.n) ? jj[i] : 0;
                b0[i] = a.colptr[jc];
                b1[i] = a.colptr[jc + 1];
            }
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const bool valid = p0 + i < f;
            const bool inr = jj[i] >= 0 && jj[i] < a.n;
            bad |= valid && !inr;
            st[i] = (valid && inr) ? b0[i] : 0;
            ln[i] = (valid && inr) ? b1[i] - b0[i] : 0;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) xv[i] = (p0 + i < f) ? x_value<XMODE>(a.x_val, p0 + i, jj[i]) : 0u;
        if (bad) atomicOr(&a.ctrl->err, ERR_X_RANGE);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            lmax = max(lmax, ln[i]);
            lsum += (uint64_t)ln[i];
            lcnt += ln[i] > 0 ? 1u : 0u;
        }
        uint64_t tile_sum, tile_cnt;
        const uint64_t tex_sum = block_exclusive_u64<BLOCK>(lsum, s_tmp, tile_sum);
        const uint64_t tex_cnt = block_exclusive_u64<BLOCK>(lcnt, s_tmp, tile_cnt);
        // The two chains run concurrently in waves 0 and 1.
        if (tid < kWave) {
            const uint64_t es = lookback(lb_sum, tile, tile_sum, &a.ctrl->err);
            if (tid == 0) s_excl_sum = es;
        } else if (tid < 2 * kWave) {
            const uint64_t ec = lookback(lb_cnt, tile, tile_cnt, &a.ctrl->err);
            if (tid == kWave) s_excl_cnt = ec;
        }
        __syncthreads();
        uint64_t off = s_excl_sum + tex_sum;
        uint64_t c = s_excl_cnt + tex_cnt;
        // A consistent prefix keeps every column slot below f (the tables'
        // size); an inconsistent look-back state must not store past them.
        bool lost = false;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (ln[i] > 0 && c >= (uint64_t)f) lost = true;
            if (ln[i] > 0 && c < (uint64_t)f) {
                a.cstart[c] = st[i];
                a.coff[c] = (int32_t)off;   // exact whenever the total is valid (<= nnz)
                a.cxv[c] = xv[i];
                if constexpr (BATCH) {
                    // vector of position p: the last b with xoff[b] <= p
                    const int64_t p = p0 + i;
                    int lo = 0, hi = a.nbatch - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_xoff[mid] <= p) lo = mid; else hi = mid - 1;
                    }
                    a.cxid[c] = lo;
                }
                for (int64_t k = ((int64_t)off + chunk - 1) >> a.chunk_log2;
                     (k << a.chunk_log2) < (int64_t)off + ln[i] && k < a.chunk_n; ++k)
                    a.chunk_col[k] = (int32_t)c;
            }
            if (ln[i] > 0) {
                off += (uint64_t)ln[i];
                c += 1;
            }
        }
        if (lost) atomicOr(&a.ctrl->err, ERR_SPIN);
        if (tile == ntiles - 1 && tid == BLOCK - 1) {
            if (off > (uint64_t)a.nnz || c > (uint64_t)f) {
                // Single vector: more products than stored entries means x
                // has duplicate indices.  Batched: more products than the
                // bucket storage holds.
                atomicOr(&a.ctrl->err, ERR_BUCKET_OVERFLOW);
                st_ctrl(&a.ctrl->W, 0);
                st_ctrl(&a.ctrl->fnz, 0);
                a.coff[0] = 0;
            } else {
                st_ctrl(&a.ctrl->W, (int32_t)off);
                st_ctrl(&a.ctrl->fnz, (int32_t)c);
                a.coff[c] = (int32_t)off;
            }
        }
        __syncthreads();
    }
    atomicMax(&s_max, lmax);
    __syncthreads();
    if (tid == 0 && s_max > 0) atomicMax(&a.ctrl->maxlen, s_max);
}

// ------------------------------------------------------------------ step (b)
// One workgroup turns chunks of C = BLOCK * ITEMS consecutive products into
// bucket runs.  Per chunk: (1) each thread gathers ITEMS products (row id,
// Mult value) and takes a rank in its bucket from an LDS histogram; (2) the
// histogram is prefix-summed in LDS and every bucket touched by the chunk
// reserves one slot range with a single global atomic; (3) the products are
// counting-sorted by bucket into LDS (this private buffer is the thread-local
// buffer of "Performance optimizations / Cache efficiency" on a workgroup
// scale) and (4) streamed out so consecutive lanes write consecutive slots.
// The LDS region holding the chunk's column table during (1) is reused as
// the sort buffer in (3).
//
// MODE 0: one vector, bucket = row >> tile_log2, bases from the row-count
// prefix of A.  Batched calls (x is several vectors; key = vector * nbx +
// bucket) run twice: MODE 1 only counts products per key (Algorithm 2's
// counting, per workgroup in LDS, then one global add per touched key) and
// MODE 2 scatters with bases from the exclusive scan of those counts.
enum { SC_SINGLE = 0, SC_COUNT = 1, SC_BATCH = 2 };

template <int BLOCK, int ITEMS, int SR, int MODE>
__global__ __launch_bounds__(BLOCK) void k_scatter(ScatterArgs a) {
    constexpr int C = BLOCK * ITEMS;
    extern __shared__ uint32_t lds_scatter[];
    const int nb = a.nb;
    int32_t* hist = reinterpret_cast<int32_t*>(lds_scatter);   // [nb] counts, then global slot base
    int32_t* loff = hist + nb;                                  // [nb] chunk-local bucket offsets
    uint32_t* region = lds_scatter + 2 * nb + 2;                // 8-byte aligned
    // Column table (phase 1): product offset of each column inside the chunk
    // (16 bits: the first column is cut to start at the chunk, the others
    // start inside it), its first entry in A and its x value.
    uint16_t* s_off = reinterpret_cast<uint16_t*>(region);      // [C+2]
    int32_t* s_start = reinterpret_cast<int32_t*>(s_off + (C + 2));
    uint32_t* s_xv = reinterpret_cast<uint32_t*>(s_start + (C + 1));
    int32_t* s_xid = reinterpret_cast<int32_t*>(s_xv + (C + 1)); // batched: vector of each column
    uint16_t* col_of = reinterpret_cast<uint16_t*>(s_xv + (MODE != SC_SINGLE ? 2 : 1) * (C + 1));   // [C] (phase 1)
    uint2* stage = reinterpret_cast<uint2*>(region);            // [C] sort buffer (phase 3)
    int32_t* skey = reinterpret_cast<int32_t*>(stage + C);      // batched: [C] key of each staged entry
    __shared__ int s_tmp[BLOCK / kWave + 1];
    const int tid = threadIdx.x;

    // The control words, loaded together: one round trip before the work
    // instead of one per word.
    const int dir = ld_ctrl(&a.ctrl->dir);
    const int errw = ld_ctrl(reinterpret_cast<const int32_t*>(&a.ctrl->err));
    const int W = ld_ctrl(&a.ctrl->W);
    const int fnz = ld_ctrl(&a.ctrl->fnz);
    if (MODE != SC_BATCH || a.xstride) {   // the first pass over the products of this call
        if (blockIdx.x == 0 && tid == 0) {
            st_ctrl_u(&a.ctrl->ticket_scan, 0u);
            st_ctrl(&a.ctrl->fnz_last, fnz);
            st_ctrl(&a.ctrl->W_last, W);
            st_ctrl(&a.ctrl->maxlen_last, atomicExch(&a.ctrl->maxlen, 0));
        }
        for (int i = blockIdx.x * BLOCK + tid; i < a.lb1_clear; i += gridDim.x * BLOCK) {
            a.lb1[i] = 0;
            a.lb1[a.lb1_n + i] = 0;
        }
    }

    if (a.gate && dir != 0) return;   // this BFS level runs pull
    // A failed look-back leaves the column tables inconsistent: scatter
    // nothing (the error is reported with the call's status).
    if (errw & (int32_t)ERR_SPIN) return;
    const int nchunks = (int)(((int64_t)W + C - 1) / C);
    if ((int)blockIdx.x >= nchunks) return;

    for (int i = tid; i < nb; i += BLOCK) hist[i] = 0;
    const int tl = a.tile_log2;

    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int q0 = c * C;
        const int cnt = min(C, W - q0);
        const int p0 = a.chunk_col[c];
        const int pend = (c + 1 < nchunks) ? a.chunk_col[c + 1] : fnz - 1;
        const int ncols = pend - p0 + 1;
        __syncthreads();  // the previous chunk is done with hist, loff and the shared region
        for (int k = tid; k < ncols; k += BLOCK) {
            const int off = a.coff[p0 + k] - q0;   // <= 0 only for k == 0
            const int st = a.cstart[p0 + k];
            s_off[k] = (uint16_t)(k == 0 ? 0 : off);
            s_start[k] = k == 0 ? st - off : st;
            s_xv[k] = a.cxv[p0 + k];
            if constexpr (MODE != SC_SINGLE) s_xid[k] = a.cxid[p0 + k];
        }
        __syncthreads();
        // Keys this chunk can touch: every bucket of a single call; in a
        // batch, the buckets of the vectors its columns belong to (columns
        // are in vector order), so the per-key loops below skip the other
        // vectors' keys.
        int klo = 0, khi = nb;
        if constexpr (MODE != SC_SINGLE) {
            klo = s_xid[0] * a.nbx;
            khi = min(nb, (s_xid[ncols - 1] + 1) * a.nbx);
        }

        // (1) gather + rank.  Column map: each thread finds the column of
        // its ITEMS consecutive products (one binary search, then a forward
        // walk) and records it in LDS.  Products are then taken strided
        // (item i of thread t is product i * BLOCK + t), so the lanes of a
        // wave read consecutive row ids and values: one request per cache
        // line instead of one per lane.  All row-id / value / mask loads are
        // issued together (indices clamped into range); ranks are taken in
        // LDS.
        int32_t row[ITEMS], rank[ITEMS], qq[ITEMS], xid[ITEMS];
        uint32_t xcol[ITEMS];
        {
            const int rq0 = tid * ITEMS;
            int lo = 0, hi = ncols - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= rq0) lo = mid; else hi = mid - 1;
            }
            int next = lo + 1 < ncols ? s_off[lo + 1] : 0x7fffffff;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int rq = rq0 + i;
                while (rq >= next) {
                    ++lo;
                    next = lo + 1 < ncols ? s_off[lo + 1] : 0x7fffffff;
                }
                if (rq < cnt) col_of[rq] = (uint16_t)lo;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int k = i * BLOCK + tid;
            const int lo = k < cnt ? col_of[k] : 0;
            qq[i] = k < cnt ? s_start[lo] + (k - s_off[lo]) : -1;
            xcol[i] = s_xv[lo];
            xid[i] = MODE != SC_SINGLE ? s_xid[lo] : 0;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) row[i] = a.rowids[qq[i] >= 0 ? qq[i] : 0];
        uint32_t val[ITEMS];
        if constexpr (MODE != SC_COUNT) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) val[i] = mult<SR>(a.values, qq[i] >= 0 ? qq[i] : 0, xcol[i]);
        }
        uint32_t mw[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            mw[i] = a.mask ? a.mask[(int64_t)xid[i] * a.mask_words + ((uint32_t)row[i] >> 5)] : 0u;
        // A product's bucket (key) is recomputed from its row where needed;
        // rank < 0 marks a product that is dropped (past the chunk, masked).
        auto bucket = [&](int i) { return MODE != SC_SINGLE ? xid[i] * a.nbx + (row[i] >> tl) : row[i] >> tl; };
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            rank[i] = -1;
            if (qq[i] >= 0 && (!a.mask || ((mw[i] >> (row[i] & 31)) & 1u) == (uint32_t)a.mask_keep))
                rank[i] = atomicAdd(&hist[bucket(i)], 1);
        }
        __syncthreads();
        if constexpr (MODE == SC_COUNT) {
            // Algorithm 2's per-bucket counts, accumulated over workgroups.
            for (int b = klo + tid; b < khi; b += BLOCK) {
                const int n = hist[b];
                if (n) {
                    atomicAdd(&a.kcount[b], n);
                    hist[b] = 0;
                }
            }
            continue;   // the loop head synchronises before hist is reused
        }
        // (2) chunk-local offsets and one slot reservation per touched
        // bucket.  With at most one bucket per thread (the usual case) the
        // reservation's round trip overlaps the counting sort (3), which
        // does not need it; its result is stored after the sort.
        int kept;
        if (nb <= BLOCK) {
            const int b = tid;
            const int n = b < nb ? hist[b] : 0;
            const int e = block_exclusive_i32<BLOCK>(n, s_tmp, kept);
            int base = 0, top = 0, g = 0;   // the bucket's slots are [base, top)
            if (b < nb) loff[b] = e;
            if (n > 0) {
                g = atomicAdd(&a.cursor[b], n);
                if (MODE == SC_BATCH && a.xstride == 0) {
                    base = a.kbase[b];
                    top = a.kbase[b + 1];
                } else {
                    const int r0 = (MODE == SC_BATCH ? b - (b / a.nbx) * a.nbx : b) << tl;
                    base = a.rcp[r0];
                    top = a.rcp[min(r0 + (1 << tl), a.m)];
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i)
                if (rank[i] >= 0) {
                    const int bi = bucket(i);
                    stage[loff[bi] + rank[i]] = make_uint2((uint32_t)row[i], val[i]);
                    if constexpr (MODE == SC_BATCH) skey[loff[bi] + rank[i]] = bi;
                }
            if (n > 0) {
                if (base + g + n > top) {
                    atomicOr(&a.ctrl->err, ERR_BUCKET_OVERFLOW);
                    hist[b] = -1;
                } else {
                    hist[b] = base + g;
                }
            }
            __syncthreads();
        } else {
            int carry = 0;
            for (int b0 = klo; b0 < khi; b0 += BLOCK) {
                const int b = b0 + tid;
                const int n = b < khi ? hist[b] : 0;
                int tot;
                const int e = block_exclusive_i32<BLOCK>(n, s_tmp, tot);
                if (b < khi) {
                    loff[b] = carry + e;
                    if (n > 0) {
                        int base, cap;
                        if (MODE == SC_BATCH && a.xstride == 0) {
                            base = a.kbase[b];
                            cap = a.kbase[b + 1] - base;
                        } else {   // row-count prefix (inside the vector's slice for fixed batched bases)
                            const int r0 = (MODE == SC_BATCH ? b - (b / a.nbx) * a.nbx : b) << tl;
                            base = a.rcp[r0];
                            cap = a.rcp[min(r0 + (1 << tl), a.m)] - base;
                        }
                        const int g = atomicAdd(&a.cursor[b], n);
                        if (g + n > cap) {
                            atomicOr(&a.ctrl->err, ERR_BUCKET_OVERFLOW);
                            hist[b] = -1;
                        } else {
                            hist[b] = base + g;
                        }
                    }
                }
                carry += tot;
            }
            kept = carry;
            __syncthreads();
            // (3) counting sort into the LDS buffer
#pragma unroll
            for (int i = 0; i < ITEMS; ++i)
                if (rank[i] >= 0) {
                    const int bi = bucket(i);
                    stage[loff[bi] + rank[i]] = make_uint2((uint32_t)row[i], val[i]);
                    if constexpr (MODE == SC_BATCH) skey[loff[bi] + rank[i]] = bi;
                }
            __syncthreads();
        }
        // (4) coalesced write-out of the bucket runs
        for (int t = tid; t < kept; t += BLOCK) {
            const uint2 e = stage[t];
            const int b = MODE == SC_BATCH ? skey[t] : (int)e.x >> tl;
            const int gb = hist[b];
            const int64_t slice = (MODE == SC_BATCH && a.xstride) ? (int64_t)(b / a.nbx) * a.xstride : 0;
            if (gb >= 0) a.buckets[slice + gb + (t - loff[b])] = e;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (rank[i] == 0) hist[bucket(i)] = 0;
    }
}

// ---------------------------------------------------------------- steps (c, d)
// One workgroup per bucket.  The bucket's rows [row0, row0 + T) get an LDS
// sparse accumulator (T values) and a T-bit touched bitmap.  The whole tile
// is initialised while the bucket's first entries are in flight (a store
// per row is far cheaper here than tracking first touches row by row);
// every entry then updates its row as described above, and the number of
// unique rows of Algorithm 1 step 2 is the population count of the bitmap.
// The unique count joins a decoupled look-back across buckets to give the
// bucket's offset in y (Algorithm 1, step 3) and the bitmap is walked in
// order, so y comes out ascending; the walk compacts rows through a small
// LDS list for coalesced y writes.
//
// Batched calls (BATCH): workgroup k merges key k = vector * nbx + bucket;
// the look-back runs over all keys, so y holds the vectors' results one
// after another (each ascending) and the first bucket of each vector
// publishes where its part starts (yoff).
template <int BLOCK, int ITEMS, int SR, bool BFS, bool BATCH>
__global__ __launch_bounds__(BLOCK) void k_merge(MergeArgs a) {
    extern __shared__ uint32_t lds_merge[];
    const int tl = a.tile_log2;
    const int T = 1 << tl;
    constexpr bool kWide = SR == SR_PLUS_TIMES;                      // fp64 cells
    uint32_t* spa = lds_merge;                                       // [T] cells of 4 or 8 bytes
    uint32_t* bm = spa + (kWide ? 2 * T : T);                        // [T/32]
    uint16_t* list = reinterpret_cast<uint16_t*>(bm + (T >> 5));     // [merge_list_cap(tl, kWide)]
    __shared__ int64_t s_excl;
    __shared__ int s_tmp[BLOCK / kWave + 1];
    const int tid = threadIdx.x;

    // Buckets in blockIdx order: a bucket's look-back predecessors belong to
    // workgroups dispatched no later than its own (the wait is bounded).
    if (a.gate && ld_ctrl(&a.ctrl->dir) != 0) return;   // this BFS level runs pull
    const int b = blockIdx.x;
    int xb = 0, bt = b;   // vector and bucket within it
    if constexpr (BATCH) {
        xb = b / a.nbx;
        bt = b - xb * a.nbx;
    }
    const int row0 = bt << tl;
    const int W = ld_ctrl(&a.ctrl->W);
    const int cnt_raw = ld_ctrl(&a.cursor[b]);
    int64_t base;
    int cap;
    if (BATCH && a.xstride == 0) {
        base = a.kbase[b];
        cap = a.kbase[b + 1] - a.kbase[b];
    } else {
        base = (BATCH ? (int64_t)xb * a.xstride : 0) + a.rcp[row0];
        cap = a.rcp[min(row0 + T, a.m)] - a.rcp[row0];
    }
    __syncthreads();
    // a tile with no entries still writes its (empty) words of y's bitmap
    auto zero_bits = [&]() {
        if (!BFS && !BATCH && a.y_bits) {
            const int zw = (min(T, a.m - row0) + 31) >> 5;
            for (int w = tid; w < zw; w += BLOCK) a.y_bits[(row0 >> 5) + w] = 0u;
        }
    };
    if (W == 0) {
        zero_bits();
        if (tid == 0) {
            if (BATCH && bt == 0) a.yoff[xb] = 0;
            if (b == a.nb - 1) {
                a.ctrl->nnz_y = 0;
                if (a.d_nnz_y) *a.d_nnz_y = 0;
                if (a.set_f) st_ctrl(&a.ctrl->f, 0);
                if (BATCH) a.yoff[a.nbatch] = 0;
            }
        }
        return;
    }
    const int rows = min(T, a.m - row0);
    if (cnt_raw == 0 && b != a.nb - 1 && (!BATCH || bt != 0)) {
        zero_bits();
        if (tid == 0) st_release64(&a.lb3[b], (b == 0 ? LB_INC : LB_AGG));
        return;
    }
    // Slots past the bucket's capacity exist only after an overflow
    // (duplicate x indices); never read past the bucket.
    const int cnt = min(cnt_raw, cap);
    const int nw = (rows + 31) >> 5;
    const bool small = cnt <= BLOCK * ITEMS;
    const bool sparse = cnt < rows / 8;   // plus-times: mark rows per entry, skip the ballot pass
    uint32_t rr[ITEMS], vv[ITEMS];
    if (small) {   // the whole bucket in registers: issue every load before the tile set-up
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int e = i * BLOCK + tid;
            const uint2 ent = a.buckets[base + (e < cnt ? e : 0)];
            rr[i] = e < cnt ? ent.x : 0xffffffffu;
            vv[i] = ent.y;
        }
    }
    for (int w = tid; w < nw; w += BLOCK) bm[w] = 0u;
    {
        // whole bitmap words of cells, 16 bytes per store
        uint4* spa4 = reinterpret_cast<uint4*>(spa);
        if constexpr (kWide) {
            const uint4 z = make_uint4(0u, 0x80000000u, 0u, 0x80000000u);   // two -0.0 doubles
            for (int q = tid; q < nw * 16; q += BLOCK) spa4[q] = z;
        } else {
            const uint32_t id = identity<SR>();
            for (int q = tid; q < nw * 8; q += BLOCK) spa4[q] = make_uint4(id, id, id, id);
        }
    }
    __syncthreads();
    bool bad = false;
    if (small) {
        bool ok[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            ok[i] = rr[i] != 0xffffffffu;
            rr[i] -= (uint32_t)row0;
            if (ok[i] && rr[i] >= (uint32_t)rows) {   // unwritten slot after an overflow
                ok[i] = false;
                bad = true;
            }
        }
        add_rows<SR, ITEMS>(rr, vv, ok, spa, bm, sparse);
    } else {
        constexpr int kBatch = 8;   // entries per thread in flight per step
        for (int e0 = 0; e0 < cnt; e0 += BLOCK * kBatch) {
            uint2 ent[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int e = e0 + u * BLOCK + tid;
                ent[u] = e < cnt ? a.buckets[base + e] : make_uint2(0xffffffffu, 0u);
            }
            uint32_t r[kBatch], v[kBatch];
            bool ok[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                r[u] = ent[u].x - (uint32_t)row0;
                v[u] = ent[u].y;
                ok[u] = e0 + u * BLOCK + tid < cnt;
                if (ok[u] && r[u] >= (uint32_t)rows) {
                    ok[u] = false;
                    bad = true;
                }
            }
            add_rows<SR, kBatch>(r, v, ok, spa, bm, sparse);
        }
    }
    if (bad) atomicOr(&a.ctrl->err, ERR_BUCKET_OVERFLOW);
    __syncthreads();
    if (kWide && !sparse) {
        touched_bits64<BLOCK>(spa, bm, rows);
        __syncthreads();
    }
    int pc = 0;
    for (int w = tid; w < nw; w += BLOCK) pc += __popc(bm[w]);
    int ucnt;
    (void)block_exclusive_i32<BLOCK>(pc, s_tmp, ucnt);
    if (tid < kWave) {
        const uint64_t e = lookback(a.lb3, b, (uint64_t)ucnt, &a.ctrl->err);
        if (tid == 0) {
            s_excl = (int64_t)e;
            if (BATCH && bt == 0) a.yoff[xb] = (int64_t)e;
            if (b == a.nb - 1) {
                const int64_t total = (int64_t)e + ucnt;
                a.ctrl->nnz_y = total;
                if (a.d_nnz_y) *a.d_nnz_y = total;
                if (a.set_f) st_ctrl(&a.ctrl->f, (int32_t)total);
                if (BATCH) a.yoff[a.nbatch] = total;
            }
        }
    }
    __syncthreads();
    const int64_t excl = s_excl;
    const int lvl = BFS ? ld_ctrl(&a.ctrl->level) : 0;
    int32_t* level = BFS ? ld_ctrl_ptr(&a.ctrl->bfs_level) : nullptr;
    int32_t* parent = BFS ? ld_ctrl_ptr(&a.ctrl->bfs_parent) : nullptr;
    uint32_t* visited = a.visited;
    if (BATCH && BFS) {
        level += (int64_t)xb * a.n_stride;
        if (parent) parent += (int64_t)xb * a.n_stride;
        visited += (int64_t)xb * a.mask_words;
    }

    // In-order walk of the bitmap: one word per thread per round, as many
    // words as the LDS list holds (the whole tile up to 16K rows).
    const int round_words = min(BLOCK, merge_list_cap(tl, kWide) >> 5);
    int64_t carry = 0;
    for (int w0 = 0; w0 < nw; w0 += round_words) {
        const int w = w0 + tid;
        const bool mine = tid < round_words && w < nw;
        const uint32_t bits = mine ? bm[w] : 0u;
        if (!BFS && !BATCH && a.y_bits && mine) a.y_bits[(row0 >> 5) + w] = bits;
        int tot;
        const int pos = block_exclusive_i32<BLOCK>(__popc(bits), s_tmp, tot);
        if (BFS && bits) visited[(row0 >> 5) + w] |= bits;
        uint32_t rest = bits;
        int k = 0;
        while (rest) {
            const int bitpos = __ffs(rest) - 1;
            rest &= rest - 1u;
            list[pos + k] = (uint16_t)((w << 5) + bitpos);
            ++k;
        }
        __syncthreads();
        for (int t = tid; t < tot; t += BLOCK) {
            const int r = list[t];
            const int64_t o = excl + carry + t;
            uint32_t v;
            if constexpr (kWide) v = __float_as_uint((float)reinterpret_cast<const double*>(spa)[r]);
            else v = spa[r];
            if (o < a.y_cap) {
                a.y_idx[o] = row0 + r;
                if (a.y_val) store_value<SR>(a.y_val, o, v);
            }
            if (BFS) {
                level[row0 + r] = lvl;
                if (parent) parent[row0 + r] = (int32_t)v;
            }
        }
        carry += tot;
        __syncthreads();
    }
}

}  // namespace

size_t merge_lds_bytes(int tile_log2, int semiring) {
    const bool wide = semiring == SR_PLUS_TIMES;
    const size_t T = size_t(1) << tile_log2;
    return T * (wide ? 8 : 4) + (T / 32) * 4 + size_t(merge_list_cap(tile_log2, wide)) * 2;
}

size_t scatter_lds_bytes(int nb, int chunk, bool batch) {
    // column table (+ the per-product column map) in phase 1, sort buffer in phase 3
    const size_t table = size_t(chunk + 2) * 2 + size_t(chunk + 1) * (batch ? 12 : 8) + size_t(chunk) * 2,
                 sortbuf = size_t(chunk) * (batch ? 12 : 8);
    return size_t(2 * nb + 2) * 4 + (table > sortbuf ? table : sortbuf);
}

template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <typename K, typename... Args>
static void launch_k(K kern, dim3 grid, dim3 block, size_t lds, hipStream_t s, const LaunchEvents* ev,
                     Args... args) {
    if (ev) hipExtLaunchKernelGGL(kern, grid, block, (uint32_t)lds, s, ev->start, ev->stop, 0, args...);
    else hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
}

template <int ITEMS, bool BATCH, bool CHAIN = false>
static hipError_t scan_mode(const ScanArgs& a, int grid, hipStream_t s, const LaunchEvents* ev) {
    switch (a.xmode) {
        case XV_BITS32:
            launch_k(k_scan<kScanBlock, ITEMS, XV_BITS32, BATCH, CHAIN>, dim3(grid), dim3(kScanBlock), 0, s, ev, a);
            break;
        case XV_INDEX:
            launch_k(k_scan<kScanBlock, ITEMS, XV_INDEX, BATCH, CHAIN>, dim3(grid), dim3(kScanBlock), 0, s, ev, a);
            break;
        case XV_U8:
            launch_k(k_scan<kScanBlock, ITEMS, XV_U8, BATCH, CHAIN>, dim3(grid), dim3(kScanBlock), 0, s, ev, a);
            break;
        case XV_TRUE:
            launch_k(k_scan<kScanBlock, ITEMS, XV_TRUE, BATCH, CHAIN>, dim3(grid), dim3(kScanBlock), 0, s, ev, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Frontier lengths known only on the device (BFS, PageRank) and batched
// calls use a fixed grid that loops over tiles; their tiles, and those of a
// host-known f too large for one narrow tile per workgroup, are 4x wider so
// a large frontier needs fewer look-back rounds.
hipError_t launch_scan(const ScanArgs& a, int grid, hipStream_t s, const LaunchEvents* ev) {
    if (a.xoff) {
        if (a.nbatch < 1 || a.nbatch > kMaxBatch || !a.cxid || !a.kcount) return hipErrorInvalidValue;
        return scan_mode<kScanItemsWide, true>(a, grid, s, ev);
    }
    if (a.chain) {
        if (!a.f_dev || !a.xbits || (a.chain == 2 && !a.sel)) return hipErrorInvalidValue;
        return scan_mode<kScanItemsWide, false, true>(a, grid, s, ev);
    }
    if (a.f_dev || a.wide) return scan_mode<kScanItemsWide, false>(a, grid, s, ev);
    return scan_mode<kScanItems, false>(a, grid, s, ev);
}

template <int BLOCK, int ITEMS, int SR, int MODE>
static hipError_t scatter_one(const ScatterArgs& a, int grid, hipStream_t s, const LaunchEvents* ev) {
    const size_t lds = scatter_lds_bytes(a.nb, BLOCK * ITEMS, MODE != SC_SINGLE);
    auto kern = k_scatter<BLOCK, ITEMS, SR, MODE>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    launch_k(kern, dim3(grid), dim3(BLOCK), lds, s, ev, a);
    return hipGetLastError();
}

template <int BLOCK, int ITEMS, int MODE>
static hipError_t scatter_sr(const ScatterArgs& a, int semiring, int grid, hipStream_t s, const LaunchEvents* ev) {
    if constexpr (MODE == SC_COUNT) return scatter_one<BLOCK, ITEMS, SR_MIN_SELECT2ND, MODE>(a, grid, s, ev);
    switch (semiring) {
        case SR_PLUS_TIMES: return scatter_one<BLOCK, ITEMS, SR_PLUS_TIMES, MODE>(a, grid, s, ev);
        case SR_MIN_SELECT2ND: return scatter_one<BLOCK, ITEMS, SR_MIN_SELECT2ND, MODE>(a, grid, s, ev);
        default: return scatter_one<BLOCK, ITEMS, SR_OR_AND, MODE>(a, grid, s, ev);
    }
}

bool scatter_shape_supported(int block, int items) {
    return (block == 256 && (items == 4 || items == 8 || items == 16)) ||
           (block == 512 && (items == 4 || items == 8)) || (block == 1024 && (items == 4 || items == 8));
}

template <int MODE>
static hipError_t scatter_shape(const ScatterArgs& a, int semiring, int block, int items, int grid, hipStream_t s,
                                const LaunchEvents* ev = nullptr) {
    if (block == 256) {
        if (items == 4) return scatter_sr<256, 4, MODE>(a, semiring, grid, s, ev);
        if (items == 8) return scatter_sr<256, 8, MODE>(a, semiring, grid, s, ev);
        if (items == 16) return scatter_sr<256, 16, MODE>(a, semiring, grid, s, ev);
    } else if (block == 512) {
        if (items == 4) return scatter_sr<512, 4, MODE>(a, semiring, grid, s, ev);
        if (items == 8) return scatter_sr<512, 8, MODE>(a, semiring, grid, s, ev);
    } else if (block == 1024) {
        if (items == 4) return scatter_sr<1024, 4, MODE>(a, semiring, grid, s, ev);
        if (items == 8) return scatter_sr<1024, 8, MODE>(a, semiring, grid, s, ev);
    }
    return hipErrorInvalidValue;
}

// Workgroups of one scatter instantiation a compute unit holds at once, as
// the runtime computes it from the kernel's registers, LDS and threads.
template <int BLOCK, int ITEMS, int SR, int MODE>
static int resident_one(size_t lds) {
    auto kern = k_scatter<BLOCK, ITEMS, SR, MODE>;
    if (allow_lds(kern, lds) != hipSuccess) return 1;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(kern), BLOCK, lds) !=
        hipSuccess)
        return 1;
    return n;
}

template <int BLOCK, int ITEMS, int MODE>
static int resident_sr(int semiring, size_t lds) {
    switch (semiring) {
        case SR_PLUS_TIMES: return resident_one<BLOCK, ITEMS, SR_PLUS_TIMES, MODE>(lds);
        case SR_MIN_SELECT2ND: return resident_one<BLOCK, ITEMS, SR_MIN_SELECT2ND, MODE>(lds);
        default: return resident_one<BLOCK, ITEMS, SR_OR_AND, MODE>(lds);
    }
}

template <int MODE>
static int resident_shape(int semiring, int block, int items, size_t lds) {
    if (block == 256) {
        if (items == 4) return resident_sr<256, 4, MODE>(semiring, lds);
        if (items == 8) return resident_sr<256, 8, MODE>(semiring, lds);
        if (items == 16) return resident_sr<256, 16, MODE>(semiring, lds);
    } else if (block == 512) {
        if (items == 4) return resident_sr<512, 4, MODE>(semiring, lds);
        if (items == 8) return resident_sr<512, 8, MODE>(semiring, lds);
    } else if (block == 1024) {
        if (items == 4) return resident_sr<1024, 4, MODE>(semiring, lds);
        if (items == 8) return resident_sr<1024, 8, MODE>(semiring, lds);
    }
    return 1;
}

int scatter_resident(int semiring, int block, int items, int nb, bool batch) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, bool>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    const auto key = std::make_tuple(dev, semiring, block, items, nb, batch);
    {
        std::lock_guard<std::mutex> g(mu);
        const auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const size_t lds = scatter_lds_bytes(nb, block * items, batch);
    int n = batch ? std::min(resident_shape<SC_BATCH>(semiring, block, items, lds),
                             resident_shape<SC_COUNT>(semiring, block, items, lds))
                  : resident_shape<SC_SINGLE>(semiring, block, items, lds);
    if (n < 1) n = 1;
    std::lock_guard<std::mutex> g(mu);
    cache[key] = n;
    return n;
}

hipError_t launch_scatter(const ScatterArgs& a, int semiring, int block, int items, int grid, hipStream_t s,
                          const LaunchEvents* ev) {
    return scatter_shape<SC_SINGLE>(a, semiring, block, items, grid, s, ev);
}

hipError_t launch_scatter_batch(const ScatterArgs& a, int semiring, int block, int items, int grid, bool count,
                                hipStream_t s) {
    if (!a.cxid || a.nbx < 1 || (count && !a.kcount) || (!count && !a.kbase && a.xstride == 0))
        return hipErrorInvalidValue;
    return count ? scatter_shape<SC_COUNT>(a, semiring, block, items, grid, s)
                 : scatter_shape<SC_BATCH>(a, semiring, block, items, grid, s);
}

template <int BLOCK, int SR, bool BFS, bool BATCH>
static hipError_t merge_one(const MergeArgs& a, hipStream_t s, const LaunchEvents* ev) {
    const size_t lds = merge_lds_bytes(a.tile_log2, SR);
    auto kern = k_merge<BLOCK, kMergeItems, SR, BFS, BATCH>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    launch_k(kern, dim3(a.nb), dim3(BLOCK), lds, s, ev, a);
    return hipGetLastError();
}

template <int BLOCK, bool BATCH>
static hipError_t merge_block(const MergeArgs& a, int semiring, bool bfs, hipStream_t s, const LaunchEvents* ev) {
    switch (semiring) {
        case SR_PLUS_TIMES:
            if (bfs) return hipErrorInvalidValue;
            return merge_one<BLOCK, SR_PLUS_TIMES, false, BATCH>(a, s, ev);
        case SR_MIN_SELECT2ND:
            return bfs ? merge_one<BLOCK, SR_MIN_SELECT2ND, true, BATCH>(a, s, ev)
                       : merge_one<BLOCK, SR_MIN_SELECT2ND, false, BATCH>(a, s, ev);
        default:
            return bfs ? merge_one<BLOCK, SR_OR_AND, true, BATCH>(a, s, ev)
                       : merge_one<BLOCK, SR_OR_AND, false, BATCH>(a, s, ev);
    }
}

template <bool BATCH>
static hipError_t merge_dispatch(const MergeArgs& a, int semiring, int block, bool bfs, hipStream_t s,
                                 const LaunchEvents* ev = nullptr) {
    if (block == 256) return merge_block<256, BATCH>(a, semiring, bfs, s, ev);
    if (block == 512) return merge_block<512, BATCH>(a, semiring, bfs, s, ev);
    if (block == 1024) return merge_block<1024, BATCH>(a, semiring, bfs, s, ev);
    return hipErrorInvalidValue;
}

hipError_t launch_merge(const MergeArgs& a, int semiring, int block, bool bfs, hipStream_t s,
                        const LaunchEvents* ev) {
    return merge_dispatch<false>(a, semiring, block, bfs, s, ev);
}

hipError_t launch_merge_batch(const MergeArgs& a, int semiring, int block, bool bfs, hipStream_t s) {
    if ((!a.kbase && a.xstride == 0) || !a.yoff || a.nbx < 1 || a.nbatch < 1 || (int64_t)a.nbx * a.nbatch != a.nb)
        return hipErrorInvalidValue;
    return merge_dispatch<true>(a, semiring, block, bfs, s);
}

}  // namespace spv
