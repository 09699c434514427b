// Pull (matrix-driven) direction: y(i) = Add over the stored entries A(i, j)
// of row i whose column j is selected by x.  This is the other class of
// SpMSpV algorithms in the paper's Background ("Classes of SpMSpV
// algorithms"): it touches every stored entry of the rows it scans, so its
// cost is O(m + nnz(A)) rather than the vector-driven O(df), and it wins when
// x is dense; switching between the two is the paper's stated future work
// (Conclusions).  Rows are read in CSR form: the transpose built at create,
// or A itself when the caller declares A symmetric.
//
// Three launches: k_pull_prep scatters x into a bitmap + dense values;
// k_pull walks a merge-path partition of (row ends + stored entries) so every
// workgroup gets the same number of steps whatever the row lengths; k_emit
// walks the result bitmap in order (decoupled look-back across workgroups),
// writes y ascending and restores the zeroed / identity state of the dense
// buffers for the next call.

#include "internal.h"

namespace spv {

namespace {

constexpr uint64_t LBP_AGG = 1ull << 62;
constexpr uint64_t LBP_INC = 2ull << 62;
constexpr uint64_t LBP_VAL = (1ull << 62) - 1;
constexpr int kSpinMaxP = 1 << 20;

__device__ __forceinline__ int32_t ldc(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t* ldc_ptr(int32_t* const* p) {
    return reinterpret_cast<int32_t*>(__hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT));
}

template <int SR>
__device__ __forceinline__ uint32_t ident() {
    if constexpr (SR == SR_PLUS_TIMES) return 0u;
    else if constexpr (SR == SR_MIN_SELECT2ND) return 0x7fffffffu;
    else return 0u;
}

template <int SR>
__device__ __forceinline__ uint32_t comb(uint32_t x, uint32_t y) {
    if constexpr (SR == SR_PLUS_TIMES) return __float_as_uint(__uint_as_float(x) + __uint_as_float(y));
    else if constexpr (SR == SR_MIN_SELECT2ND) return (uint32_t)min((int)x, (int)y);
    else return x | y;
}

template <int SR>
__device__ __forceinline__ void comb_global(uint32_t* cell, uint32_t v) {
    if constexpr (SR == SR_PLUS_TIMES) atomicAdd(reinterpret_cast<float*>(cell), __uint_as_float(v));
    else if constexpr (SR == SR_MIN_SELECT2ND) atomicMin(reinterpret_cast<int*>(cell), (int)v);
    else atomicOr(cell, v);
}

// ---------------------------------------------------------------- x -> dense
template <int XMODE>
__global__ __launch_bounds__(256) void k_pull_prep(PullArgs a) {
    if (a.gate && ldc(&a.ctrl->dir) != 1) return;   // this BFS level runs push
    const int f = a.f_dev ? ldc(a.f_dev) : a.f_host;
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.bump_level && f > 0) stc(&a.ctrl->level, ldc(&a.ctrl->level) + 1);
    // the emit look-back words of this call (the previous emit has finished)
    for (int i = blockIdx.x * 256 + threadIdx.x; i < a.emit_blocks; i += gridDim.x * 256) a.lbp[i] = 0;
    // after a pull level the x bitmap already holds this frontier (its emit
    // wrote it); the BFS pull reads vertex ids, not xdense
    if (a.chain && __hip_atomic_load(&a.ctrl->chain_ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    // Bitmap words are ORed once per run of lanes sharing a word (a sorted
    // frontier puts up to 32 consecutive lanes on one word, whose atomics
    // would otherwise serialise on one address).
    const int lane = threadIdx.x & 63;
    for (int base = blockIdx.x * 256; base < f; base += gridDim.x * 256) {
        const int p = base + threadIdx.x;
        const int32_t j = p < f ? a.x_idx[p] : -1;
        const bool inr = j >= 0 && j < a.n;
        if (p < f && !inr) atomicOr(&a.ctrl->err, ERR_X_RANGE);
        if (inr) {
            uint32_t v;
            if constexpr (XMODE == XV_BITS32) v = reinterpret_cast<const uint32_t*>(a.x_val)[p];
            else if constexpr (XMODE == XV_INDEX) v = (uint32_t)j;
            else if constexpr (XMODE == XV_U8) v = reinterpret_cast<const uint8_t*>(a.x_val)[p] ? 1u : 0u;
            else v = 1u;
            a.xdense[j] = v;
        }
        const uint32_t word = inr ? (uint32_t)j >> 5 : 0xffffffffu;
        uint32_t bits = inr ? 1u << (j & 31) : 0u;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t ow = (uint32_t)__shfl_down((int)word, d, 64);
            const uint32_t ob = (uint32_t)__shfl_down((int)bits, d, 64);
            if (lane + d < 64 && ow == word) bits |= ob;
        }
        const uint32_t prev = (uint32_t)__shfl_up((int)word, 1, 64);
        if (inr && (lane == 0 || prev != word)) atomicOr(&a.xbits[word], bits);
    }
}

// ------------------------------------------------------------- row walk
// Workgroup c covers merge-path diagonals [c*C, (c+1)*C) of the sequence
// "stored entries of row 0, end of row 0, entries of row 1, ...".  part[c] =
// rows ended before diagonal c*C (computed once per matrix), so the
// workgroup's stored entries are the contiguous range [q0, q1).
//   A: the entries are read coalesced (lane k of a pass takes entry q0 + k),
//      probed against the x bitmap and multiplied; products and hit bits go
//      to LDS.
//   B: each thread walks ITEMS consecutive diagonals, folding the products
//      of its rows from LDS; a row that starts and ends inside the thread is
//      final.
//   C: a block-wide segmented scan carries the open row of each thread into
//      the next, so a row split across threads is combined in registers; only
//      rows that cross a workgroup boundary take a global atomic.
//   D: result bits are ORed once per run of lanes sharing a bitmap word.
template <int SR>
struct Seg {   // open-segment state of the carry scan
    uint32_t v;
    bool hit, end;
};

template <int SR>
__device__ __forceinline__ Seg<SR> seg_comb(const Seg<SR>& l, const Seg<SR>& r) {
    if (r.end) return r;
    Seg<SR> o;
    o.end = l.end;
    o.hit = l.hit || r.hit;
    o.v = l.hit ? (r.hit ? comb<SR>(l.v, r.v) : l.v) : r.v;
    return o;
}

template <int SR>
__device__ __forceinline__ Seg<SR> seg_shfl_up(const Seg<SR>& s, int d) {
    Seg<SR> o;
    o.v = (uint32_t)__shfl_up((int)s.v, d, 64);
    const int fl = __shfl_up((int)s.hit | ((int)s.end << 1), d, 64);
    o.hit = fl & 1;
    o.end = (fl >> 1) & 1;
    return o;
}

// OR `bits` into ybits[word] once per run of lanes holding the same word
// (words are non-decreasing across lanes; 0xffffffff = nothing).
__device__ __forceinline__ void or_bits_wave(uint32_t* ybits, uint32_t word, uint32_t bits) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t ow = (uint32_t)__shfl_down((int)word, d, 64);
        const uint32_t ob = (uint32_t)__shfl_down((int)bits, d, 64);
        if (lane + d < 64 && ow == word) bits |= ob;
    }
    const uint32_t prev = (uint32_t)__shfl_up((int)word, 1, 64);
    if (word != 0xffffffffu && bits && (lane == 0 || prev != word)) atomicOr(&ybits[word], bits);
}

template <int BLOCK, int ITEMS, int SR>
__global__ __launch_bounds__(BLOCK) void k_pull(PullArgs a) {
    constexpr int C = BLOCK * ITEMS;
    constexpr int NW = BLOCK / 64;
    __shared__ int32_t s_re[C + 2];       // diagonal index of each row end touched by this workgroup
    __shared__ uint32_t s_prod[C];        // product of entry q0 + k (where its hit bit is set)
    __shared__ uint32_t s_hit[C / 32];
    __shared__ uint32_t s_wv[NW];
    __shared__ int s_wf[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (a.gate && ldc(&a.ctrl->dir) != 1) return;
    const int f = a.f_dev ? ldc(a.f_dev) : a.f_host;
    if (f <= 0) return;
    const int64_t total = (int64_t)a.m + a.nnz;
    const int64_t d0 = (int64_t)blockIdx.x * C;
    if (d0 >= total) return;
    const int64_t d1 = min(d0 + C, total);
    const int r0 = a.part[blockIdx.x];
    const int r1 = a.part[blockIdx.x + 1];
    const int rlast = min(r1, a.m - 1);
    for (int k = tid; k <= rlast - r0; k += BLOCK) s_re[k] = (r0 + k) + a.rowptr[r0 + k + 1];

    // A: products of the workgroup's entries
    const int64_t q0 = d0 - r0;
    const int ne = (int)((d1 - r1) - q0);
    {
        uint32_t cj[ITEMS];
        bool hv[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int k = i * BLOCK + tid;
            cj[i] = k < ne ? a.colids[q0 + k] : 0u;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int k = i * BLOCK + tid;
            hv[i] = k < ne && ((a.xbits[cj[i] >> 5] >> (cj[i] & 31)) & 1u);
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int k = i * BLOCK + tid;
            uint32_t pv = 0u;
            if (hv[i]) {
                if constexpr (SR == SR_PLUS_TIMES) {
                    const float av = a.values ? a.values[q0 + k] : 1.0f;
                    pv = __float_as_uint(__fmul_rn(av, __uint_as_float(a.xdense[cj[i]])));
                } else if constexpr (SR == SR_MIN_SELECT2ND) {
                    pv = a.xdense[cj[i]];
                } else {
                    const uint32_t av = a.values ? (a.values[q0 + k] != 0.0f ? 1u : 0u) : 1u;
                    pv = av & a.xdense[cj[i]];
                }
            }
            s_prod[k] = pv;
            const uint64_t bal = __ballot(hv[i]);
            if (lane == 0) s_hit[k >> 5] = (uint32_t)bal;
            else if (lane == 32) s_hit[k >> 5] = (uint32_t)(bal >> 32);
        }
    }
    __syncthreads();

    // B: this thread's diagonals [dt, dend)
    const int64_t dt = d0 + (int64_t)tid * ITEMS;
    const int nsteps = dt < d1 ? (int)(min(dt + ITEMS, d1) - dt) : 0;
    int lo = 0, hi = rlast - r0 + 1;   // rows ended before dt
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)s_re[mid] < dt) lo = mid + 1; else hi = mid;
    }
    int r = r0 + lo;
    int64_t q = dt - r;
    // the thread's first row began before the thread (false when it has no steps)
    const bool open0 = nsteps > 0 && r < a.m && q != a.rowptr[r];
    Seg<SR> own;             // the thread's trailing open segment (end = it saw a row end)
    own.v = ident<SR>();
    own.hit = false;
    own.end = false;
    int rowA = -1;           // first row ending here when it began before the thread
    uint32_t headv = ident<SR>();
    bool headhit = false;
    uint32_t wA = 0xffffffffu, bA = 0u, wB = 0xffffffffu, bB = 0u;   // result bits, at most two words
    auto mark = [&](int row) {
        const uint32_t w = (uint32_t)row >> 5, bit = 1u << (row & 31);
        if (wA == 0xffffffffu || wA == w) {
            wA = w;
            bA |= bit;
        } else {
            wB = w;
            bB |= bit;
        }
    };
    bool masked = r < a.m && a.mask && ((a.mask[r >> 5] >> (r & 31)) & 1u);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (i < nsteps && r < a.m) {
            const int64_t rend = (int64_t)s_re[r - r0] - r;   // rowptr[r + 1]
            if (q < rend) {
                const int k = (int)(q - q0);
                if (!masked && ((s_hit[k >> 5] >> (k & 31)) & 1u)) {
                    const uint32_t p = s_prod[k];
                    own.v = own.hit ? comb<SR>(own.v, p) : p;
                    own.hit = true;
                }
                ++q;
            } else {   // end of row r
                if (!own.end && open0) {
                    rowA = r;
                    headv = own.v;
                    headhit = own.hit;
                } else if (own.hit) {   // the row began and ended in this thread
                    a.ydense[r] = own.v;
                    mark(r);
                }
                own.end = true;
                own.v = ident<SR>();
                own.hit = false;
                ++r;
                masked = r < a.m && a.mask && ((a.mask[r >> 5] >> (r & 31)) & 1u);
            }
        }
    }

    // C: exclusive segmented scan of the threads' open segments
    Seg<SR> inc = own;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const Seg<SR> o = seg_shfl_up<SR>(inc, d);
        if (lane >= d) inc = seg_comb<SR>(o, inc);
    }
    if (lane == 63) {
        s_wv[wid] = inc.v;
        s_wf[wid] = (int)inc.hit | ((int)inc.end << 1);
    }
    __syncthreads();
    Seg<SR> carry;   // open segment arriving from the threads before this one
    carry.v = ident<SR>();
    carry.hit = false;
    carry.end = false;
    for (int w = 0; w < wid; ++w) {
        Seg<SR> ws;
        ws.v = s_wv[w];
        ws.hit = s_wf[w] & 1;
        ws.end = (s_wf[w] >> 1) & 1;
        carry = seg_comb<SR>(carry, ws);
    }
    {
        Seg<SR> prev = seg_shfl_up<SR>(inc, 1);
        if (lane > 0) carry = seg_comb<SR>(carry, prev);
    }
    // A row that began before the workgroup gets contributions from another
    // workgroup too: combine it atomically.  Only the workgroup's first row
    // can have begun before it.
    const bool first_mid = q0 > (int64_t)a.rowptr[r0];
    if (rowA >= 0) {
        const bool hit = carry.hit || headhit;
        if (hit) {
            const uint32_t v = carry.hit ? (headhit ? comb<SR>(carry.v, headv) : carry.v) : headv;
            if (rowA == r0 && first_mid) comb_global<SR>(&a.ydense[rowA], v);
            else a.ydense[rowA] = v;
            mark(rowA);
        }
    }
    // the open row at the workgroup's end continues in the next workgroup
    if (nsteps > 0 && dt + nsteps == d1 && r < a.m) {
        const Seg<SR> tail = own.end ? own : seg_comb<SR>(carry, own);
        if (tail.hit) {
            comb_global<SR>(&a.ydense[r], tail.v);
            mark(r);
        }
    }
    // D
    if (wA != 0xffffffffu && wB != 0xffffffffu && wB < wA) {   // keep the pair ordered
        const uint32_t tw = wA, tb = bA;
        wA = wB;
        bA = bB;
        wB = tw;
        bB = tb;
    }
    or_bits_wave(a.ybits, wA, bA);
    or_bits_wave(a.ybits, wB, bB);
}

// Bottom-up BFS step: one thread per row, unvisited rows only, stopping at
// the first selected column (or-and: the row is reached; min-select2nd with
// ascending column ids and x value = column id: the first hit is the
// minimum).  Four column ids and four bitmap probes are in flight at a time.
template <int SR, bool FIRST_HIT>
__global__ __launch_bounds__(256) void k_pull_bfs(PullArgs a) {
    if (a.gate && ldc(&a.ctrl->dir) != 1) return;
    const int f = a.f_dev ? ldc(a.f_dev) : a.f_host;
    if (f <= 0) return;
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * 256;
    for (int r0 = blockIdx.x * 256 + (threadIdx.x & ~63); r0 < a.m; r0 += stride) {
        const int r = r0 + lane;
        bool hit = false;
        uint32_t acc = ident<SR>();
        if (r < a.m && !(a.mask && ((a.mask[r >> 5] >> (r & 31)) & 1u))) {
            const int q1 = a.rowptr[r + 1];
            for (int q = a.rowptr[r]; q < q1; q += 4) {
                uint32_t j[4];
                bool in[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    in[u] = q + u < q1;
                    j[u] = in[u] ? a.colids[q + u] : 0u;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) in[u] = in[u] && ((a.xbits[j[u] >> 5] >> (j[u] & 31)) & 1u);
                bool stop = false;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (in[u] && !stop) {
                        const uint32_t t = SR == SR_MIN_SELECT2ND ? (a.x_index ? j[u] : a.xdense[j[u]]) : 1u;
                        acc = hit ? comb<SR>(acc, t) : t;
                        hit = true;
                        if (FIRST_HIT || SR == SR_OR_AND) stop = true;
                    }
                }
                if (stop) break;
            }
        }
        if (hit) a.ydense[r] = acc;
        const uint64_t hm = __ballot(hit);
        if (lane == 0 && (uint32_t)hm) atomicOr(&a.ybits[r0 >> 5], (uint32_t)hm);
        if (lane == 32 && (uint32_t)(hm >> 32)) atomicOr(&a.ybits[(r0 >> 5) + 1], (uint32_t)(hm >> 32));
    }
}

// -------------------------------------------------------------- emit y
// Walks ybits in order, kEmitWords words per workgroup, and writes y with a
// decoupled look-back for the offsets.  Resets ybits / ydense for the next
// call and clears the x bits this call set; in a direction-switching BFS it
// writes the new frontier over the x bits instead and leaves per-workgroup
// sums of its column lengths for the next level's decision.
constexpr int kEmitBlock = 256;
constexpr int kEmitWords = 1024;

__device__ uint64_t lookback_p(uint64_t* st, int tile, uint64_t agg, uint32_t* err) {
    const int lane = threadIdx.x & 63;
    if (tile == 0) {
        if (lane == 0) __hip_atomic_store(&st[0], LBP_INC | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    if (lane == 0) __hip_atomic_store(&st[tile], LBP_AGG | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    int base = tile - 1, spins = 0;
    for (;;) {
        const int idx = base - lane;
        const uint64_t w = idx >= 0 ? __hip_atomic_load(&st[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : LBP_INC;
        const uint64_t status = w >> 62;
        const uint64_t inc = __ballot(status == 2), emp = __ballot(status == 0);
        const uint64_t need = inc ? (((inc & (~inc + 1)) << 1) - 1) : ~0ull;
        if (emp & need) {
            if (++spins > kSpinMaxP) {
                if (lane == 0) atomicOr(err, ERR_SPIN);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint64_t v = ((need >> lane) & 1ull) ? (w & LBP_VAL) : 0ull;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        excl += v;
        if (inc) break;
        base -= 64;
    }
    if (lane == 0) __hip_atomic_store(&st[tile], LBP_INC | ((excl + agg) & LBP_VAL), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

template <int SR, bool BFS>
__global__ __launch_bounds__(kEmitBlock) void k_emit(PullArgs a) {
    __shared__ int s_tmp[kEmitBlock / 64 + 1];
    __shared__ uint16_t s_list[kEmitWords * 32];
    __shared__ int64_t s_excl;
    const int tid = threadIdx.x;
    if (a.gate && ldc(&a.ctrl->dir) != 1) return;
    const int f = a.f_dev ? ldc(a.f_dev) : a.f_host;
    const int nw = (a.m + 31) >> 5;
    const int w0 = blockIdx.x * kEmitWords;
    // Clear this call's x bits (every workgroup shares the work).  In a
    // direction-switching BFS (chain) every x bitmap word is overwritten with
    // the next frontier below instead (square A: the same words).
    if (!a.chain) {
        for (int p = blockIdx.x * kEmitBlock + tid; p < f; p += gridDim.x * kEmitBlock) {
            const int32_t j = a.x_idx[p];
            if (j >= 0 && j < a.n) a.xbits[j >> 5] = 0u;
        }
    }
    constexpr int PER = kEmitWords / kEmitBlock;
    uint32_t bits[PER];
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int w = w0 + tid * PER + k;
        bits[k] = w < nw ? a.ybits[w] : 0u;
        cnt += __popc(bits[k]);
        if (a.chain && w < nw) a.xbits[w] = bits[k];
    }
    // block exclusive scan of cnt
    const int lane = tid & 63, wid = tid >> 6;
    int x = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_tmp[wid] = x;
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int w = 0; w < kEmitBlock / 64; ++w) {
            const int t = s_tmp[w];
            s_tmp[w] = acc;
            acc += t;
        }
        s_tmp[kEmitBlock / 64] = acc;
    }
    __syncthreads();
    const int pos = s_tmp[wid] + x - cnt;
    const int tot = s_tmp[kEmitBlock / 64];
    if (tid < 64) {
        const uint64_t e = lookback_p(a.lbp, blockIdx.x, (uint64_t)tot, &a.ctrl->err);
        if (tid == 0) {
            s_excl = (int64_t)e;
            if (blockIdx.x == gridDim.x - 1) {
                const int64_t total = (int64_t)e + tot;
                a.ctrl->nnz_y = total;
                if (a.d_nnz_y) *a.d_nnz_y = total;
                if (a.set_f) stc(&a.ctrl->f, (int32_t)total);
            }
        }
    }
    __syncthreads();
    const int64_t excl = s_excl;
    const int lvl = BFS ? ldc(&a.ctrl->level) : 0;
    int32_t* const level = BFS ? ldc_ptr(&a.ctrl->bfs_level) : nullptr;
    int32_t* const parent = BFS ? ldc_ptr(&a.ctrl->bfs_parent) : nullptr;
    // Rows of this workgroup's words go to an LDS list in order, then every
    // thread writes list entries t, t + block, ...: consecutive lanes write
    // consecutive y slots (coalesced) and increasing rows.
    int c = pos;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int wl = tid * PER + k;
        uint32_t b = bits[k];
        if (b) {
            a.ybits[w0 + wl] = 0u;
            if (BFS) a.visited[w0 + wl] |= b;
        }
        while (b) {
            const int bit = __ffs(b) - 1;
            b &= b - 1u;
            s_list[c++] = (uint16_t)((wl << 5) + bit);
        }
    }
    __syncthreads();
    int64_t csum = 0;   // chain: column lengths of this workgroup's new frontier vertices
    int cmax = 0, cnz = 0;
    for (int t = tid; t < tot; t += kEmitBlock) {
        const int r = (w0 << 5) + s_list[t];
        if (a.chain) {
            const int d = a.colptr[r + 1] - a.colptr[r];
            csum += d;
            cmax = max(cmax, d);
            cnz += d > 0 ? 1 : 0;
        }
        const uint32_t v = a.ydense[r];
        a.ydense[r] = ident<SR>();
        const int64_t o = excl + t;
        if (o < a.y_cap) {
            a.y_idx[o] = r;
            if (a.y_val) {
                if (SR == SR_OR_AND) reinterpret_cast<uint8_t*>(a.y_val)[o] = (uint8_t)(v != 0u);
                else reinterpret_cast<uint32_t*>(a.y_val)[o] = v;
            }
        }
        if (BFS) {
            level[r] = lvl;
            if (parent) parent[r] = (int32_t)v;
        }
    }
    if (a.chain) {   // this workgroup's sums, read by the next level's scan (a later kernel)
        __shared__ int64_t s_sum[kEmitBlock / 64];
        __shared__ int s_mx[kEmitBlock / 64], s_nz[kEmitBlock / 64];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            csum += __shfl_xor(csum, d, 64);
            cmax = max(cmax, __shfl_xor(cmax, d, 64));
            cnz += __shfl_xor(cnz, d, 64);
        }
        if (lane == 0) {
            s_sum[wid] = csum;
            s_mx[wid] = cmax;
            s_nz[wid] = cnz;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < kEmitBlock / 64; ++w) {
                csum += s_sum[w];
                cmax = max(cmax, s_mx[w]);
                cnz += s_nz[w];
            }
            a.chain_part[2 * blockIdx.x] = csum;
            a.chain_part[2 * blockIdx.x + 1] = ((int64_t)cmax << 32) | (uint32_t)cnz;
            if (blockIdx.x == 0) __hip_atomic_store(&a.ctrl->chain_ready, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // the look-back words of this call are cleared by the next k_pull_prep
}

__global__ void k_lbp_clear(uint64_t* lbp, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) lbp[i] = 0;
}

__global__ void k_fill32(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// part[c] = rows ended before diagonal c*C of the (row ends + entries) merge path.
__global__ void k_pull_partition(const int32_t* rowptr, int32_t m, int64_t nnz, int C, int32_t* part, int nparts) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nparts; c += gridDim.x * blockDim.x) {
        const int64_t d = min((int64_t)c * C, (int64_t)m + nnz);
        // smallest r in [0, m] with r + rowptr[r + 1] >= d (row r's end token at or after d)
        int lo = 0, hi = m;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((int64_t)mid + rowptr[mid + 1] < d) lo = mid + 1; else hi = mid;
        }
        part[c] = lo;
    }
}

// Transpose: CSR column ids / values from CSC, slot order within a row is
// the order of atomic arrival.
__global__ void k_transpose(const int32_t* colptr, const int32_t* rowids, const float* values, int32_t n,
                            const int32_t* rowptr, int32_t* cursor, int32_t* colids, float* tvalues) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        for (int q = colptr[j]; q < colptr[j + 1]; ++q) {
            const int32_t i = rowids[q];
            const int32_t slot = rowptr[i] + atomicAdd(&cursor[i], 1);
            colids[slot] = j;
            if (tvalues) tvalues[slot] = values ? values[q] : 1.0f;
        }
    }
}

// Row ids ascending inside every column (enables the first-hit exit of the
// pull min-select2nd BFS on a symmetric matrix).
__global__ void k_check_sorted(const int32_t* colptr, const int32_t* rowids, int32_t n, uint32_t* unsorted) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        for (int q = colptr[j] + 1; q < colptr[j + 1]; ++q)
            if (rowids[q] <= rowids[q - 1]) {
                atomicOr(unsorted, 1u);
                break;
            }
}

}  // namespace

hipError_t launch_pull(const PullArgs& a, int semiring, int xmode, bool bfs, bool early, bool rowwise,
                       hipStream_t s) {
    if (rowwise && semiring == SR_PLUS_TIMES) return hipErrorInvalidValue;
    int64_t fg = (a.f_host + 255) / 256 + 1;
    if (a.f_dev || fg > 512) fg = 512;
    const int f_grid = (int)fg;
    switch (xmode) {
        case XV_BITS32: hipLaunchKernelGGL(k_pull_prep<XV_BITS32>, dim3(f_grid), dim3(256), 0, s, a); break;
        case XV_INDEX: hipLaunchKernelGGL(k_pull_prep<XV_INDEX>, dim3(f_grid), dim3(256), 0, s, a); break;
        case XV_U8: hipLaunchKernelGGL(k_pull_prep<XV_U8>, dim3(f_grid), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(k_pull_prep<XV_TRUE>, dim3(f_grid), dim3(256), 0, s, a); break;
    }
    if (rowwise) {
        // bottom-up step: one thread per row, first-hit exit
        const dim3 gb((a.m + 255) / 256 < 2048 ? (a.m + 255) / 256 : 2048), bb(256);
        if (semiring == SR_MIN_SELECT2ND) {
            if (early) hipLaunchKernelGGL((k_pull_bfs<SR_MIN_SELECT2ND, true>), gb, bb, 0, s, a);
            else hipLaunchKernelGGL((k_pull_bfs<SR_MIN_SELECT2ND, false>), gb, bb, 0, s, a);
        } else {
            hipLaunchKernelGGL((k_pull_bfs<SR_OR_AND, true>), gb, bb, 0, s, a);
        }
    } else {   // merge-path walk over every row (no early exit: each row's full fold)
        const dim3 g(a.pull_blocks), b(kPullBlock);
        switch (semiring) {
            case SR_PLUS_TIMES: hipLaunchKernelGGL((k_pull<kPullBlock, kPullItems, SR_PLUS_TIMES>), g, b, 0, s, a); break;
            case SR_MIN_SELECT2ND:
                hipLaunchKernelGGL((k_pull<kPullBlock, kPullItems, SR_MIN_SELECT2ND>), g, b, 0, s, a);
                break;
            default: hipLaunchKernelGGL((k_pull<kPullBlock, kPullItems, SR_OR_AND>), g, b, 0, s, a); break;
        }
    }
    const dim3 ge(a.emit_blocks), be(kEmitBlock);
    switch (semiring) {
        case SR_PLUS_TIMES: hipLaunchKernelGGL((k_emit<SR_PLUS_TIMES, false>), ge, be, 0, s, a); break;
        case SR_MIN_SELECT2ND:
            if (bfs) hipLaunchKernelGGL((k_emit<SR_MIN_SELECT2ND, true>), ge, be, 0, s, a);
            else hipLaunchKernelGGL((k_emit<SR_MIN_SELECT2ND, false>), ge, be, 0, s, a);
            break;
        default:
            if (bfs) hipLaunchKernelGGL((k_emit<SR_OR_AND, true>), ge, be, 0, s, a);
            else hipLaunchKernelGGL((k_emit<SR_OR_AND, false>), ge, be, 0, s, a);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_clear_u64(uint64_t* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lbp_clear, dim3(64), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_ident(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill32, dim3(2048), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

int pull_emit_blocks(int32_t m) { return ((m + 31) / 32 + kEmitWords - 1) / kEmitWords; }
int pull_blocks(int32_t m, int64_t nnz) { return (int)(((int64_t)m + nnz + kPullChunk - 1) / kPullChunk); }

hipError_t launch_pull_setup(const int32_t* colptr, const int32_t* rowids, const float* values, int32_t m,
                             int32_t n, int64_t nnz, const int32_t* rowptr, int32_t* cursor, int32_t* colids,
                             float* tvalues, int32_t* part, uint32_t* unsorted, hipStream_t s) {
    if (colids) {
        hipLaunchKernelGGL(k_transpose, dim3(1024), dim3(256), 0, s, colptr, rowids, values, n, rowptr, cursor, colids,
                           tvalues);
    } else if (unsorted) {
        hipLaunchKernelGGL(k_check_sorted, dim3(1024), dim3(256), 0, s, colptr, rowids, n, unsorted);
    }
    const int nparts = pull_blocks(m, nnz) + 1;
    hipLaunchKernelGGL(k_pull_partition, dim3((nparts + 255) / 256), dim3(256), 0, s, colids ? rowptr : colptr, m,
                       nnz, kPullChunk, part, nparts);
    return hipGetLastError();
}

}  // namespace spv
