// Deterministic plus-times multiply.  y(i) is the fp32 sum of row i's
// products, each rounded to fp32 (Mult), added one at a time in product
// order: x order, then the column's storage order -- the order in which
// Algorithm 1 forms the products.  Its bits depend on the input alone, not on
// bucket counts, workgroup counts or the timing of atomics.
//   k_det_gather   product w -> (row, RN32(a * x)) at list position w; the
//                  scan's column tables give each product's column.
//   radix passes   a stable LSD sort of that list by row, digits of up to
//                  11 bits: per-block digit counts, their exclusive scan in
//                  digit-major order (Algorithm 2's count matrix: every
//                  (digit, block) run gets its position), then each block
//                  writes its entries at those positions, ranked stably
//                  (wave ballots, waves in order, rounds in order).
//   k_det_heads / k_det_fold  every row's products now form one run in
//                  product order; the run's first entry folds it
//                  sequentially and writes y at the run's ordinal, so y is
//                  ascending.
// A product whose row the mask removes carries row m and sorts after every
// real row; it is never written.

#include "device_ops.h"

namespace spv {

namespace {

constexpr int kGatherBlock = 256;
constexpr int kMaxDigits = 1 << kDetMaxDigitBits;
constexpr int kDetWaves = kDetBlock / kWave;

__global__ __launch_bounds__(kGatherBlock) void k_det_gather(DetArgs a, uint2* list) {
    extern __shared__ int32_t s_off[];   // coff of the chunk's columns (chunk + 2 entries at most)
    const int W = ld_ctrl(&a.ctrl->W);
    const int fnz = ld_ctrl(&a.ctrl->fnz);
    // The per-call bookkeeping the bucket scatter does on the other paths:
    // the scan's statistics, and its look-back words cleared for the next call.
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st_ctrl_u(&a.ctrl->ticket_scan, 0u);
        st_ctrl(&a.ctrl->maxlen_last, atomicExch(&a.ctrl->maxlen, 0));
        st_ctrl(&a.ctrl->fnz_last, fnz);
        st_ctrl(&a.ctrl->W_last, W);
    }
    for (int i = blockIdx.x * kGatherBlock + threadIdx.x; i < a.lb1_clear; i += gridDim.x * kGatherBlock) {
        a.lb1[i] = 0;
        a.lb1[a.lb1_n + i] = 0;
    }
    // a failed look-back leaves the column tables inconsistent: write
    // nothing (the error is reported with the call's status)
    if (ld_ctrl(reinterpret_cast<const int32_t*>(&a.ctrl->err)) & (int32_t)ERR_SPIN) return;
    const int64_t chunk = int64_t(1) << a.chunk_log2;
    const int64_t w0 = (int64_t)blockIdx.x << a.chunk_log2;
    if (w0 >= W) return;
    const int64_t w1 = w0 + chunk < W ? w0 + chunk : (int64_t)W;
    // chunk_col[k] is the column holding product k * chunk, so the chunk's
    // last product lies in a column no later than chunk_col[k + 1]
    const int c_lo = a.chunk_col[blockIdx.x];
    const int c_hi = w1 < W ? a.chunk_col[blockIdx.x + 1] : fnz - 1;
    const int ncol = c_hi - c_lo + 1;
    for (int i = threadIdx.x; i <= ncol; i += kGatherBlock) s_off[i] = a.coff[c_lo + i];
    __syncthreads();
    for (int64_t w = w0 + threadIdx.x; w < w1; w += kGatherBlock) {
        int lo = 0, hi = ncol - 1;   // the last column starting at or before w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        const int c = c_lo + lo;
        const int64_t q = (int64_t)a.cstart[c] + (w - s_off[lo]);
        int32_t row = a.rowids[q];
        const float av = a.values ? a.values[q] : 1.0f;
        const float t = __fmul_rn(av, __uint_as_float(a.cxv[c]));
        if (a.mask && ((a.mask[row >> 5] >> (row & 31)) & 1u) != (uint32_t)a.mask_keep) row = a.m;
        list[w] = make_uint2((uint32_t)row, __float_as_uint(t));
    }
}

__global__ __launch_bounds__(kDetBlock) void k_det_hist(DetArgs a, const uint2* in, int shift, int dbits) {
    __shared__ int h[kMaxDigits];
    const int nd = 1 << dbits;
    for (int d = threadIdx.x; d < nd; d += kDetBlock) h[d] = 0;
    __syncthreads();
    const int W = ld_ctrl(&a.ctrl->W);
    const int64_t base = (int64_t)blockIdx.x * kDetTile;
#pragma unroll 4
    for (int i = 0; i < kDetItems; ++i) {
        const int64_t e = base + i * kDetBlock + threadIdx.x;
        if (e < W) atomicAdd(&h[(in[e].x >> shift) & (uint32_t)(nd - 1)], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < nd; d += kDetBlock) a.counts[(int64_t)d * a.nblk + blockIdx.x] = h[d];
    if (blockIdx.x == 0 && threadIdx.x == 0) a.counts[(int64_t)nd * a.nblk] = 0;
}

__global__ __launch_bounds__(kDetBlock) void k_det_scatter(DetArgs a, const uint2* in, uint2* out, int shift,
                                                           int dbits) {
    __shared__ int s_run[kMaxDigits];             // next position of each digit's run
    __shared__ int s_wc[kDetWaves][kMaxDigits];   // this round's count per wave and digit
    const int nd = 1 << dbits;
    const int W = ld_ctrl(&a.ctrl->W);
    const int64_t base = (int64_t)blockIdx.x * kDetTile;
    if (base >= W) return;
    for (int d = threadIdx.x; d < nd; d += kDetBlock) {
        s_run[d] = a.counts[(int64_t)d * a.nblk + blockIdx.x];
        for (int w = 0; w < kDetWaves; ++w) s_wc[w][d] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int r = 0; r < kDetItems; ++r) {
        const int64_t e = base + r * kDetBlock + threadIdx.x;
        const bool valid = e < W;
        uint2 it = make_uint2(0u, 0u);
        int d = 0;
        if (valid) {
            it = in[e];
            d = (int)((it.x >> shift) & (uint32_t)(nd - 1));
        }
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
}

__global__ __launch_bounds__(kDetBlock) void k_det_heads(DetArgs a, const uint2* list) {
    __shared__ int s_tmp[kDetWaves + 1];
    const int W = ld_ctrl(&a.ctrl->W);
    const int64_t base = (int64_t)blockIdx.x * kDetTile;
    // every row and its predecessor's first, then the comparisons
    uint32_t rw[kDetItems], pv[kDetItems];
#pragma unroll
    for (int i = 0; i < kDetItems; ++i) {
        const int64_t e = base + i * kDetBlock + threadIdx.x;
        rw[i] = e < W ? list[e].x : ~0u;
        pv[i] = (e < W && e > 0) ? list[e - 1].x : ~0u;
    }
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < kDetItems; ++i) {
        const int64_t e = base + i * kDetBlock + threadIdx.x;
        if (e < W && rw[i] < (uint32_t)a.m && (e == 0 || pv[i] != rw[i])) ++cnt;
    }
    int total;
    block_exclusive_i32<kDetBlock>(cnt, s_tmp, total);
    if (threadIdx.x == 0) a.counts[blockIdx.x] = total;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.counts[a.nblk] = 0;
}

// The block's kDetTile entries are staged in LDS.  (1) Heads (first entry
// of each row's run) get their output ordinals from wave ballots and one
// table of per-round, per-wave head counts; (2) each thread folds its own
// heads' runs in order from LDS (a run that reaches the block's end goes on
// from global memory), with no further barrier, so a long run delays only
// its own thread.  Past kDetShortRun entries after its head a run is handed
// to k_det_fold_long.
__global__ __launch_bounds__(kDetBlock) void k_det_fold(DetArgs a, const uint2* list) {
    __shared__ uint2 s_e[kDetTile];
    __shared__ uint64_t s_bal[kDetItems][kDetWaves];   // heads of each round, per wave
    __shared__ int s_nlong;
    __shared__ uint32_t s_prev;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int W = ld_ctrl(&a.ctrl->W);
    if (blockIdx.x == 0 && tid == 0) {
        const int64_t total = a.counts[a.nblk];
        __hip_atomic_store(&a.ctrl->nnz_y, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a.d_nnz_y) *a.d_nnz_y = total;
    }
    const int64_t base = (int64_t)blockIdx.x * kDetTile;
    if (base >= W) {
        if (tid == 0) a.long_count[blockIdx.x] = 0;
        return;
    }
    const int n_in = (int)min((int64_t)kDetTile, (int64_t)W - base);
#pragma unroll
    for (int r = 0; r < kDetItems; ++r) {
        const int i = r * kDetBlock + tid;
        if (i < n_in) s_e[i] = list[base + i];
    }
    if (tid == 0) {
        s_nlong = 0;
        s_prev = base > 0 ? list[base - 1].x : ~0u;
    }
    __syncthreads();
    // (1) item r of thread t is entry r * kDetBlock + t
    uint32_t heads = 0;   // bit r: item r is a head
#pragma unroll
    for (int r = 0; r < kDetItems; ++r) {
        const int i = r * kDetBlock + tid;
        bool head = false;
        if (i < n_in) {
            const uint32_t row = s_e[i].x;
            const uint32_t prev = i == 0 ? s_prev : s_e[i - 1].x;
            head = row < (uint32_t)a.m && (base + i == 0 || prev != row);
        }
        const uint64_t bal = __ballot(head);
        if (lane == 0) s_bal[r][wave] = bal;
        heads |= head ? (1u << r) : 0u;
    }
    __syncthreads();
    // (2) folds, one add at a time in entry order; a head's ordinal is the
    // heads of earlier rounds, of lower waves in its round and of lower lanes
    // in its wave
    int64_t run = a.counts[blockIdx.x];
    const uint64_t lower = (1ull << lane) - 1ull;
#pragma unroll 1
    for (int r = 0; r < kDetItems; ++r) {
        int64_t p = run;
        for (int w = 0; w < kDetWaves; ++w) {
            const uint64_t bw = s_bal[r][w];
            run += __popcll(bw);
            if (w < wave) p += __popcll(bw);
            else if (w == wave) p += __popcll(bw & lower);
        }
        if (!((heads >> r) & 1u)) continue;
        const int i = r * kDetBlock + tid;
        const uint32_t row = s_e[i].x;
        float acc = __uint_as_float(s_e[i].y);
        bool more = true;
        const int64_t qlim = base + i + kDetShortRun + 1;   // the short fold's end
        const int64_t qend = min((int64_t)W, qlim);
        const int64_t lend = min(qend, base + n_in);
        int64_t q = base + i + 1;
        for (; more && q < lend; q += 8) {   // from LDS, eight reads ahead of the adds
            uint2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = q + u < lend ? s_e[q + u - base] : make_uint2(~0u, 0u);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (q + u < lend) {
                    more = more && v[u].x == row;
                    if (more) acc = __fadd_rn(acc, __uint_as_float(v[u].y));
                }
            }
        }
        if (more) q = lend;
        for (; more && q < qend; q += 8) {   // past the block: from global memory
            uint2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = q + u < qend ? list[q + u] : make_uint2(~0u, 0u);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (q + u < qend) {
                    more = more && v[u].x == row;
                    if (more) acc = __fadd_rn(acc, __uint_as_float(v[u].y));
                }
            }
        }
        if (more) q = qend;
        const bool longrun = more && q == qlim && q < W &&
                             (q - base < n_in ? s_e[q - base].x : list[q].x) == row;
        if (longrun) {
            // more than kDetShortRun + 1 entries, so runs starting in one
            // block are that far apart and at most kDetLongPerBlock start here
            const int slot = atomicAdd(&s_nlong, 1);
            if (slot < kDetLongPerBlock)
                a.long_runs[(int64_t)blockIdx.x * kDetLongPerBlock + slot] =
                    make_int4((int)row, (int)__float_as_uint(acc), (int)q, (int)p);
            else
                atomicOr(&a.ctrl->err, ERR_SPIN);   // not reached (see above)
        } else if (p < a.y_cap) {
            a.y_idx[p] = (int32_t)row;
            if (a.y_val) a.y_val[p] = acc;
        }
    }
    __syncthreads();
    if (tid == 0) a.long_count[blockIdx.x] = min(s_nlong, kDetLongPerBlock);
}

// One wave per long run.  The wave keeps kLongDepth steps of 64 consecutive
// entries in flight (one coalesced load per step, issued kLongDepth steps
// ahead); each step's values go to the wave's LDS row and one lane adds them
// in order from there, so the run costs its dependent adds and little more.
// (Folding through lane reads cost about 90 cycles per entry, a 16K-entry
// hub row 0.6 ms; one thread per run with sixteen loads ahead left the
// memory latency exposed.)
constexpr int kLongDepth = 4;

__global__ __launch_bounds__(kDetBlock) void k_det_fold_long(DetArgs a, const uint2* list) {
    __shared__ __attribute__((aligned(16))) float s_v[kDetWaves][kWave];
    const int W = ld_ctrl(&a.ctrl->W);
    const int nblk_used = (W + kDetTile - 1) / kDetTile;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int nwaves = gridDim.x * kDetWaves;
    const int64_t npairs = (int64_t)nblk_used * kDetLongPerBlock;
    auto load = [&](int64_t k) { return k + lane < W ? list[k + lane] : make_uint2(~0u, 0u); };
    for (int64_t pr = blockIdx.x * kDetWaves + wv; pr < npairs; pr += nwaves) {
        const int b = (int)(pr / kDetLongPerBlock), slot = (int)(pr % kDetLongPerBlock);
        if (slot >= a.long_count[b]) continue;
        const int4 rec = a.long_runs[pr];
        const uint32_t row = (uint32_t)rec.x;
        float acc = __uint_as_float((uint32_t)rec.y);
        int64_t k = rec.z;
        uint2 ring[kLongDepth];
#pragma unroll
        for (int d = 0; d < kLongDepth; ++d) ring[d] = load(k + (int64_t)d * kWave);
        bool more = true;
        while (more) {
            const uint2 v = ring[0];
#pragma unroll
            for (int d = 0; d + 1 < kLongDepth; ++d) ring[d] = ring[d + 1];
            ring[kLongDepth - 1] = load(k + (int64_t)kLongDepth * kWave);
            const uint64_t match = __ballot(v.x == row);
            // entries of the run in this step: the lanes before the first mismatch
            const int n = (~match == 0ull) ? kWave : __ffsll((unsigned long long)~match) - 1;
            s_v[wv][lane] = __uint_as_float(v.y);
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {
                // all 64 values into registers first, then the dependent adds
                float4 q[kWave / 4];
#pragma unroll
                for (int j = 0; j < kWave / 4; ++j) q[j] = *reinterpret_cast<const float4*>(&s_v[wv][4 * j]);
#pragma unroll
                for (int j = 0; j < kWave / 4; ++j) {
                    if (4 * j < n) acc = __fadd_rn(acc, q[j].x);
                    if (4 * j + 1 < n) acc = __fadd_rn(acc, q[j].y);
                    if (4 * j + 2 < n) acc = __fadd_rn(acc, q[j].z);
                    if (4 * j + 3 < n) acc = __fadd_rn(acc, q[j].w);
                }
            }
            __builtin_amdgcn_wave_barrier();
            more = n == kWave;
            k += kWave;
        }
        if (lane == 0 && rec.w < a.y_cap) {
            a.y_idx[rec.w] = (int32_t)row;
            if (a.y_val) a.y_val[rec.w] = acc;
        }
    }
}

}  // namespace

hipError_t launch_det_gather(const DetArgs& a, uint2* list, int grid, hipStream_t s) {
    const size_t lds = ((size_t(1) << a.chunk_log2) + 2) * sizeof(int32_t);
    hipLaunchKernelGGL(k_det_gather, dim3(grid), dim3(kGatherBlock), lds, s, a, list);
    return hipGetLastError();
}

hipError_t launch_det_pass(const DetArgs& a, const uint2* in, uint2* out, int shift, int digit_bits,
                           int32_t* partials, hipStream_t s) {
    if (digit_bits < 1 || digit_bits > kDetMaxDigitBits) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_det_hist, dim3(a.nblk), dim3(kDetBlock), 0, s, a, in, shift, digit_bits);
    hipError_t e = launch_exclusive_scan_i32(a.counts, (int64_t(1) << digit_bits) * a.nblk + 1, partials, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_det_scatter, dim3(a.nblk), dim3(kDetBlock), 0, s, a, in, out, shift, digit_bits);
    return hipGetLastError();
}

hipError_t launch_det_fold(const DetArgs& a, const uint2* list, int32_t* partials, hipStream_t s) {
    hipLaunchKernelGGL(k_det_heads, dim3(a.nblk), dim3(kDetBlock), 0, s, a, list);
    hipError_t e = launch_exclusive_scan_i32(a.counts, int64_t(a.nblk) + 1, partials, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_det_fold, dim3(a.nblk), dim3(kDetBlock), 0, s, a, list);
    hipLaunchKernelGGL(k_det_fold_long, dim3(2048), dim3(kDetBlock), 0, s, a, list);
    return hipGetLastError();
}

}  // namespace spv
