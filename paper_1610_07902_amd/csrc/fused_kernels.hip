// One-launch SpMSpV-bucket: the scan (Algorithm 2's work estimate), the
// bucketing (Algorithm 1 step 1) and the merge with its compaction
// (Algorithm 1 steps 2-3) of one y <- A x in a single cooperative launch of
// one 1024-thread workgroup per compute unit.
//
// A multiply with about a million products spends most of its time in
// fixed costs when it runs as three kernels: on gfx950 each kernel boundary
// costs a few microseconds, and the bucketing's slot reservations (one
// returning atomic per chunk and bucket on a few hundred counters) serialise
// at the counters.  Here the phases are separated by exchanges among the
// resident workgroups instead, no atomic update of shared memory is on the
// hot path, and workgroup 0 coordinates every exchange so that no word is
// polled by more than one workgroup (hundreds of workgroups polling the
// same few cache lines made each exchange cost several microseconds):
//
//   (a) workgroup g owns x positions [g F, (g+1) F) (F = ceil(f / G)): it
//       gathers their column ranges, compacts the non-empty columns into its
//       own list (first entry, local exclusive product offset, x value), its
//       local offsets at 64 evenly spaced list positions, and then publishes
//       its product and column counts under this call's tag (the call
//       counter, so nothing is ever cleared).
//   (X1) workgroup 0 gathers the counts, publishes the prefix of products
//       over sources (W, and where each source's products sit among all W)
//       and one record per chunk: W and the chunk's first and last source.
//   (b) the products are split into equal chunks, one per workgroup (more
//       when W exceeds G chunks of kFChunk products).  A chunk reads the
//       prefix of its sources and the two boundary sources' samples (one
//       round trip) and then just the list entries covering it (one round
//       trip), gathers its row ids and values, applies Mult, counting-sorts
//       them by bucket in LDS and writes the sorted run at its own position
//       (chunk k at k * chunk) plus the run's per-bucket offsets: no slot
//       reservations.
//   (X2) every workgroup reports its runs complete; workgroup 0 releases
//       every workgroup once all have.
//   (c, d) workgroup b merges bucket b (and b + G, ...): it reads bucket b's
//       offset pair from every chunk's row, fetches the entries of every
//       run, accumulates them in the LDS tile (as the bucketing path's
//       merge) and publishes its unique count; workgroup 0 turns each
//       round's counts into offsets in y, and each bucket writes its rows in
//       ascending order.
//
// Every word that crosses workgroups is written and read with relaxed
// agent-scope atomics (coherent across the dies without cache maintenance);
// each wave waits for its own vector memory operations before its
// workgroup publishes a tag.  Every wait is bounded (ERR_SPIN), and a
// workgroup that gives up returns before writing anything further.

#include <hip/hip_ext.h>

#include "device_ops.h"

namespace spv {

namespace {

constexpr int B = kFBlock;
constexpr int kWaves = B / kWave;
constexpr int kFSpin = 1 << 21;
// Tags take 20 bits.  Exchange words: tag in bits 63:44; the products word
// of (X1) holds the column count in 43:31 and the product count in 30:0.
constexpr int kTagShift = 44;
constexpr uint64_t kVal31 = (uint64_t(1) << 31) - 1;
constexpr uint32_t kTagMod = (1u << 20) - 1;
static_assert(kFMaxF < (1 << 13), "column counts take 13 bits of the exchange word");
// Column-list entries one chunk may load: its products' columns plus at
// most one sample stride of columns before and after them.
constexpr int kSampleStrideMax = (kFMaxF + kFSamples - 1) / kFSamples;
constexpr int kListCap = kFChunk + 2 * kSampleStrideMax + 8;

__device__ __forceinline__ uint64_t ldw(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stw(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ldi(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void sti(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ldu(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stu(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last index i in [0, n) with a[i] <= v (a ascending, a[0] <= v).
template <typename T, typename V>
__device__ __forceinline__ int last_le(const T* a, int n, V v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// One wave polls words [0, G) until each carries `tag`; lane l keeps the
// words of sources l, l + 64, ... (at most kFMaxGrid / 64) in `got`.
// Returns false after the bound.
__device__ bool poll_tags(const uint64_t* w, int G, uint64_t tag, uint64_t (&got)[kFMaxGrid / kWave]) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int spins = 0;;) {
        bool ok = true;
#pragma unroll
        for (int k = 0; k < kFMaxGrid / kWave; ++k) {
            const int s = lane + k * kWave;
            if (s < G) {
                got[k] = ldw(&w[s]);
                ok &= (got[k] >> kTagShift) == tag;
            }
        }
        if (__all(ok)) return true;
        if (++spins > kFSpin) return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

// LDS layout (byte offsets from the dynamic base), one region reused by the
// phases: the scatter's source prefix, histograms, column table, column map
// and sort buffer, then the merge's tile, bitmap, list and run index.
struct Lay {
    size_t poff, cnt, slc, hist, hoff, tstart, toff, txv, colof, stage, scatter_end;
    size_t spa, bm, list, rbase, rpre, runmap, merge_end;
};
__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~size_t(15); }
__host__ __device__ inline Lay fused_layout(int G, int tl, bool wide, int nb) {
    Lay L{};
    size_t o = 0;
    L.poff = o; o = al16(o + size_t(G + 1) * 8);
    L.cnt = o; o = al16(o + size_t(G > 2 * kFSamples ? G : 2 * kFSamples) * 4);   // also the two sources' samples
    L.slc = o; o = al16(o + size_t(G + 1) * 4);
    L.hist = o; o = al16(o + size_t(nb + 1) * 4);
    L.hoff = o; o = al16(o + size_t(nb + 1) * 4);
    L.tstart = o; o = al16(o + size_t(kListCap) * 4);
    L.stage = L.tstart;   // the sort buffer replaces the column table once the gathers are done
    L.toff = o; o = al16(o + size_t(kListCap + 1) * 4);
    L.txv = o; o = al16(o + size_t(kListCap) * 4);
    if (o < L.stage + size_t(kFChunk) * 8) o = al16(L.stage + size_t(kFChunk) * 8);
    L.colof = o; o = al16(o + size_t(kFChunk) * 2);
    L.scatter_end = o;
    const size_t T = size_t(1) << tl;
    o = 0;
    L.spa = o; o = al16(o + T * (wide ? 8 : 4));
    L.bm = o; o = al16(o + (T / 32) * 4);
    L.list = o; o = al16(o + size_t(merge_list_cap(tl, wide)) * 2);
    L.rbase = o; o = al16(o + size_t(kFRunGroup) * 4);
    L.rpre = o; o = al16(o + size_t(kFRunGroup + 1) * 4);
    // run of each entry of a batch: in the walk's list when that holds a
    // batch (the two are never used at once), else a region of its own
    if (merge_list_cap(tl, wide) >= kFChunk) {
        L.runmap = L.list;
    } else {
        L.runmap = o;
        o = al16(o + size_t(kFChunk) * 2);
    }
    L.merge_end = o;
    return L;
}

template <int SR, int XMODE>
__global__ __launch_bounds__(B) void k_fused(FusedArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int64_t s_w64[kWaves + 1];
    __shared__ int s_w32[kWaves + 1];
    __shared__ uint32_t s_epoch;
    __shared__ int s_stop;
    __shared__ int s_max;
    __shared__ int s_src[2];        // first and last source of the chunk
    __shared__ int s_k[2];          // first list index in the first source, end index in the last
    __shared__ int64_t s_W;
    __shared__ int64_t s_excl;
    constexpr bool kWide = SR == SR_PLUS_TIMES;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int G = gridDim.x, g = blockIdx.x;
    Ctrl* const ctrl = a.ctrl;
    uint32_t* const err = &ctrl->err;
    uint64_t* const xw = a.xw;
    const int tl = a.tile_log2, nb = a.nb;
    const Lay L = fused_layout(G, tl, kWide, nb);

    if (tid == 0) {
        s_epoch = ldu(&ctrl->fused_epoch);
        s_stop = 0;
        s_max = 0;
    }
    __syncthreads();
    const uint64_t tag = (s_epoch % kTagMod) + 1u;   // 1 .. 2^20 - 1, never the zero of fresh memory
    const uint64_t hi = tag << kTagShift;
    // Thread 0 waits for word w to carry this call's tag; false after the bound.
    auto wait_word = [&](const uint64_t* w, uint64_t& got) -> bool {
        for (int spins = 0;;) {
            got = ldw(w);
            if ((got >> kTagShift) == tag) return true;
            if (++spins > kFSpin) return false;
            __builtin_amdgcn_s_sleep(1);
        }
    };

    // ---------------------------------------------------------------- (a)
    const int f = a.f;
    const int F = (f + G - 1) / G;
    const int64_t p0 = (int64_t)g * F;
    int32_t b0[4], ln[4];
    uint32_t xv[4];
    {
        int32_t jj[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = tid * 4 + i;
            jj[i] = (k < F && p0 + k < f) ? a.x_idx[p0 + k] : -1;
        }
        int32_t c1[4];
        bool bad = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool inr = jj[i] >= 0 && jj[i] < a.n;
            const int32_t jc = inr ? jj[i] : 0;
            b0[i] = a.colptr[jc];
            c1[i] = a.colptr[jc + 1];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = tid * 4 + i;
            const bool valid = k < F && p0 + k < f;
            const bool inr = jj[i] >= 0 && jj[i] < a.n;
            bad |= valid && !inr;
            ln[i] = (valid && inr) ? c1[i] - b0[i] : 0;
            xv[i] = valid ? x_value<XMODE>(a.x_val, (int)(p0 + k), jj[i]) : 0u;
        }
        if (bad) atomicOr(err, ERR_X_RANGE);
    }
    int64_t lsum = 0;
    int lcnt = 0, lmax = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        lsum += ln[i];
        lcnt += ln[i] > 0 ? 1 : 0;
        lmax = max(lmax, ln[i]);
    }
    uint64_t Pg_u;
    int Cg;
    const uint64_t eo = block_exclusive_u64<B>((uint64_t)lsum, reinterpret_cast<uint64_t*>(s_w64), Pg_u);
    const int ec = block_exclusive_i32<B>(lcnt, s_w32, Cg);
    {
        const int stride = Cg > 0 ? (Cg + kFSamples - 1) / kFSamples : 1;
        int c = ec;
        uint64_t o = eo;
        const int64_t base = (int64_t)g * F;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (ln[i] > 0) {
                sti(&a.lstart[base + c], b0[i]);
                sti(&a.loff[base + c], (int32_t)o);
                stu(&a.lxv[base + c], xv[i]);
                if (c % stride == 0) sti(&a.samples[g * kFSamples + c / stride], (int32_t)o);
                o += (uint64_t)ln[i];
                ++c;
            }
        }
    }
    atomicMax(&s_max, lmax);
    wait_vmem();   // the lists are complete before the counts are published
    __syncthreads();
    if (tid == 0) {
        // counts saturate at 2^31 - 1, which only inputs with more products
        // than stored entries reach
        stw(&xw[kXM + g], hi | (uint64_t)s_max);
        stw(&xw[kXA + g], hi | ((uint64_t)Cg << 31) | (Pg_u < kVal31 ? Pg_u : kVal31));
    }

    // ---------------------------------------------------------------- (X1)
    // Workgroup 0 gathers every source's counts, publishes the prefix (with
    // each source's column count) and one record per chunk (W and the
    // chunk's first and last source); every workgroup then waits only for
    // its own record.
    int64_t* const s_poff = reinterpret_cast<int64_t*>(lds + L.poff);
    int* const s_cnt = reinterpret_cast<int*>(lds + L.cnt);
    if (g == 0) {
        if (wid == 0) {
            uint64_t got[kFMaxGrid / kWave];
            if (!poll_tags(xw + kXA, G, tag, got)) {
                if (lane == 0) {
                    atomicOr(err, ERR_SPIN);
                    s_stop = 1;
                }
            } else {
#pragma unroll
                for (int k = 0; k < kFMaxGrid / kWave; ++k) {
                    const int s2 = lane + k * kWave;
                    if (s2 < G) {
                        s_poff[s2] = (int64_t)(got[k] & kVal31);
                        s_cnt[s2] = (int)((got[k] >> 31) & 0x1fffu);
                    }
                }
            }
        }
        __syncthreads();
        if (s_stop) return;
        const uint64_t P = tid < G ? (uint64_t)s_poff[tid] : 0u;
        const int cs = tid < G ? s_cnt[tid] : 0;
        uint64_t Wu;
        int fnz;
        const uint64_t pex = block_exclusive_u64<B>(P, reinterpret_cast<uint64_t*>(s_w64), Wu);
        (void)block_exclusive_i32<B>(cs, s_w32, fnz);
        if (tid < G) s_poff[tid] = (int64_t)pex;
        if (tid == 0) s_poff[G] = (int64_t)Wu;
        __syncthreads();
        const int64_t W = (int64_t)Wu;
        for (int s2 = tid; s2 <= G; s2 += B)
            __hip_atomic_store(&a.gpoff[s2], s_poff[s2] | ((int64_t)(s2 < G ? s_cnt[s2] : 0) << 48),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (tid == 0) {
            // Every workgroup has read this call's tag (it published under
            // it): advance the counter for the next call; this call's sizes.
            stu(&ctrl->fused_epoch, s_epoch + 1u);
            const int32_t Wc = W > INT32_MAX ? INT32_MAX : (int32_t)W;
            sti(&ctrl->W, Wc);
            sti(&ctrl->fnz, fnz);
            sti(&ctrl->W_last, Wc);
            sti(&ctrl->fnz_last, fnz);
            sti(&ctrl->f, f);
            if (W > a.nnz) atomicOr(err, ERR_BUCKET_OVERFLOW);   // more products than stored entries: duplicate x
            if (W == 0 || W > a.nnz) {
                sti(&ctrl->maxlen_last, 0);
                __hip_atomic_store(&ctrl->nnz_y, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (a.d_nnz_y) *a.d_nnz_y = 0;
            }
        }
        const bool work = W > 0 && W <= a.nnz;
        const int64_t Cw = !work ? 1 : (W <= (int64_t)G * kFChunk ? (W + G - 1) / G : (int64_t)kFChunk);
        const int64_t nchunks = !work ? 0 : (W + Cw - 1) / Cw;
        wait_vmem();   // the prefix is complete before any record names it
        __syncthreads();
        const int64_t nrec = nchunks > G ? nchunks : G;
        for (int64_t k = tid; k < nrec && k < a.rows_cap; k += B) {
            uint64_t w1 = hi;
            if (k < nchunks) {
                const int64_t q0 = k * Cw;
                const int64_t q1 = q0 + Cw < W ? q0 + Cw : W;
                w1 |= (uint64_t)last_le(s_poff, G + 1, q0) | ((uint64_t)last_le(s_poff, G + 1, q1 - 1) << 16);
            }
            stw(&a.xrec[2 * k + 1], w1);
            stw(&a.xrec[2 * k], hi | (uint64_t)W);
        }
    }

    // ---------------------------------------------------------------- (b)
    if (tid == 0) {
        uint64_t w0 = 0, w1 = 0;
        if (!wait_word(&a.xrec[2 * g], w0) || !wait_word(&a.xrec[2 * g + 1], w1)) {
            atomicOr(err, ERR_SPIN);
            s_stop = 1;
        }
        s_W = (int64_t)(w0 & ((uint64_t(1) << kTagShift) - 1));
        s_src[0] = (int)(w1 & 0xffffu);
        s_src[1] = (int)((w1 >> 16) & 0xffffu);
    }
    __syncthreads();
    if (s_stop) return;
    const int64_t W = s_W;
    if (W == 0 || W > a.nnz) return;
    const int64_t Cw = W <= (int64_t)G * kFChunk ? (W + G - 1) / G : (int64_t)kFChunk;
    const int64_t nchunks = (W + Cw - 1) / Cw;
    if (nchunks > a.rows_cap) {   // the run offsets cannot hold this call (not reached: rows_cap covers W <= nnz)
        if (tid == 0) atomicOr(err, ERR_BUCKET_OVERFLOW);
        return;
    }
    int64_t* const s_pl = s_poff;   // prefix (and column counts) of the chunk's sources
    int* const s_slc = reinterpret_cast<int*>(lds + L.slc);
    int* const s_smp = s_cnt;       // the two boundary sources' samples
    int* const hist = reinterpret_cast<int*>(lds + L.hist);
    int* const hoff = reinterpret_cast<int*>(lds + L.hoff);
    int32_t* const t_start = reinterpret_cast<int32_t*>(lds + L.tstart);
    int32_t* const t_off = reinterpret_cast<int32_t*>(lds + L.toff);
    uint32_t* const t_xv = reinterpret_cast<uint32_t*>(lds + L.txv);
    uint16_t* const col_of = reinterpret_cast<uint16_t*>(lds + L.colof);
    uint2* const stage = reinterpret_cast<uint2*>(lds + L.stage);
    for (int b = tid; b <= nb; b += B) hist[b] = 0;
    for (int64_t k = g; k < nchunks; k += G) {
        const int64_t q0 = k * Cw;
        const int cnt = (int)min(Cw, W - q0);
        if (k != g && tid == 0) {
            uint64_t w1 = 0;
            if (!wait_word(&a.xrec[2 * k + 1], w1)) {
                atomicOr(err, ERR_SPIN);
                s_stop = 1;
            }
            s_src[0] = (int)(w1 & 0xffffu);
            s_src[1] = (int)((w1 >> 16) & 0xffffu);
        }
        __syncthreads();
        if (s_stop) return;
        const int slo = s_src[0], shi = s_src[1];
        const int nsrc = shi - slo + 1;
        // one round trip: the sources' prefix and column counts, and the
        // samples of the first and last source
        for (int t = tid; t <= nsrc; t += B)
            s_pl[t] = __hip_atomic_load(&a.gpoff[slo + t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (tid < 2 * kWave) s_smp[tid] = ldi(&a.samples[(tid < kWave ? slo : shi) * kFSamples + lane]);
        __syncthreads();
        constexpr int64_t kPre = (int64_t(1) << 48) - 1;
        if (tid < 2 * kWave) {
            const int si = tid < kWave ? 0 : nsrc - 1;
            const int c = (int)(s_pl[si] >> 48);
            const int stride = c > 0 ? (c + kFSamples - 1) / kFSamples : 1;
            const int j = lane;
            const int v = j * stride < c ? s_smp[tid] : INT32_MAX;
            const int64_t t = tid < kWave ? q0 - (s_pl[0] & kPre) : q0 + cnt - 1 - (s_pl[nsrc - 1] & kPre);
            if (tid < kWave) {
                // first list index: the last sample at or below the chunk's first product
                const uint64_t le = __ballot(j * stride < c && (int64_t)v <= t);
                if (lane == 0) s_k[0] = le ? (63 - __clzll((long long)le)) * stride : 0;
            } else {
                // end index: the first sample above the chunk's last product
                const uint64_t gt = __ballot((int64_t)v > t);
                if (lane == 0) s_k[1] = gt ? min(c, (__ffsll((unsigned long long)gt) - 1) * stride) : c;
            }
        }
        __syncthreads();
        const int ka = s_k[0], kb = s_k[1];
        // list entries to load, source by source
        int total_e;
        {
            int len = 0;
            if (tid < nsrc) {
                const int beg = tid == 0 ? ka : 0;
                const int end = tid == nsrc - 1 ? kb : (int)(s_pl[tid] >> 48);
                len = end > beg ? end - beg : 0;
            }
            const int e = block_exclusive_i32<B>(len, s_w32, total_e);
            if (tid < nsrc) s_slc[tid] = e;
            if (tid == 0) s_slc[nsrc] = total_e;
        }
        if (total_e > kListCap || total_e < 1) {   // inconsistent lists; never reached with consistent input
            if (tid == 0) atomicOr(err, ERR_SPIN);
            return;
        }
        __syncthreads();
        for (int e = tid; e < total_e; e += B) {
            const int si = last_le(s_slc, nsrc, e);
            const int64_t pos = (int64_t)(slo + si) * F + (si == 0 ? ka : 0) + (e - s_slc[si]);
            t_start[e] = ldi(&a.lstart[pos]);
            t_off[e] = (int32_t)((s_pl[si] & kPre) + ldi(&a.loff[pos]) - q0);
            t_xv[e] = ldu(&a.lxv[pos]);
        }
        if (tid == 0) t_off[total_e] = INT32_MAX;
        __syncthreads();
        // column of each product: one search per thread, then a forward walk
        {
            const int r0 = tid * kFItems;
            if (r0 < cnt) {
                int e = last_le(t_off, total_e, r0);
#pragma unroll
                for (int i = 0; i < kFItems; ++i) {
                    const int r = r0 + i;
                    while (e + 1 < total_e && r >= t_off[e + 1]) ++e;
                    if (r < cnt) col_of[r] = (uint16_t)e;
                }
            }
        }
        __syncthreads();
        // gathers: item i of thread t is product i * B + t (lanes read consecutive entries)
        int32_t row[kFItems], bk[kFItems], rank[kFItems];
        uint32_t val[kFItems];
        {
            int32_t qq[kFItems];
            uint32_t xc[kFItems];
#pragma unroll
            for (int i = 0; i < kFItems; ++i) {
                const int r = i * B + tid;
                const int e = r < cnt ? col_of[r] : 0;
                qq[i] = r < cnt ? t_start[e] + (r - t_off[e]) : -1;
                xc[i] = t_xv[e];
            }
#pragma unroll
            for (int i = 0; i < kFItems; ++i) row[i] = a.rowids[qq[i] >= 0 ? qq[i] : 0];
#pragma unroll
            for (int i = 0; i < kFItems; ++i) val[i] = mult<SR>(a.values, qq[i] >= 0 ? qq[i] : 0, xc[i]);
            uint32_t mw[kFItems];
#pragma unroll
            for (int i = 0; i < kFItems; ++i) mw[i] = a.mask ? a.mask[(uint32_t)row[i] >> 5] : 0u;
#pragma unroll
            for (int i = 0; i < kFItems; ++i) {
                bk[i] = -1;
                rank[i] = 0;
                if (qq[i] >= 0 && ((mw[i] >> (row[i] & 31)) & 1u) == 0u) {
                    bk[i] = row[i] >> tl;
                    rank[i] = atomicAdd(&hist[bk[i]], 1);
                }
            }
        }
        __syncthreads();
        // chunk-local bucket offsets: the run's row of offsets
        int kept = 0;
        int32_t* const orow = a.roff + k * (nb + 1);
        for (int b0i = 0; b0i < nb; b0i += B) {
            const int b = b0i + tid;
            const int n = b < nb ? hist[b] : 0;
            if (b < nb) hist[b] = 0;
            int tot;
            const int e = block_exclusive_i32<B>(n, s_w32, tot);
            if (b < nb) {
                hoff[b] = kept + e;
                sti(&orow[b], kept + e);
            }
            kept += tot;
        }
        if (tid == 0) sti(&orow[nb], kept);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kFItems; ++i)
            if (bk[i] >= 0) stage[hoff[bk[i]] + rank[i]] = make_uint2((uint32_t)row[i], val[i]);
        __syncthreads();
        uint64_t* const out = reinterpret_cast<uint64_t*>(a.buckets + q0);
        for (int t = tid; t < kept; t += B) {
            const uint2 e = stage[t];
            stw(&out[t], (uint64_t)e.x | ((uint64_t)e.y << 32));
        }
        __syncthreads();
    }

    // ---------------------------------------------------------------- (X2)
    wait_vmem();   // this workgroup's runs are complete
    __syncthreads();
    if (tid == 0) stw(&xw[kXD + g], hi);
    if (g == 0) {
        // every run complete: release every workgroup
        if (wid == 0) {
            uint64_t got[kFMaxGrid / kWave];
            if (!poll_tags(xw + kXD, G, tag, got) && lane == 0) {
                atomicOr(err, ERR_SPIN);
                s_stop = 1;
            }
        }
        __syncthreads();
        if (s_stop) return;
        for (int s2 = tid; s2 < G; s2 += B) stw(&xw[kXG + s2], hi);
    }
    const int T = 1 << tl;
    uint32_t* const spa = reinterpret_cast<uint32_t*>(lds + L.spa);
    uint32_t* const bm = reinterpret_cast<uint32_t*>(lds + L.bm);
    uint16_t* const list = reinterpret_cast<uint16_t*>(lds + L.list);
    int32_t* const s_rbase = reinterpret_cast<int32_t*>(lds + L.rbase);
    int32_t* const s_rpre = reinterpret_cast<int32_t*>(lds + L.rpre);
    uint16_t* const runmap = reinterpret_cast<uint16_t*>(lds + L.runmap);
    auto init_tile = [&](int rows) {
        const int nw = (rows + 31) >> 5;
        for (int w = tid; w < nw; w += B) bm[w] = 0u;
        uint4* spa4 = reinterpret_cast<uint4*>(spa);
        if constexpr (kWide) {
            const uint4 z = make_uint4(0u, 0x80000000u, 0u, 0x80000000u);   // two -0.0 doubles
            for (int q = tid; q < nw * 16; q += B) spa4[q] = z;
        } else {
            const uint32_t id = identity<SR>();
            for (int q = tid; q < nw * 8; q += B) spa4[q] = make_uint4(id, id, id, id);
        }
    };
    if (g < nb) init_tile(min(T, a.m - (g << tl)));   // while the last runs are written
    if (tid == 0) {
        uint64_t w;
        if (!wait_word(&xw[kXG + g], w)) {
            atomicOr(err, ERR_SPIN);
            s_stop = 1;
        }
    }
    __syncthreads();
    if (s_stop) return;

    // ------------------------------------------------------------- (c, d)
    // Buckets in rounds of G (workgroup g merges g, g + G, ...); after each
    // round workgroup 0 turns the round's unique counts into y offsets.
    int64_t ycarry = 0;   // workgroup 0: unique rows of the finished rounds
    const int rounds = (nb + G - 1) / G;
    for (int rd = 0; rd < rounds; ++rd) {
        const int b = g + rd * G;
        if (b >= nb) break;   // only workgroups past the last bucket stop early; workgroup 0 never does
        const int row0 = b << tl;
        const int rows = min(T, a.m - row0);
        const int nw = (rows + 31) >> 5;
        if (rd > 0) {
            init_tile(rows);
            __syncthreads();
        }
        bool bad = false, sparse = false;
        for (int64_t k0 = 0; k0 < nchunks; k0 += kFRunGroup) {
            const int nr = (int)min((int64_t)kFRunGroup, nchunks - k0);
            int len = 0;
            if (tid < nr) {
                const int32_t* orow = a.roff + (k0 + tid) * (nb + 1);
                const int32_t o0 = ldi(&orow[b]), o1 = ldi(&orow[b + 1]);
                len = o1 - o0;
                s_rbase[tid] = (int32_t)((k0 + tid) * Cw + o0);
            }
            int rcnt;
            const int e = block_exclusive_i32<B>(len, s_w32, rcnt);
            if (tid < nr) s_rpre[tid] = e;
            if (tid == 0) s_rpre[nr] = rcnt;
            if (k0 == 0) sparse = nchunks <= kFRunGroup && rcnt < rows / 8;
            __syncthreads();
            for (int e0 = 0; e0 < rcnt; e0 += kFChunk) {
                // run of every entry of this batch: one search per thread for
                // its first of kFItems consecutive entries, then a forward
                // step or, past empty runs, another search
                const int nE = min(kFChunk, rcnt - e0);
                {
                    const int r0 = tid * kFItems;
                    if (r0 < nE) {
                        int ri = last_le(s_rpre, nr, e0 + r0);
#pragma unroll
                        for (int i = 0; i < kFItems; ++i) {
                            const int ei = e0 + r0 + i;
                            if (ri + 1 < nr && s_rpre[ri + 1] <= ei)
                                ri = (ri + 2 < nr && s_rpre[ri + 2] <= ei)
                                         ? ri + 2 + last_le(s_rpre + ri + 2, nr - ri - 2, ei)
                                         : ri + 1;
                            if (r0 + i < nE) runmap[r0 + i] = (uint16_t)ri;
                        }
                    }
                }
                __syncthreads();
                uint64_t ent[kFItems];
#pragma unroll
                for (int u = 0; u < kFItems; ++u) {
                    const int kk = u * B + tid;
                    ent[u] = 0xffffffffull;
                    if (kk < nE) {
                        const int ri = runmap[kk];
                        ent[u] = ldw(reinterpret_cast<const uint64_t*>(a.buckets) + s_rbase[ri] + (e0 + kk - s_rpre[ri]));
                    }
                }
                uint32_t r[kFItems], v[kFItems];
                bool ok[kFItems];
#pragma unroll
                for (int u = 0; u < kFItems; ++u) {
                    r[u] = (uint32_t)ent[u] - (uint32_t)row0;
                    v[u] = (uint32_t)(ent[u] >> 32);
                    ok[u] = u * B + tid < nE;
                    if (ok[u] && r[u] >= (uint32_t)rows) {
                        ok[u] = false;
                        bad = true;
                    }
                }
                add_rows<SR, kFItems>(r, v, ok, spa, bm, sparse);
                __syncthreads();   // the run map is rebuilt for the next batch
            }
        }
        if (bad) atomicOr(err, ERR_BUCKET_OVERFLOW);
        if (kWide && !sparse) {
            touched_bits64<B>(spa, bm, rows);
            __syncthreads();
        }
        int pc = 0;
        for (int w = tid; w < nw; w += B) pc += __popc(bm[w]);
        int ucnt;
        (void)block_exclusive_i32<B>(pc, s_w32, ucnt);
        if (tid == 0) stw(&xw[kXU + b], hi | (uint64_t)ucnt);
        if (g == 0) {
            // this round's buckets: unique counts -> offsets in y
            const int rb0 = rd * G, rn = min(G, nb - rb0);
            if (wid == 0) {
                uint64_t got[kFMaxGrid / kWave];
                if (!poll_tags(xw + kXU + rb0, rn, tag, got)) {
                    if (lane == 0) {
                        atomicOr(err, ERR_SPIN);
                        s_stop = 1;
                    }
                } else {
                    // prefix over the round's buckets, lane by lane and k by k
                    int64_t carry = ycarry;
#pragma unroll
                    for (int k = 0; k < kFMaxGrid / kWave; ++k) {
                        const int bi = lane + k * kWave;
                        int64_t u = bi < rn ? (int64_t)(got[k] & ((uint64_t(1) << kTagShift) - 1)) : 0;
                        int64_t x = u;
#pragma unroll
                        for (int d = 1; d < kWave; d <<= 1) {
                            const int64_t y = __shfl_up(x, d, kWave);
                            if (lane >= d) x += y;
                        }
                        if (bi < rn) stw(&xw[kXY + rb0 + bi], hi | (uint64_t)(carry + x - u));
                        carry += __shfl(x, kWave - 1, kWave);
                    }
                    ycarry = carry;   // the same in every lane
                    if (lane == 0 && rd == rounds - 1) {
                        __hip_atomic_store(&ctrl->nnz_y, carry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (a.d_nnz_y) *a.d_nnz_y = carry;
                    }
                }
            }
            __syncthreads();
            if (s_stop) return;
        }
        if (tid == 0) {
            uint64_t w;
            if (!wait_word(&xw[kXY + b], w)) {
                atomicOr(err, ERR_SPIN);
                s_stop = 1;
            }
            s_excl = (int64_t)(w & ((uint64_t(1) << kTagShift) - 1));
        }
        __syncthreads();
        if (s_stop) return;
        const int64_t excl = s_excl;
        // in-order walk of the bitmap; rows staged through the LDS list for coalesced writes
        const int round_words = min(B, merge_list_cap(tl, kWide) >> 5);
        int64_t carry = 0;
        for (int w0 = 0; w0 < nw; w0 += round_words) {
            const int w = w0 + tid;
            const bool mine = tid < round_words && w < nw;
            const uint32_t bits = mine ? bm[w] : 0u;
            int tot;
            const int pos = block_exclusive_i32<B>(__popc(bits), s_w32, tot);
            uint32_t rest = bits;
            int kk = 0;
            while (rest) {
                const int bitpos = __ffs(rest) - 1;
                rest &= rest - 1u;
                list[pos + kk] = (uint16_t)((w << 5) + bitpos);
                ++kk;
            }
            __syncthreads();
            for (int t = tid; t < tot; t += B) {
                const int rr = list[t];
                const int64_t o = excl + carry + t;
                uint32_t v;
                if constexpr (kWide) v = __float_as_uint((float)reinterpret_cast<const double*>(spa)[rr]);
                else v = spa[rr];
                if (o < a.y_cap) {
                    a.y_idx[o] = row0 + rr;
                    if (a.y_val) store_value<SR>(a.y_val, o, v);
                }
            }
            carry += tot;
            __syncthreads();
        }
    }
    if (g == 0 && wid == 0) {
        // longest selected column of the call, for the call's statistics
        int lm = 0;
        for (int s2 = lane; s2 < G; s2 += kWave) lm = max(lm, (int)(ldw(&xw[kXM + s2]) & kVal31));
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) lm = max(lm, __shfl_xor(lm, d, kWave));
        if (lane == 0) sti(&ctrl->maxlen_last, lm);
    }
}

template <int SR>
const void* fused_fn(int xmode) {
    switch (xmode) {
        case XV_BITS32: return reinterpret_cast<const void*>(k_fused<SR, XV_BITS32>);
        case XV_INDEX: return reinterpret_cast<const void*>(k_fused<SR, XV_INDEX>);
        case XV_U8: return reinterpret_cast<const void*>(k_fused<SR, XV_U8>);
        default: return reinterpret_cast<const void*>(k_fused<SR, XV_TRUE>);
    }
}

const void* fused_kernel(int semiring, int xmode) {
    switch (semiring) {
        case SR_PLUS_TIMES: return fused_fn<SR_PLUS_TIMES>(xmode);
        case SR_MIN_SELECT2ND: return fused_fn<SR_MIN_SELECT2ND>(xmode);
        default: return fused_fn<SR_OR_AND>(xmode);
    }
}

}  // namespace

size_t fused_lds_bytes(int tile_log2, int semiring, int nb) {
    // sized for the largest grid the launcher uses (one workgroup per CU, at most kFMaxGrid)
    const Lay L = fused_layout(kFMaxGrid, tile_log2, semiring == SR_PLUS_TIMES, nb);
    return L.scatter_end > L.merge_end ? L.scatter_end : L.merge_end;
}

// Workgroups of the one-launch multiply that are resident together (one per
// compute unit), or 0 when the device cannot hold one workgroup per unit.
int fused_grid(int num_cu, size_t lds_bytes) {
    if (num_cu < 1 || num_cu > kFMaxGrid) return 0;
    int per_cu = 0;
    for (int sr = 0; sr < 3; ++sr) {
        const void* fn = fused_kernel(sr, XV_BITS32);
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) != hipSuccess)
            return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), B,
                                                          lds_bytes) != hipSuccess ||
            per_cu < 1)
            return 0;
    }
    return num_cu;
}

hipError_t launch_fused(const FusedArgs& a, int semiring, int grid, hipStream_t s, const LaunchEvents* ev) {
    if (grid < 1 || grid > kFMaxGrid || a.nb < 1 || a.nb > kFMaxNb || a.f < 0 ||
        (int64_t)a.f > (int64_t)grid * kFMaxF)
        return hipErrorInvalidValue;
    const void* fn = fused_kernel(semiring, a.xmode);
    const size_t lds = fused_lds_bytes(a.tile_log2, semiring, a.nb);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    void* args[] = {const_cast<FusedArgs*>(&a)};
    // A plain launch: the grid is one workgroup per compute unit and a
    // workgroup takes a whole unit (LDS), so on an otherwise idle device
    // every workgroup is resident at once (fused_grid checks that one fits
    // per unit).  A cooperative launch would guarantee it even beside other
    // streams' work, but costs about 17 us more per call on this device.
    // Should a workgroup not become resident, the others' bounded waits end
    // the call with ERR_SPIN instead of hanging.
    if (ev) return hipExtLaunchKernel(fn, dim3(grid), dim3(B), args, lds, s, ev->start, ev->stop, 0);
    return hipLaunchKernel(fn, dim3(grid), dim3(B), args, lds, s);
}

}  // namespace spv
