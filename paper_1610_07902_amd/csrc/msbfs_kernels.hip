// Multi-source BFS in the pull direction (bottom-up), bit-parallel over the
// sources.  The paper names switching SpMSpV-driven BFS to the matrix-driven
// direction as future work (Conclusions); with many sources one pull step
// serves all of them: source s owns bit s % 64 of word s / 64 of every
// vertex's frontier and seen masks (G = ceil(nsrc / 64) words per vertex,
// stored vertex-major: word g of vertex v at v * G + g).
//
// A vertex v not yet seen by some sources scans its row (the in-neighbours
// u, ascending) and takes, for every such source, the first u whose frontier
// mask has the source's bit: with ascending rows that is the smallest
// frontier in-neighbour, the parent the push direction's min-select2nd
// gives.  The scan stops once every unseen source is found.  Rows of up to
// kMsLong entries are scanned by one thread each, eight entries in flight
// (levels and parents then stored source by source for the wave's 64
// vertices); longer rows by one wave, 64 entries per step.
//
// Switching a search from push to pull converts its state once: the
// per-source visited bitmaps become the seen masks (transposed), the
// per-source frontier lists become frontier masks.

#include "device_ops.h"

namespace spv {

namespace {

constexpr int kMsBlock = 256;
constexpr int kMsUnroll = 8;

__device__ __forceinline__ uint64_t group_valid(int nsrc, int g) {
    const int k = nsrc - 64 * g;
    return k >= 64 ? ~0ull : ((1ull << k) - 1ull);
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v |= __shfl_xor(v, d);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d);
    return v;
}

// One wave covers 64 consecutive vertices.  A vertex's parent for each
// newly found source is kept in LDS (slot [source][lane] of its wave) while
// its row is scanned; afterwards the wave stores source by source, so each
// store instruction writes consecutive vertices of one source's level and
// parent rows instead of 64 scattered words.
constexpr int kMsShortBlock = 128;

template <bool PARENT>
__global__ __launch_bounds__(kMsShortBlock) void k_ms_pull_short(MsArgs a) {
    __shared__ uint32_t s_par[PARENT ? kMsShortBlock / kWave : 1][64][kWave];
    const int g = blockIdx.y;
    const uint64_t valid = group_valid(a.nsrc, g);
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = PARENT ? threadIdx.x / kWave : 0;
    uint32_t cnt = 0;
    for (int64_t base = (int64_t)blockIdx.x * kMsShortBlock; base < a.n;
         base += (int64_t)gridDim.x * kMsShortBlock) {
        const int64_t v = base + threadIdx.x;
        uint64_t found = 0ull;
        bool mine = false;   // this thread owns v's words in this kernel
        if (v < a.n) {
            const int32_t b = a.rowptr[v], e = a.rowptr[v + 1];
            mine = e - b <= kMsLong;   // longer rows are k_ms_pull_long's
            if (mine) {
                const int64_t at = v * a.G + g;
                const uint64_t seen = a.seen[at];
                const uint64_t unseen = valid & ~seen;
                if (unseen) {
                    for (int32_t k = b; k < e; k += kMsUnroll) {
                        uint32_t u[kMsUnroll];
                        uint64_t fu[kMsUnroll];
#pragma unroll
                        for (int q = 0; q < kMsUnroll; ++q) u[q] = k + q < e ? a.colids[k + q] : 0u;
#pragma unroll
                        for (int q = 0; q < kMsUnroll; ++q)
                            fu[q] = k + q < e ? a.fcur[(int64_t)u[q] * a.G + g] : 0ull;
#pragma unroll
                        for (int q = 0; q < kMsUnroll; ++q) {
                            uint64_t nf = fu[q] & unseen & ~found;
                            found |= nf;
                            if (PARENT) {
                                while (nf) {
                                    const int sb = __ffsll((unsigned long long)nf) - 1;
                                    nf &= nf - 1ull;
                                    s_par[wv][sb][lane] = u[q];
                                }
                            }
                        }
                        if (found == unseen) break;
                    }
                }
                a.fnext[at] = found;
                if (found) {
                    a.seen[at] = seen | found;
                    cnt += (uint32_t)__popcll(found);
                }
            }
        }
        // source-major stores of this wave's new levels and parents
        uint64_t any = wave_or64(found);   // uniform
        while (any) {
            const int sb = __ffsll((unsigned long long)any) - 1;
            any &= any - 1ull;
            if ((found >> sb) & 1ull) {
                const int64_t o = (int64_t)(64 * g + sb) * a.n + v;
                a.level[o] = a.lvl;
                if (PARENT) a.parent[o] = (int32_t)s_par[wv][sb][lane];
            }
        }
    }
    cnt = wave_sum_u32(cnt);
    if (lane == 0 && cnt) atomicAdd(a.found_total, (unsigned long long)cnt);
}

template <bool PARENT>
__global__ __launch_bounds__(kMsBlock) void k_ms_pull_long(MsArgs a) {
    const int g = blockIdx.y;
    const uint64_t valid = group_valid(a.nsrc, g);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = (int64_t)gridDim.x * (kMsBlock / kWave);
    const int32_t count = *a.long_count;
    uint32_t cnt = 0;
    for (int64_t r = (int64_t)blockIdx.x * (kMsBlock / kWave) + threadIdx.x / kWave; r < count; r += nwaves) {
        const int32_t v = a.long_rows[r];
        const int32_t b = a.rowptr[v], e = a.rowptr[v + 1];
        const int64_t at = (int64_t)v * a.G + g;
        const uint64_t seen = a.seen[at];
        const uint64_t unseen = valid & ~seen;
        uint64_t found = 0ull;
        if (unseen) {
            for (int32_t k = b; k < e; k += kWave) {
                const int32_t idx = k + lane;
                const uint32_t u = idx < e ? a.colids[idx] : 0u;
                const uint64_t f = idx < e ? (a.fcur[(int64_t)u * a.G + g] & unseen & ~found) : 0ull;
                const uint64_t nf = wave_or64(f);   // uniform
                if (nf) {
                    uint64_t rest = nf;
                    while (rest) {   // every new source: its first lane (smallest u of this step)
                        const int s = __ffsll((unsigned long long)rest) - 1;
                        rest &= rest - 1ull;
                        const uint64_t lanes = __ballot((f >> s) & 1ull);
                        const int first = __ffsll((unsigned long long)lanes) - 1;
                        const uint32_t pu = (uint32_t)__shfl((int)u, first);
                        if (lane == 0) {
                            const int64_t o = (int64_t)(64 * g + s) * a.n + v;
                            a.level[o] = a.lvl;
                            if (PARENT) a.parent[o] = (int32_t)pu;
                        }
                    }
                    found |= nf;
                    if (found == unseen) break;
                }
            }
        }
        if (lane == 0) {
            a.fnext[at] = found;
            if (found) {
                a.seen[at] = seen | found;
                cnt += (uint32_t)__popcll(found);
            }
        }
    }
    if (lane == 0 && cnt) atomicAdd(a.found_total, (unsigned long long)cnt);
}

// Rows longer than kMsLong entries, listed once per handle.
__global__ void k_ms_long_rows(const int32_t* rowptr, int32_t n, int32_t* rows, int32_t* count) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (rowptr[v + 1] - rowptr[v] > kMsLong) rows[atomicAdd(count, 1)] = (int32_t)v;
}

// Seen masks from the per-source visited bitmaps (source s's bitmap at
// visited + s * mask_words).  A vertex with an empty row can never be
// reached in the pull direction: it is marked seen by every source so no
// later step reads its row.
__global__ void k_ms_seen(MsArgs a, const uint32_t* visited, int32_t mask_words) {
    const int g = blockIdx.y;
    const uint64_t valid = group_valid(a.nsrc, g);
    const int ns = a.nsrc - 64 * g < 64 ? a.nsrc - 64 * g : 64;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += (int64_t)gridDim.x * blockDim.x) {
        uint64_t bits = 0ull;
        if (a.rowptr[v + 1] == a.rowptr[v]) {
            bits = valid;
        } else {
            const uint32_t* w = visited + (int64_t)(64 * g) * mask_words + (v >> 5);
            for (int s = 0; s < ns; ++s) bits |= (uint64_t)((w[(int64_t)s * mask_words] >> (v & 31)) & 1u) << s;
        }
        a.seen[v * a.G + g] = bits;
    }
}

// Frontier masks from the per-source frontier lists (source s's entries at
// [xoff[s], xoff[s+1]) of front) into fm, cleared before.
__global__ __launch_bounds__(kMsBlock) void k_ms_front(MsArgs a, const int32_t* front, const int64_t* xoff,
                                                       uint64_t* fm) {
    __shared__ int64_t s_off[kMaxBatch + 1];
    for (int i = threadIdx.x; i <= a.nsrc; i += kMsBlock) s_off[i] = xoff[i];
    __syncthreads();
    const int64_t total = s_off[a.nsrc];
    for (int64_t p = (int64_t)blockIdx.x * kMsBlock + threadIdx.x; p < total; p += (int64_t)gridDim.x * kMsBlock) {
        int lo = 0, hi = a.nsrc - 1;   // the source whose range holds p
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= p) lo = mid;
            else hi = mid - 1;
        }
        const int32_t v = front[p];
        if (v >= 0 && v < a.n)
            atomicOr(reinterpret_cast<unsigned long long*>(&fm[(int64_t)v * a.G + (lo >> 6)]), 1ull << (lo & 63));
    }
}

// Sum of the column lengths (out-degrees) of every entry of the frontier
// lists: the push direction's work for the next level.
__global__ __launch_bounds__(kMsBlock) void k_ms_degsum(const int32_t* front, const int64_t* xoff, int nsrc,
                                                        const int32_t* colptr, int32_t n, unsigned long long* out) {
    const int64_t total = xoff[nsrc];
    unsigned long long sum = 0;
    for (int64_t p = (int64_t)blockIdx.x * kMsBlock + threadIdx.x; p < total; p += (int64_t)gridDim.x * kMsBlock) {
        const int32_t v = front[p];
        if (v >= 0 && v < n) sum += (unsigned long long)(colptr[v + 1] - colptr[v]);
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) sum += __shfl_xor(sum, d);
    if ((threadIdx.x & (kWave - 1)) == 0 && sum) atomicAdd(out, sum);
}

inline unsigned grid_for_n(int64_t n, int cap) {
    int64_t g = (n + kMsBlock - 1) / kMsBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_ms_long_rows(const int32_t* rowptr, int32_t n, int32_t* rows, int32_t* count, hipStream_t s) {
    hipLaunchKernelGGL(k_ms_long_rows, dim3(grid_for_n(n, 4096)), dim3(kMsBlock), 0, s, rowptr, n, rows, count);
    return hipGetLastError();
}

hipError_t launch_ms_to_pull(const MsArgs& a, const uint32_t* visited, int32_t mask_words, const int32_t* front,
                             const int64_t* xoff, uint64_t* fm, hipStream_t s) {
    hipLaunchKernelGGL(k_ms_seen, dim3(grid_for_n(a.n, 8192), a.G), dim3(kMsBlock), 0, s, a, visited, mask_words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ms_front, dim3(4096), dim3(kMsBlock), 0, s, a, front, xoff, fm);
    return hipGetLastError();
}

hipError_t launch_ms_pull(const MsArgs& a, bool parent, int num_cu, hipStream_t s) {
    int64_t gshort = (a.n + kMsShortBlock - 1) / kMsShortBlock;
    if (gshort > 32768) gshort = 32768;
    if (gshort < 1) gshort = 1;
    const dim3 gs((unsigned)gshort, a.G), gl((unsigned)(8 * num_cu), a.G);
    if (parent) {
        hipLaunchKernelGGL(k_ms_pull_short<true>, gs, dim3(kMsShortBlock), 0, s, a);
        hipLaunchKernelGGL(k_ms_pull_long<true>, gl, dim3(kMsBlock), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_ms_pull_short<false>, gs, dim3(kMsShortBlock), 0, s, a);
        hipLaunchKernelGGL(k_ms_pull_long<false>, gl, dim3(kMsBlock), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_ms_degsum(const int32_t* front, const int64_t* xoff, int nsrc, const int32_t* colptr, int32_t n,
                            unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(k_ms_degsum, dim3(1024), dim3(kMsBlock), 0, s, front, xoff, nsrc, colptr, n, out);
    return hipGetLastError();
}

}  // namespace spv
