// Format variants of the SpMSpV operands (Background, "Sparse matrix and
// vector data structures"):
//   DCSC     only the non-empty columns are stored (ids jc, starts cp).  The
//            scan finds column j through a column index over jc: aux[c] is
//            the first stored column at or after c << shift, so j is searched
//            among jc[aux[j >> shift], aux[(j >> shift) + 1]) (the auxiliary
//            array the format description mentions for constant expected
//            lookup; with about nzc chunks each holds one stored column on
//            average).
//   bitvector  a sparse vector as a bitmap of its length plus its values in
//            ascending index order.  The multiply itself runs on index lists:
//            the input bitmap is expanded to its ascending index list (two
//            kernels: per-tile bit counts, then each tile emits at the sum of
//            the counts before it); the output bitmap is written by the merge
//            from its tiles' touched-row bitmaps.

#include "device_ops.h"

namespace spv {

namespace {

constexpr int kFmtBlock = 256;
constexpr int kWordsPerThread = 8;
constexpr int kTileWords = kFmtBlock * kWordsPerThread;   // 2048 words = 65536 bits per tile

__global__ void k_dcsc_aux(const int32_t* jc, int32_t nzc, int32_t shift, int32_t nchunk, int32_t* aux) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c <= nchunk;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t key = c << shift;
        int32_t lo = 0, hi = nzc;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if ((int64_t)jc[mid] < key) lo = mid + 1;
            else hi = mid;
        }
        aux[c] = lo;
    }
}

__global__ void k_validate_jc(const int32_t* jc, int32_t nzc, int32_t n, Ctrl* ctrl) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nzc; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = jc[k];
        if (j < 0 || j >= n || (k + 1 < nzc && jc[k + 1] <= j)) atomicOr(&ctrl->err, ERR_CSC);
    }
}

// Word w of the bitmap with bits at or past n cleared.
__device__ __forceinline__ uint32_t word_in_range(const uint32_t* bits, int64_t w, int32_t n, bool& stray) {
    const int64_t nwords = ((int64_t)n + 31) >> 5;
    if (w >= nwords) return 0u;
    uint32_t v = bits[w];
    const int64_t top = (int64_t)n - (w << 5);   // valid bits in this word
    if (top < 32) {
        const uint32_t keep = (1u << top) - 1u;
        stray |= (v & ~keep) != 0u;
        v &= keep;
    }
    return v;
}

__global__ __launch_bounds__(kFmtBlock) void k_bits_count(const uint32_t* bits, int32_t n, int32_t* tile_counts,
                                                          Ctrl* ctrl) {
    __shared__ int s_tmp[kFmtBlock / kWave + 1];
    const int64_t w0 = (int64_t)blockIdx.x * kTileWords + (int64_t)threadIdx.x * kWordsPerThread;
    bool stray = false;
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < kWordsPerThread; ++i) cnt += __popc(word_in_range(bits, w0 + i, n, stray));
    if (stray) atomicOr(&ctrl->err, ERR_X_RANGE);
    int total;
    block_exclusive_i32<kFmtBlock>(cnt, s_tmp, total);
    if (threadIdx.x == 0) tile_counts[blockIdx.x] = total;
}

__global__ __launch_bounds__(kFmtBlock) void k_bits_emit(const uint32_t* bits, int32_t n, const int32_t* tile_counts,
                                                         int32_t ntiles, int32_t* out, int32_t* count) {
    __shared__ int s_tmp[kFmtBlock / kWave + 1];
    const int tile = blockIdx.x;
    // this tile's output offset: the bit counts of the tiles before it
    int before = 0;
    for (int t = threadIdx.x; t < tile; t += kFmtBlock) before += tile_counts[t];
    int base;
    block_exclusive_i32<kFmtBlock>(before, s_tmp, base);
    const int64_t w0 = (int64_t)tile * kTileWords + (int64_t)threadIdx.x * kWordsPerThread;
    bool stray = false;
    uint32_t v[kWordsPerThread];
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < kWordsPerThread; ++i) {
        v[i] = word_in_range(bits, w0 + i, n, stray);
        cnt += __popc(v[i]);
    }
    int tile_total;
    int p = base + block_exclusive_i32<kFmtBlock>(cnt, s_tmp, tile_total);
#pragma unroll
    for (int i = 0; i < kWordsPerThread; ++i) {
        uint32_t x = v[i];
        while (x) {
            const int b = __ffs(x) - 1;
            out[p++] = (int32_t)(((w0 + i) << 5) + b);
            x &= x - 1u;
        }
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) *count = base + tile_total;
}

inline int grid_of(int64_t count, int block) {
    int64_t g = (count + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

}  // namespace

int64_t bits_tiles(int64_t n) {
    const int64_t nwords = (n + 31) / 32;
    const int64_t t = (nwords + kTileWords - 1) / kTileWords;
    return t < 1 ? 1 : t;
}

hipError_t launch_dcsc_aux(const int32_t* jc, int32_t nzc, int32_t shift, int32_t nchunk, int32_t* aux,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_dcsc_aux, dim3(grid_of((int64_t)nchunk + 1, 256)), dim3(256), 0, s, jc, nzc, shift, nchunk,
                       aux);
    return hipGetLastError();
}

hipError_t launch_validate_jc(const int32_t* jc, int32_t nzc, int32_t n, Ctrl* ctrl, hipStream_t s) {
    if (nzc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate_jc, dim3(grid_of(nzc, 256)), dim3(256), 0, s, jc, nzc, n, ctrl);
    return hipGetLastError();
}

hipError_t launch_bits_to_list(const uint32_t* bits, int32_t n, int32_t* out, int32_t* count, int32_t* tile_counts,
                               Ctrl* ctrl, hipStream_t s) {
    const int64_t nt = bits_tiles(n);
    hipLaunchKernelGGL(k_bits_count, dim3((unsigned)nt), dim3(kFmtBlock), 0, s, bits, n, tile_counts, ctrl);
    hipLaunchKernelGGL(k_bits_emit, dim3((unsigned)nt), dim3(kFmtBlock), 0, s, bits, n, tile_counts, (int32_t)nt, out,
                       count);
    return hipGetLastError();
}

}  // namespace spv
