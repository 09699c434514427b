// Set-up kernels: run once per matrix (spmspv_create) or once per BFS.
// Not on the per-multiply path.

#include "decide.h"

namespace spv {

namespace {

constexpr int kSetupBlock = 256;
constexpr int kScanBlk = 1024;
constexpr int kScanPer = 4;
constexpr int kScanSpan = kScanBlk * kScanPer;

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// counts[r] += 1 for every row id r (counts has m+1 zeroed entries).
__global__ void k_row_counts(const int32_t* rowids, int64_t nnz, int32_t m, int32_t* counts, Ctrl* ctrl) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rowids[q];
        if (r >= 0 && r < m) atomicAdd(&counts[r], 1);
        else atomicOr(&ctrl->err, ERR_ROW_RANGE);
    }
}

// colptr[0] == 0, colptr monotone, colptr[n] == nnz; also the longest column.
__global__ void k_validate_colptr(const int32_t* colptr, int32_t n, int64_t nnz, Ctrl* ctrl, int32_t* maxout) {
    int lmax = 0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = colptr[j], b = colptr[j + 1];
        if (b < a) atomicOr(&ctrl->err, ERR_CSC);
        lmax = max(lmax, b - a);
        if (j == 0 && a != 0) atomicOr(&ctrl->err, ERR_CSC);
        if (j == n - 1 && (int64_t)b != nnz) atomicOr(&ctrl->err, ERR_CSC);
    }
    if (lmax > 0) atomicMax(maxout, lmax);
}

__device__ int block_scan_excl(int v, int* s) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            const int t = s[w];
            s[w] = acc;
            acc += t;
        }
        s[16] = acc;
    }
    __syncthreads();
    const int r = s[wid] + x - v;
    return r;
}

__global__ __launch_bounds__(kScanBlk) void k_span_sums(const int32_t* data, int64_t count, int32_t* partials) {
    __shared__ int s[17];
    const int64_t base = (int64_t)blockIdx.x * kScanSpan + threadIdx.x * kScanPer;
    int v = 0;
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < count) v += data[base + i];
    block_scan_excl(v, s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s[16];
}

__global__ __launch_bounds__(kScanBlk) void k_scan_partials(int32_t* partials, int64_t np) {
    __shared__ int s[17];
    int carry = 0;
    for (int64_t b0 = 0; b0 < np; b0 += kScanBlk) {
        const int64_t i = b0 + threadIdx.x;
        const int v = i < np ? partials[i] : 0;
        const int e = block_scan_excl(v, s);
        const int tot = s[16];
        if (i < np) partials[i] = carry + e;
        carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanBlk) void k_span_apply(int32_t* data, int64_t count, const int32_t* partials) {
    __shared__ int s[17];
    const int64_t base = (int64_t)blockIdx.x * kScanSpan + threadIdx.x * kScanPer;
    int v[kScanPer];
    int sum = 0;
    for (int i = 0; i < kScanPer; ++i) {
        v[i] = base + i < count ? data[base + i] : 0;
        sum += v[i];
    }
    int run = block_scan_excl(sum, s) + partials[blockIdx.x];
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < count) data[base + i] = run;
        run += v[i];
    }
}

__global__ void k_bfs_init(int32_t n, int32_t root, int32_t* level, int32_t* parent, uint32_t* visited,
                           uint32_t* xbits, int32_t* frontier, Ctrl* ctrl, int64_t nnz, int policy) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
        level[v] = (v == root) ? 0 : -1;
        if (parent) parent[v] = (v == root) ? root : -1;
    }
    const int64_t nw = ((int64_t)n + 31) >> 5;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nw; w += stride) {
        visited[w] = (w == (root >> 5)) ? (1u << (root & 31)) : 0u;
        if (xbits) xbits[w] = 0u;   // a BFS that stopped early may have left a pull frontier there
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->chain_ready = 0;
        ctrl->chain_word = 0;
        frontier[0] = root;
        ctrl->f = 1;
        ctrl->level = 0;
        ctrl->bfs_level = level;
        ctrl->bfs_parent = parent;
        ctrl->dir = 0;
        ctrl->policy = policy;
        ctrl->edges_left = nnz;
    }
}

// Multi-source BFS start: source x owns level / parent entries
// [x * n, (x + 1) * n) and visited words [x * mask_words, ...); its frontier
// is its root, so the first batched frontier is roots[0 .. nsrc).
__global__ void k_msbfs_init(int32_t n, int nsrc, const int32_t* roots, int32_t* level, int32_t* parent,
                             uint32_t* visited, int32_t mask_words, int32_t* frontier, int64_t* xoff, Ctrl* ctrl) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t total = (int64_t)nsrc * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += stride) {
        const int64_t x = i / n;
        const int32_t v = (int32_t)(i - x * n);
        const int32_t r = roots[x];
        level[i] = v == r ? 0 : -1;
        if (parent) parent[i] = v == r ? r : -1;
    }
    const int64_t words = (int64_t)nsrc * mask_words;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += stride) {
        const int64_t x = i / mask_words;
        const int64_t w = i - x * mask_words;
        const int32_t r = roots[x];
        visited[i] = w == (r >> 5) ? (1u << (r & 31)) : 0u;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= nsrc; i += stride) {
        if (i < nsrc) frontier[i] = roots[i];
        xoff[i] = i;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->f = nsrc;
        ctrl->level = 0;
        ctrl->bfs_level = level;
        ctrl->bfs_parent = parent;
        ctrl->dir = 0;
        ctrl->policy = 0;
    }
}

// Tuning input: column j is drawn with probability `thresh / 2^32`, with a
// value in (0, 1] on a 2^-24 grid, both from the SplitMix64 finaliser of
// (seed, j).  Entries are appended in any order, one counter update per wave.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void k_gen_x(int32_t n, uint64_t thresh, uint64_t seed, int32_t* x_idx, float* x_val, Ctrl* ctrl) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        const int64_t j = base + threadIdx.x;
        const uint64_t h = j < n ? mix64(seed * 0x2545f4914f6cdd1dull + (uint64_t)j) : 0ull;
        const bool take = j < n && (h >> 32) < thresh;
        const uint64_t vote = __ballot(take);
        int32_t first = 0;
        if (lane == 0 && vote) first = atomicAdd(&ctrl->gen_count, (int32_t)__popcll(vote));
        first = __shfl(first, 0, 64);
        if (take) {
            const int p = first + (int)__popcll(vote & ((1ull << lane) - 1ull));
            x_idx[p] = (int32_t)j;
            if (x_val) x_val[p] = (float)((h & 0xffffffull) + 1ull) * (1.0f / 16777216.0f);
        }
    }
}

// Direction of the next BFS level from the frontier just scanned (the
// frontier-edge rule of heuristic_step), unless the scan of this level
// already took the decision.
__global__ void k_decide(Ctrl* ctrl, int32_t n, int64_t nnz) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (consume_chain(ctrl)) return;
    heuristic_step(ctrl, n, dc_ld(&ctrl->f), dc_ld(&ctrl->W));
    (void)nnz;
}

inline int grid_for(int64_t count, int block, int cap = 4096) {
    int64_t g = (count + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, kSetupBlock)), dim3(kSetupBlock), 0, s, p, v, count);
    return hipGetLastError();
}

hipError_t launch_row_counts(const int32_t* rowids, int64_t nnz, int32_t m, int32_t* counts, Ctrl* ctrl,
                             hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_counts, dim3(grid_for(nnz, kSetupBlock)), dim3(kSetupBlock), 0, s, rowids, nnz, m,
                       counts, ctrl);
    return hipGetLastError();
}

// In-place exclusive scan of `count` int32 values; `partials` needs
// ceil(count / 4096) entries.
hipError_t launch_exclusive_scan_i32(int32_t* data, int64_t count, int32_t* partials, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t np = (count + kScanSpan - 1) / kScanSpan;
    hipLaunchKernelGGL(k_span_sums, dim3((unsigned)np), dim3(kScanBlk), 0, s, data, count, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanBlk), 0, s, partials, np);
    hipLaunchKernelGGL(k_span_apply, dim3((unsigned)np), dim3(kScanBlk), 0, s, data, count, partials);
    return hipGetLastError();
}

// out[k] = a[k * (count - 1) / (K - 1)] for k < K (K >= 2, count >= 1):
// evenly spaced samples of a device array, first and last included.
__global__ void k_sample_i32(const int32_t* a, int64_t count, int32_t* out, int32_t K) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x)
        out[k] = count > 0 ? a[(int64_t)k * (count - 1) / (K - 1)] : 0;
}

hipError_t launch_sample_i32(const int32_t* a, int64_t count, int32_t* out, int32_t K, hipStream_t s) {
    if (K < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sample_i32, dim3((K + 255) / 256), dim3(256), 0, s, a, count, out, K);
    return hipGetLastError();
}

hipError_t launch_validate_colptr(const int32_t* colptr, int32_t n, int64_t nnz, Ctrl* ctrl, int32_t* maxout,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_validate_colptr, dim3(grid_for(n, kSetupBlock)), dim3(kSetupBlock), 0, s, colptr, n, nnz,
                       ctrl, maxout);
    return hipGetLastError();
}

hipError_t launch_decide(Ctrl* ctrl, int32_t n, int64_t nnz, hipStream_t s) {
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(64), 0, s, ctrl, n, nnz);
    return hipGetLastError();
}

hipError_t launch_bfs_init(int32_t n, int32_t root, int32_t* level, int32_t* parent, uint32_t* visited,
                           uint32_t* xbits, int32_t* frontier, Ctrl* ctrl, int64_t nnz, int policy, hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_init, dim3(grid_for(n, kSetupBlock)), dim3(kSetupBlock), 0, s, n, root, level, parent,
                       visited, xbits, frontier, ctrl, nnz, policy);
    return hipGetLastError();
}

hipError_t launch_msbfs_init(int32_t n, int nsrc, const int32_t* roots, int32_t* level, int32_t* parent,
                             uint32_t* visited, int32_t mask_words, int32_t* frontier, int64_t* xoff, Ctrl* ctrl,
                             hipStream_t s) {
    const int64_t total = (int64_t)nsrc * n;
    hipLaunchKernelGGL(k_msbfs_init, dim3(grid_for(total, kSetupBlock)), dim3(kSetupBlock), 0, s, n, nsrc, roots,
                       level, parent, visited, mask_words, frontier, xoff, ctrl);
    return hipGetLastError();
}

hipError_t launch_gen_x(int32_t n, double density, uint64_t seed, int32_t* x_idx, float* x_val, Ctrl* ctrl,
                        hipStream_t s) {
    double t = density * 4294967296.0;
    if (t < 0) t = 0;
    if (t > 4294967296.0) t = 4294967296.0;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(&ctrl->gen_count), 0u,
                       (int64_t)1);
    hipLaunchKernelGGL(k_gen_x, dim3(grid_for(n, kSetupBlock)), dim3(kSetupBlock), 0, s, n, (uint64_t)t, seed, x_idx,
                       x_val, ctrl);
    return hipGetLastError();
}

}  // namespace spv
