// Data-driven (delta) PageRank around the SpMSpV hot path.  The paper names
// PageRank among the data-driven uses of SpMSpV, where a vertex stops
// sending updates once its value has converged (Introduction); the rule
// implemented is:
//   rank = 0, delta = (1 - d) / n everywhere, every vertex active;
//   each step: rank += delta; x = { (j, d * delta(j) / outdeg(j)) : j active,
//   outdeg(j) > 0 }; delta = A x (plus-times SpMSpV, structural pattern);
//   j is active next when delta(j) > tol * rank(j) (rank before adding).
// Only the entries of the current x and y are touched per step.  The x list
// is appended in any order (one counter update per wave).

#include "internal.h"

namespace spv {

namespace {

__device__ __forceinline__ void append(bool take, int32_t j, float v, int32_t* x_idx, float* x_val, Ctrl* ctrl) {
    const int lane = threadIdx.x & 63;
    const uint64_t vote = __ballot(take);
    int32_t first = 0;
    if (lane == 0 && vote) first = atomicAdd(&ctrl->gen_count, (int32_t)__popcll(vote));
    first = __shfl(first, 0, 64);
    if (take) {
        const int p = first + (int)__popcll(vote & ((1ull << lane) - 1ull));
        x_idx[p] = j;
        x_val[p] = v;
    }
}

__global__ void k_pr_init(int32_t n, const int32_t* colptr, float d, float* rank, int32_t* x_idx, float* x_val,
                          Ctrl* ctrl) {
    const float base = (1.0f - d) / (float)n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < n; b += stride) {
        const int64_t j = b + threadIdx.x;
        int32_t len = 0;
        if (j < n) {
            rank[j] = base;
            len = colptr[j + 1] - colptr[j];
        }
        append(j < n && len > 0, (int32_t)j, len > 0 ? d * base / (float)len : 0.f, x_idx, x_val, ctrl);
    }
}

__global__ void k_pr_update(const int32_t* colptr, float d, float tol, float* rank, const int32_t* y_idx,
                            const float* y_val, int32_t* x_idx, float* x_val, Ctrl* ctrl) {
    const int64_t cnt = __hip_atomic_load(&ctrl->nnz_y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t f = __hip_atomic_load(&ctrl->f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (f <= 0) return;   // the multiply was a no-op; y holds stale entries
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < cnt; b += stride) {
        const int64_t p = b + threadIdx.x;
        bool take = false;
        int32_t i = 0;
        float out = 0.f;
        if (p < cnt) {
            i = y_idx[p];
            const float v = y_val[p];
            const float r = rank[i];
            rank[i] = r + v;
            const int32_t len = colptr[i + 1] - colptr[i];
            take = v > tol * r && len > 0;
            out = take ? d * v / (float)len : 0.f;
        }
        append(take, i, out, x_idx, x_val, ctrl);
    }
}

// Next frontier length; counts the multiply that just ran if it had input.
__global__ void k_pr_publish(Ctrl* ctrl) {
    if (threadIdx.x == 0) {
        const int32_t fp = __hip_atomic_load(&ctrl->f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t nx = __hip_atomic_load(&ctrl->gen_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (fp > 0) __hip_atomic_store(&ctrl->level, ctrl->level + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl->f, nx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl->gen_count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_pr_reset(Ctrl* ctrl) {
    if (threadIdx.x == 0) {
        ctrl->f = 0;
        ctrl->level = 0;
        ctrl->gen_count = 0;
        ctrl->nnz_y = 0;
    }
}

inline int grid_of(int64_t count) {
    int64_t g = (count + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

}  // namespace

hipError_t launch_pr_init(int32_t n, const int32_t* colptr, float d, float* rank, int32_t* x_idx, float* x_val,
                          Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_pr_reset, dim3(1), dim3(64), 0, s, ctrl);
    hipLaunchKernelGGL(k_pr_init, dim3(grid_of(n)), dim3(256), 0, s, n, colptr, d, rank, x_idx, x_val, ctrl);
    hipLaunchKernelGGL(k_pr_publish, dim3(1), dim3(64), 0, s, ctrl);
    return hipGetLastError();
}

hipError_t launch_pr_update(int32_t n, const int32_t* colptr, float d, float tol, float* rank, const int32_t* y_idx,
                            const float* y_val, int32_t* x_idx, float* x_val, Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_pr_update, dim3(grid_of(n)), dim3(256), 0, s, colptr, d, tol, rank, y_idx, y_val, x_idx,
                       x_val, ctrl);
    hipLaunchKernelGGL(k_pr_publish, dim3(1), dim3(64), 0, s, ctrl);
    return hipGetLastError();
}

}  // namespace spv
