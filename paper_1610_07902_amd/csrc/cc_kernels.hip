// Connected components by data-driven label propagation around the SpMSpV
// hot path (the paper's introduction lists connected components among the
// data-driven uses of SpMSpV):
//   label(v) = v for every vertex; the first x lists every vertex with an
//   out-edge, valued by its label;
//   each step: y = A x over min-select2nd (y(i) = the smallest label among
//   x's in-neighbours of i); every i with y(i) < label(i) takes y(i) and
//   joins the next x (when it has out-edges); stop when x is empty.
// At the fixed point label(v) = the smallest vertex that reaches v (for a
// symmetric A, the smallest vertex of v's component).  Only the entries of
// the current x and y are touched per step; x is appended in any order
// (one counter update per wave).

#include "internal.h"

namespace spv {

namespace {

__device__ __forceinline__ void append(bool take, int32_t j, int32_t v, int32_t* x_idx, int32_t* x_val, Ctrl* ctrl) {
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

__global__ void k_cc_reset(Ctrl* ctrl) {
    if (threadIdx.x == 0) {
        ctrl->f = 0;
        ctrl->level = 0;
        ctrl->gen_count = 0;
        ctrl->nnz_y = 0;
    }
}

__global__ void k_cc_init(int32_t n, const int32_t* colptr, int32_t* label, int32_t* x_idx, int32_t* x_val,
                          Ctrl* ctrl) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < n; b += stride) {
        const int64_t v = b + threadIdx.x;
        bool take = false;
        if (v < n) {
            label[v] = (int32_t)v;
            take = colptr[v + 1] > colptr[v];
        }
        append(take, (int32_t)v, (int32_t)v, x_idx, x_val, ctrl);
    }
}

__global__ void k_cc_update(const int32_t* colptr, int32_t* label, const int32_t* y_idx, const int32_t* y_val,
                            int32_t* x_idx, int32_t* x_val, Ctrl* ctrl) {
    const int64_t cnt = __hip_atomic_load(&ctrl->nnz_y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t f = __hip_atomic_load(&ctrl->f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (f <= 0) return;   // the multiply was a no-op; y holds stale entries
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < cnt; b += stride) {
        const int64_t p = b + threadIdx.x;
        bool take = false;
        int32_t i = 0, v = 0;
        if (p < cnt) {
            i = y_idx[p];
            v = y_val[p];
            if (v < label[i]) {
                label[i] = v;   // i appears once in y: no other thread writes it
                take = colptr[i + 1] > colptr[i];
            }
        }
        append(take, i, v, x_idx, x_val, ctrl);
    }
}

// Next x length; counts the multiply that just ran if it had input.
__global__ void k_cc_publish(Ctrl* ctrl) {
    if (threadIdx.x == 0) {
        const int32_t fp = __hip_atomic_load(&ctrl->f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t nx = __hip_atomic_load(&ctrl->gen_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (fp > 0) __hip_atomic_store(&ctrl->level, ctrl->level + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl->f, nx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl->gen_count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

inline int grid_of(int64_t count) {
    int64_t g = (count + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

}  // namespace

hipError_t launch_cc_init(int32_t n, const int32_t* colptr, int32_t* label, int32_t* x_idx, int32_t* x_val,
                          Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_cc_reset, dim3(1), dim3(64), 0, s, ctrl);
    hipLaunchKernelGGL(k_cc_init, dim3(grid_of(n)), dim3(256), 0, s, n, colptr, label, x_idx, x_val, ctrl);
    hipLaunchKernelGGL(k_cc_publish, dim3(1), dim3(64), 0, s, ctrl);
    return hipGetLastError();
}

hipError_t launch_cc_update(int32_t n, const int32_t* colptr, int32_t* label, const int32_t* y_idx,
                            const int32_t* y_val, int32_t* x_idx, int32_t* x_val, Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_cc_update, dim3(grid_of(n)), dim3(256), 0, s, colptr, label, y_idx, y_val, x_idx, x_val,
                       ctrl);
    hipLaunchKernelGGL(k_cc_publish, dim3(1), dim3(64), 0, s, ctrl);
    return hipGetLastError();
}

}  // namespace spv
