// Masked multiply with accumulate and replace, w<mask, replace> = w accum
// (A x): the generalisation of the BFS visited mask that the paper's
// conclusions name as future work, with the mask / accumulate / replace
// rules of the GraphBLAS standard.
//
// The mask enters the product itself: its rows become a bitmap
// (k_mask_bits) and the bucketing drops every product whose row is outside
// the mask (as the BFS drops visited rows), so the multiply yields t, the
// product restricted to the mask, ascending.  k_combine then merges t with
// the accumulation input w (ascending) by merge path: each thread takes
// kCombineItems consecutive entries of the merged order (w before t on
// equal rows, so a row present in both is a w entry directly followed by
// its t entry) and applies the rules entry by entry:
//   t entry: its row is in the mask; output accum(w, t) when w has the row
//            and an operator is given, else t;
//   w entry without a t partner: output w when the row is in the mask and
//            an operator is given (z = w there), or when it is outside the
//            mask and replace is off; else nothing.
// Output positions come from a block scan and a decoupled look-back over
// tiles, so y is ascending.

#include "device_ops.h"

namespace spv {

namespace {

constexpr int kCBlock = 256;
constexpr int kCItems = kCombineTile / kCBlock;
enum { ACC_NONE = 0, ACC_ADD = 1, ACC_FIRST = 2, ACC_SECOND = 3 };

__global__ void k_mask_bits(const int32_t* idx, const uint8_t* val, int64_t count, int32_t m, uint32_t* bits,
                            uint32_t* err) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count; p += stride) {
        const int32_t i = idx[p];
        if (i < 0 || i >= m) {
            atomicOr(err, ERR_INDEX_RANGE);
            continue;
        }
        if (!val || val[p] != 0) atomicOr(&bits[i >> 5], 1u << (i & 31));
    }
}

template <int SR>
__device__ __forceinline__ uint32_t load_value(const void* p, int64_t k) {
    if constexpr (SR == SR_OR_AND) return reinterpret_cast<const uint8_t*>(p)[k] ? 1u : 0u;
    else return reinterpret_cast<const uint32_t*>(p)[k];
}

// The semiring's Add on two values.
template <int SR>
__device__ __forceinline__ uint32_t add_values(uint32_t w, uint32_t t) {
    if constexpr (SR == SR_PLUS_TIMES) return __float_as_uint(__fadd_rn(__uint_as_float(w), __uint_as_float(t)));
    else if constexpr (SR == SR_MIN_SELECT2ND) return (uint32_t)min((int32_t)w, (int32_t)t);
    else return (w | t) ? 1u : 0u;
}

// Walks merged entries [d0, d1) from the merge-path split (i, j) and calls
// emit(row, value) for every output entry, in order.  Sets `disorder` when
// w's indices are not strictly ascending.
template <int SR, typename Emit>
__device__ __forceinline__ void walk(const CombineArgs& a, int64_t nt, int64_t i, int64_t j, int64_t d0, int64_t d1,
                                     bool& disorder, Emit emit) {
    for (int64_t d = d0; d < d1; ++d) {
        const bool take_w = j < a.nw && (i >= nt || a.w_idx[j] <= a.t_idx[i]);
        if (take_w) {
            const int32_t row = a.w_idx[j];
            if (j + 1 < a.nw && a.w_idx[j + 1] <= row) disorder = true;
            const bool paired = i < nt && a.t_idx[i] == row;
            if (!paired) {
                const bool in_mask = a.mbits ? (((a.mbits[row >> 5] >> (row & 31)) & 1u) != (uint32_t)a.complement)
                                             : !a.complement;
                if (in_mask ? a.accum != ACC_NONE : !a.replace) emit(row, load_value<SR>(a.w_val, j));
            }
            ++j;
        } else {
            const int32_t row = a.t_idx[i];
            uint32_t v = load_value<SR>(a.t_val, i);
            if (a.accum != ACC_NONE && j > 0 && a.w_idx[j - 1] == row) {
                const uint32_t wv = load_value<SR>(a.w_val, j - 1);
                v = a.accum == ACC_FIRST ? wv : (a.accum == ACC_SECOND ? v : add_values<SR>(wv, v));
            }
            emit(row, v);
            ++i;
        }
    }
}

template <int SR>
__global__ __launch_bounds__(kCBlock) void k_combine(CombineArgs a) {
    __shared__ int s_tmp[kCBlock / kWave + 1];
    __shared__ int64_t s_excl;
    const int tid = threadIdx.x;
    const int64_t nt = __hip_atomic_load(a.d_nt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t total = nt + a.nw;
    const int64_t ntiles = (total + kCombineTile - 1) / kCombineTile;
    if (ntiles == 0) {
        if (blockIdx.x == 0 && tid == 0) {
            __hip_atomic_store(&a.ctrl->nnz_y, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a.d_nnz_y) *a.d_nnz_y = 0;
        }
        return;
    }
    if (ntiles > a.lb_n) {   // more tiles than look-back words: not reached (sized for t and w at their largest)
        if (blockIdx.x == 0 && tid == 0) atomicOr(&a.ctrl->err, ERR_SPIN);
        return;
    }
    bool disorder = false;
    // Tiles in blockIdx order: a tile's look-back predecessors belong to
    // workgroups dispatched no later than its own.
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t d0 = tile * kCombineTile + (int64_t)tid * kCItems;
        const int64_t d1 = d0 + kCItems < total ? d0 + kCItems : total;
        int64_t i = 0, j = 0;
        int cnt = 0;
        if (d0 < total) {
            // merge path: the first d0 merged entries are t[0, i) and w[0, j)
            int64_t lo = d0 - nt > 0 ? d0 - nt : 0, hi = d0 < a.nw ? d0 : a.nw;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                const int64_t ii = d0 - mid;
                if (ii > 0 && mid < a.nw && a.t_idx[ii - 1] >= a.w_idx[mid]) lo = mid + 1;
                else hi = mid;
            }
            j = lo;
            i = d0 - j;
            walk<SR>(a, nt, i, j, d0, d1, disorder, [&](int32_t, uint32_t) { ++cnt; });
        }
        int tile_total;
        const int pre = block_exclusive_i32<kCBlock>(cnt, s_tmp, tile_total);
        if (tid < kWave) {
            const uint64_t e = lookback(a.lb, (int)tile, (uint64_t)tile_total, &a.ctrl->err);
            if (tid == 0) s_excl = (int64_t)e;
        }
        __syncthreads();
        const int64_t base = s_excl + pre;
        if (d0 < total) {
            int64_t k = 0;
            walk<SR>(a, nt, i, j, d0, d1, disorder, [&](int32_t row, uint32_t v) {
                const int64_t o = base + k++;
                if (o < a.y_cap) {
                    a.y_idx[o] = row;
                    if (a.y_val) store_value<SR>(a.y_val, o, v);
                }
            });
        }
        if (tile == ntiles - 1 && tid == kCBlock - 1) {
            const int64_t out = s_excl + pre + cnt;
            __hip_atomic_store(&a.ctrl->nnz_y, out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a.d_nnz_y) *a.d_nnz_y = out;
        }
        __syncthreads();
    }
    if (disorder) atomicOr(&a.ctrl->err, ERR_ORDER);
}

}  // namespace

hipError_t launch_mask_bits(const int32_t* idx, const uint8_t* val, int64_t count, int32_t m, uint32_t* bits,
                            uint32_t* err, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t grid = (count + 255) / 256;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_mask_bits, dim3((unsigned)grid), dim3(256), 0, s, idx, val, count, m, bits, err);
    return hipGetLastError();
}

hipError_t launch_combine(const CombineArgs& a, int semiring, int grid, hipStream_t s) {
    if (grid < 1) return hipErrorInvalidValue;
    switch (semiring) {
        case SR_PLUS_TIMES: hipLaunchKernelGGL(k_combine<SR_PLUS_TIMES>, dim3(grid), dim3(kCBlock), 0, s, a); break;
        case SR_MIN_SELECT2ND:
            hipLaunchKernelGGL(k_combine<SR_MIN_SELECT2ND>, dim3(grid), dim3(kCBlock), 0, s, a);
            break;
        default: hipLaunchKernelGGL(k_combine<SR_OR_AND>, dim3(grid), dim3(kCBlock), 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace spv
