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
// kCItems consecutive entries of the merged order (w before t on equal
// rows, so a row present in both is a w entry directly followed by its t
// entry), read from the tile's window staged in LDS, and applies the rules
// entry by entry:
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

// Mask list -> byte map: one byte store per listed row (a device-scope
// atomic OR per row into the bitmap costs several times more on random
// rows).
__global__ void k_mask_bytes(const int32_t* idx, const uint8_t* val, int64_t count, int32_t m, uint8_t* bytes,
                             uint32_t* err) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count; p += stride) {
        const int32_t i = idx[p];
        if (i < 0 || i >= m) {
            atomicOr(err, ERR_INDEX_RANGE);
            continue;
        }
        if (!val || val[p] != 0) bytes[i] = 1;
    }
}

// Byte map -> bitmap, one 32-bit word per thread from 32 bytes (each 0 or
// 1), clearing the bytes for the next call.
__global__ void k_pack_mask(uint8_t* bytes, int64_t nwords, uint32_t* bits) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        uint4* src = reinterpret_cast<uint4*>(bytes + (w << 5));
        const uint4 lo = src[0], hi = src[1];
        const uint32_t q[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
        uint32_t word = 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t v = q[k];
            const uint32_t nib = (v & 1u) | ((v >> 7) & 2u) | ((v >> 14) & 4u) | ((v >> 21) & 8u);
            word |= nib << (4 * k);
        }
        bits[w] = word;
        if (word) {
            src[0] = make_uint4(0u, 0u, 0u, 0u);
            src[1] = make_uint4(0u, 0u, 0u, 0u);
        }
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

// Merge-path split of the first d merged entries: t[0, i) and w[0, j)
// with i + j = d (w before t on equal rows), j the first position where
// t[d - j - 1] < w[j].  One wave searches together: each round its 64
// lanes test 64 evenly spaced candidates and keep the gap between the last
// lane whose test holds and the next, so a range of 2^22 takes four
// rounds of dependent loads instead of 22.  The result stays in [lo, hi]
// whatever the data (a w that is not ascending is reported elsewhere).
__device__ __forceinline__ int64_t split_w(const CombineArgs& a, int64_t nt, int64_t d, int lane) {
    int64_t lo = d - nt > 0 ? d - nt : 0, hi = d < a.nw ? d : a.nw;
    while (lo < hi) {
        const int64_t step = (hi - lo + kWave - 1) / kWave;
        const int64_t j = lo + (int64_t)lane * step;
        const bool c = j < hi && a.t_idx[d - j - 1] >= a.w_idx[j];
        const int p = __popcll(__ballot(c));
        if (p == 0) {
            hi = lo;
        } else {
            const int64_t nlo = lo + (int64_t)(p - 1) * step + 1;
            const int64_t nhi = lo + (int64_t)p * step;
            lo = nlo;
            hi = nhi < hi ? nhi : hi;
        }
    }
    return lo;
}

// One tile of kCombineTile merged entries per workgroup.  The tile's t and w
// entries, with one w entry before and one t and w entry after (a w entry
// and its t partner can straddle the boundary), are staged in LDS with
// coalesced loads; each thread then finds its kCItems entries by a merge
// path inside LDS, walks them once into registers, and writes them at its
// offset from a block scan and the look-back over tiles.
template <int SR>
__global__ __launch_bounds__(kCBlock) void k_combine(CombineArgs a) {
    constexpr int kWin = kCombineTile + 2;
    __shared__ int32_t s_wi[kWin], s_ti[kWin];
    __shared__ uint32_t s_wv[kWin], s_tv[kWin];
    __shared__ int s_tmp[kCBlock / kWave + 1];
    __shared__ int64_t s_split[2];
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
        const int64_t d0 = tile * kCombineTile;
        const int64_t d1 = d0 + kCombineTile < total ? d0 + kCombineTile : total;
        if (tid < 2 * kWave) {
            const int64_t jj = split_w(a, nt, tid < kWave ? d0 : d1, tid & (kWave - 1));
            if ((tid & (kWave - 1)) == 0) s_split[tid / kWave] = jj;
        }
        __syncthreads();
        const int64_t j0 = s_split[0], j1 = s_split[1];
        const int64_t i0 = d0 - j0, i1 = d1 - j1;
        // windows: w[wb, we) and t[i0, te)
        const int64_t wb = j0 > 0 ? j0 - 1 : 0;
        const int64_t we = j1 + 1 < a.nw ? j1 + 1 : a.nw;
        const int64_t te = i1 + 1 < nt ? i1 + 1 : nt;
        // (both windows hold at most kWin entries for an ascending w; the
        // clamps keep any other input inside the LDS arrays)
        const int nwin = (int)max((int64_t)0, min((int64_t)kWin, we - wb));
        const int ntwin = (int)max((int64_t)0, min((int64_t)kWin, te - i0));
        for (int k = tid; k < nwin; k += kCBlock) {
            s_wi[k] = a.w_idx[wb + k];
            s_wv[k] = load_value<SR>(a.w_val, wb + k);
        }
        for (int k = tid; k < ntwin; k += kCBlock) {
            s_ti[k] = a.t_idx[i0 + k];
            s_tv[k] = load_value<SR>(a.t_val, i0 + k);
        }
        __syncthreads();
        // this thread's entries: local diagonal dl of the tile
        const int nt_l = (int)max((int64_t)0, min((int64_t)kCombineTile, i1 - i0));
        const int nw_l = (int)max((int64_t)0, min((int64_t)kCombineTile, j1 - j0));
        const int dl = tid * kCItems;
        const int dn = (int)(d1 - d0);
        const int ow = (int)(j0 - wb);   // s_wi[ow + b] = w_idx[j0 + b]
        int32_t rows[kCItems];
        uint32_t vals[kCItems];
        int cnt = 0;
        if (dl < dn) {
            int lo = dl - nt_l > 0 ? dl - nt_l : 0, hi = dl < nw_l ? dl : nw_l;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_ti[dl - mid - 1] >= s_wi[ow + mid]) lo = mid + 1;
                else hi = mid;
            }
            int b = lo, c = dl - lo;              // local positions in w and t
            const int dend = dl + kCItems < dn ? dl + kCItems : dn;
#pragma unroll
            for (int q = 0; q < kCItems; ++q) {
                if (dl + q >= dend) break;
                const int64_t jg = j0 + b, ig = i0 + c;
                const bool t_ok = ig < nt && c < ntwin;
                const bool take_w = jg < a.nw && ow + b < nwin && (!t_ok || s_wi[ow + b] <= s_ti[c]);
                if (!take_w && !t_ok) break;   // only for a w that is not ascending
                if (take_w) {
                    const int32_t row = s_wi[ow + b];
                    if (jg + 1 < a.nw && (ow + b + 1 >= nwin || s_wi[ow + b + 1] <= row)) disorder = true;
                    const bool paired = t_ok && s_ti[c] == row;
                    if (!paired) {
                        const bool in_mask = a.mbits ? (((a.mbits[row >> 5] >> (row & 31)) & 1u) !=
                                                         (uint32_t)a.complement)
                                                     : !a.complement;
                        if (in_mask ? a.accum != ACC_NONE : !a.replace) {
                            rows[cnt] = row;
                            vals[cnt] = s_wv[ow + b];
                            ++cnt;
                        }
                    }
                    ++b;
                } else {
                    const int32_t row = s_ti[c];
                    uint32_t v = s_tv[c];
                    if (a.accum != ACC_NONE && jg > 0 && s_wi[ow + b - 1] == row) {
                        const uint32_t wv = s_wv[ow + b - 1];
                        v = a.accum == ACC_FIRST ? wv : (a.accum == ACC_SECOND ? v : add_values<SR>(wv, v));
                    }
                    rows[cnt] = row;
                    vals[cnt] = v;
                    ++cnt;
                    ++c;
                }
            }
        }
        int tile_total;
        const int pre = block_exclusive_i32<kCBlock>(cnt, s_tmp, tile_total);
        if (tid < kWave) {
            const uint64_t e = lookback(a.lb, (int)tile, (uint64_t)tile_total, &a.ctrl->err);
            if (tid == 0) s_excl = (int64_t)e;
        }
        __syncthreads();
        const int64_t base = s_excl + pre;
#pragma unroll
        for (int q = 0; q < kCItems; ++q) {
            if (q >= cnt) break;
            const int64_t o = base + q;
            if (o < a.y_cap) {
                a.y_idx[o] = rows[q];
                if (a.y_val) store_value<SR>(a.y_val, o, vals[q]);
            }
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

hipError_t launch_mask_bits(const int32_t* idx, const uint8_t* val, int64_t count, int32_t m, uint8_t* bytes,
                            uint32_t* bits, uint32_t* err, hipStream_t s) {
    if (count > 0) {
        int64_t grid = (count + 255) / 256;
        if (grid > 8192) grid = 8192;
        hipLaunchKernelGGL(k_mask_bytes, dim3((unsigned)grid), dim3(256), 0, s, idx, val, count, m, bytes, err);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t nwords = ((int64_t)m + 31) / 32;
    if (nwords == 0) return hipSuccess;
    int64_t grid = (nwords + 255) / 256;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_pack_mask, dim3((unsigned)grid), dim3(256), 0, s, bytes, nwords, bits);
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
