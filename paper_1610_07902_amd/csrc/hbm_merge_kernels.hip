// Merge variant 1: the sparse accumulator in HBM.  Algorithm 1's step 2
// keeps a SPA per bucket in memory; here it is one dense m-long array of
// cells (and a touched-row bitmap) that every bucket shares, since buckets
// own disjoint rows.  It serves buckets wider than an LDS tile, so that a
// schedule can use as few buckets as it likes (down to one).
//   k_hmerge_acc  a bucket's entries are split over h_split workgroups;
//                 every entry updates its row's cell with a global atomic
//                 (fp64 add, int32 min, or a value bit) and sets the row's
//                 touched bit.
//   k_hmerge_out  tiles of kHTileRows rows walk the touched bitmap in
//                 order: bit counts, a block scan and a decoupled look-back
//                 over tiles give each row its place in y (Algorithm 1 step
//                 3, ascending); the cell and the bits are returned to the
//                 empty state for the next call.

#include "device_ops.h"

namespace spv {

namespace {

constexpr int kHBlock = 256;
constexpr int kHWords = kHTileRows / 32 / kHBlock;   // bitmap words per thread in the walk (8)
static_assert(kHWords * 32 * kHBlock == kHTileRows, "tile shape");

template <int SR>
__global__ __launch_bounds__(kHBlock) void k_hmerge_acc(MergeArgs a) {
    if (a.gate && ld_ctrl(&a.ctrl->dir) != 0) return;   // this BFS level runs pull
    const int W = ld_ctrl(&a.ctrl->W);
    if (W == 0) return;
    const int b = blockIdx.x / a.h_split, part = blockIdx.x - b * a.h_split;
    const int tl = a.tile_log2;
    const int64_t row0 = (int64_t)b << tl;
    const int64_t row1 = min(row0 + (int64_t(1) << tl), (int64_t)a.m);
    const int cnt_raw = ld_ctrl(&a.cursor[b]);
    const int64_t base = a.rcp[row0];
    const int cap = a.rcp[row1] - a.rcp[row0];
    // slots past the bucket's capacity exist only after an overflow
    // (duplicate x indices): never read past the bucket
    const int cnt = min(cnt_raw, cap);
    if (cnt_raw > cap && part == 0 && threadIdx.x == 0) atomicOr(&a.ctrl->err, ERR_BUCKET_OVERFLOW);
    const int per = (cnt + a.h_split - 1) / a.h_split;
    const int e0 = part * per, e1 = min(cnt, e0 + per);
    bool bad = false;
    for (int e = e0 + threadIdx.x; e < e1; e += kHBlock) {
        const uint2 ent = a.buckets[base + e];
        const int64_t row = (int32_t)ent.x;
        if (row < row0 || row >= row1) {   // unwritten slot after an overflow
            bad = true;
            continue;
        }
        if constexpr (SR == SR_PLUS_TIMES) unsafeAtomicAdd(&a.h_f64[row], (double)__uint_as_float(ent.y));
        else if constexpr (SR == SR_MIN_SELECT2ND) atomicMin(&a.h_i32[row], (int32_t)ent.y);
        else if (ent.y) atomicOr(&a.h_orbits[row >> 5], 1u << (row & 31));
        atomicOr(&a.h_touched[row >> 5], 1u << (row & 31));
    }
    if (bad) atomicOr(&a.ctrl->err, ERR_BUCKET_OVERFLOW);
}

template <int SR, bool BFS>
__global__ __launch_bounds__(kHBlock) void k_hmerge_out(MergeArgs a) {
    __shared__ int s_tmp[kHBlock / kWave + 1];
    __shared__ int64_t s_excl;
    if (a.gate && ld_ctrl(&a.ctrl->dir) != 0) return;
    const int tid = threadIdx.x;
    const int tile = blockIdx.x;
    const int64_t nwords = ((int64_t)a.m + 31) >> 5;
    const int64_t w0 = (int64_t)tile * (kHTileRows / 32) + (int64_t)tid * kHWords;
    uint32_t bits[kHWords];
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < kHWords; ++i) {
        bits[i] = w0 + i < nwords ? a.h_touched[w0 + i] : 0u;
        cnt += __popc(bits[i]);
        if (!BFS && a.y_bits && w0 + i < nwords) a.y_bits[w0 + i] = bits[i];
    }
    int tile_total;
    const int pre = block_exclusive_i32<kHBlock>(cnt, s_tmp, tile_total);
    if (tid < kWave) {
        const uint64_t e = lookback(a.lb3, tile, (uint64_t)tile_total, &a.ctrl->err);
        if (tid == 0) {
            s_excl = (int64_t)e;
            if (tile == (int)gridDim.x - 1) {
                const int64_t total = (int64_t)e + tile_total;
                a.ctrl->nnz_y = total;
                if (a.d_nnz_y) *a.d_nnz_y = total;
                if (a.set_f) st_ctrl(&a.ctrl->f, (int32_t)total);
            }
        }
    }
    __syncthreads();
    int64_t o = s_excl + pre;
    const int lvl = BFS ? ld_ctrl(&a.ctrl->level) : 0;
    int32_t* level = BFS ? ld_ctrl_ptr(&a.ctrl->bfs_level) : nullptr;
    int32_t* parent = BFS ? ld_ctrl_ptr(&a.ctrl->bfs_parent) : nullptr;
#pragma unroll
    for (int i = 0; i < kHWords; ++i) {
        if (!bits[i]) continue;
        const int64_t w = w0 + i;
        uint32_t vbits = 0u;
        if constexpr (SR == SR_OR_AND) vbits = a.h_orbits[w];
        uint32_t rest = bits[i];
        while (rest) {
            const int bit = __ffs(rest) - 1;
            rest &= rest - 1u;
            const int64_t row = (w << 5) + bit;
            uint32_t v;
            if constexpr (SR == SR_PLUS_TIMES) {
                v = __float_as_uint((float)a.h_f64[row]);
                a.h_f64[row] = -0.0;
            } else if constexpr (SR == SR_MIN_SELECT2ND) {
                v = (uint32_t)a.h_i32[row];
                a.h_i32[row] = 0x7fffffff;
            } else {
                v = (vbits >> bit) & 1u;
            }
            if (o < a.y_cap) {
                a.y_idx[o] = (int32_t)row;
                if (a.y_val) store_value<SR>(a.y_val, o, v);
            }
            if (BFS) {
                level[row] = lvl;
                if (parent) parent[row] = (int32_t)v;
            }
            ++o;
        }
        if (BFS) a.visited[w] |= bits[i];
        a.h_touched[w] = 0u;
        if constexpr (SR == SR_OR_AND) a.h_orbits[w] = 0u;
    }
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <int SR>
hipError_t hmerge(const MergeArgs& a, bool bfs, hipStream_t s) {
    hipLaunchKernelGGL(k_hmerge_acc<SR>, dim3(a.nb * a.h_split), dim3(kHBlock), 0, s, a);
    const int tiles = (int)hmerge_tiles(a.m);
    if (bfs) hipLaunchKernelGGL((k_hmerge_out<SR, true>), dim3(tiles), dim3(kHBlock), 0, s, a);
    else hipLaunchKernelGGL((k_hmerge_out<SR, false>), dim3(tiles), dim3(kHBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hbm_merge(const MergeArgs& a, int semiring, bool bfs, hipStream_t s) {
    if (a.nb < 1 || a.h_split < 1) return hipErrorInvalidValue;
    switch (semiring) {
        case SR_PLUS_TIMES: return hmerge<SR_PLUS_TIMES>(a, bfs, s);
        case SR_MIN_SELECT2ND: return hmerge<SR_MIN_SELECT2ND>(a, bfs, s);
        default: return hmerge<SR_OR_AND>(a, bfs, s);
    }
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t g = (count + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)g), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

}  // namespace spv
