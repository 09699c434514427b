// Device helpers shared by the bucketing kernels, the one-launch multiply
// and the masked multiply: agent-scope control-word access, the decoupled
// look-back, block-wide scans, reading x values, the semiring's Mult, and
// the merge's tile accumulation.  Not installed.
#pragma once

#include "internal.h"

namespace spv {

constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_INC = 2ull << 62;
constexpr uint64_t LB_VAL = (1ull << 62) - 1;
constexpr int kSpinMax = 1 << 20;

__device__ __forceinline__ uint64_t ld_acquire64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Control words written by an earlier kernel (plain stores or atomics) are
// read with agent-scope atomic loads, never through the scalar cache.
__device__ __forceinline__ int32_t ld_ctrl(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t* ld_ctrl_ptr(int32_t* const* p) {
    return reinterpret_cast<int32_t*>(__hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_ctrl(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_ctrl_u(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Decoupled look-back over per-tile state words (status in bits 63:62,
// value in 61:0).  Called by all 64 lanes of one wave.  Publishes `agg` for
// `tile`, returns the exclusive prefix and publishes the inclusive one.
// A wait that exceeds kSpinMax polls sets ERR_SPIN and returns a partial
// prefix rather than hanging.
__device__ inline uint64_t lookback(uint64_t* st, int tile, uint64_t agg, uint32_t* err) {
    const int lane = threadIdx.x & (kWave - 1);
    if (tile == 0) {
        if (lane == 0) st_release64(&st[0], LB_INC | (agg & LB_VAL));
        return 0;
    }
    if (lane == 0) st_release64(&st[tile], LB_AGG | (agg & LB_VAL));
    uint64_t excl = 0;
    int base = tile - 1;
    int spins = 0;
    for (;;) {
        const int idx = base - lane;
        const uint64_t w = idx >= 0 ? ld_acquire64(&st[idx]) : LB_INC;
        const uint64_t status = w >> 62;
        const uint64_t inc_mask = __ballot(status == 2);
        const uint64_t empty_mask = __ballot(status == 0);
        const uint64_t need = inc_mask ? (((inc_mask & (~inc_mask + 1)) << 1) - 1) : ~0ull;
        if (empty_mask & need) {
            if (++spins > kSpinMax) {
                if (lane == 0) atomicOr(err, ERR_SPIN);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const uint64_t v = ((need >> lane) & 1ull) ? (w & LB_VAL) : 0ull;
        excl += wave_sum_u64(v);
        if (inc_mask) break;
        base -= kWave;
    }
    if (lane == 0) st_release64(&st[tile], LB_INC | ((excl + agg) & LB_VAL));
    return excl;
}

template <int BLOCK>
__device__ __forceinline__ uint64_t block_exclusive_u64(uint64_t v, uint64_t* s_tmp, uint64_t& total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    uint64_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) s_tmp[wid] = x;
    __syncthreads();
    // every lane reads the wave totals (broadcast reads, independent of
    // each other) instead of one thread summing them in sequence
    uint64_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / kWave; ++w) {
        const uint64_t t = s_tmp[w];
        pre += w < wid ? t : 0;
        tot += t;
    }
    total = tot;
    __syncthreads();   // s_tmp is reused by the next scan
    return pre + x - v;
}

template <int BLOCK>
__device__ __forceinline__ int block_exclusive_i32(int v, int* s_tmp, int& total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    int x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) s_tmp[wid] = x;
    __syncthreads();
    // every lane reads the wave totals (broadcast reads, independent of
    // each other) instead of one thread summing them in sequence
    int pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / kWave; ++w) {
        const int t = s_tmp[w];
        pre += w < wid ? t : 0;
        tot += t;
    }
    total = tot;
    __syncthreads();   // s_tmp is reused by the next scan
    return pre + x - v;
}

template <int XMODE>
__device__ __forceinline__ uint32_t x_value(const void* x_val, int p, int32_t j) {
    if constexpr (XMODE == XV_BITS32) return reinterpret_cast<const uint32_t*>(x_val)[p];
    else if constexpr (XMODE == XV_INDEX) return (uint32_t)j;
    else if constexpr (XMODE == XV_U8) return reinterpret_cast<const uint8_t*>(x_val)[p] ? 1u : 0u;
    else return 1u;
}

template <int SR>
__device__ __forceinline__ uint32_t mult(const float* values, int32_t q, uint32_t xbits) {
    if constexpr (SR == SR_PLUS_TIMES) {
        const float av = values ? values[q] : 1.0f;
        return __float_as_uint(__fmul_rn(av, __uint_as_float(xbits)));
    } else if constexpr (SR == SR_MIN_SELECT2ND) {
        return xbits;
    } else {
        const uint32_t av = values ? (values[q] != 0.0f ? 1u : 0u) : 1u;
        return av & (xbits != 0u ? 1u : 0u);
    }
}

template <int SR>
__device__ __forceinline__ uint32_t identity() {
    if constexpr (SR == SR_PLUS_TIMES) return 0u;            // +0.0f
    else if constexpr (SR == SR_MIN_SELECT2ND) return 0x7fffffffu;
    else return 0u;
}

template <int SR>
__device__ __forceinline__ void accumulate(uint32_t* cell, uint32_t v) {
    if constexpr (SR == SR_PLUS_TIMES) atomicAdd(reinterpret_cast<float*>(cell), __uint_as_float(v));
    else if constexpr (SR == SR_MIN_SELECT2ND) atomicMin(reinterpret_cast<int*>(cell), (int)v);
    else atomicOr(cell, v);
}

template <int SR>
__device__ __forceinline__ void store_value(void* y_val, int64_t o, uint32_t v) {
    if constexpr (SR == SR_OR_AND) reinterpret_cast<uint8_t*>(y_val)[o] = (uint8_t)(v != 0u);
    else reinterpret_cast<uint32_t*>(y_val)[o] = v;
}



// Tile accumulation.  Measured on gfx950 (random addresses in a 128 KB
// tile, every lane of 256 workgroups of 1024 threads): an LDS add of a
// 64-bit float retires about 2 lanes per cycle per compute unit, and keeps
// that rate when a third of the lanes hit a few dozen hub rows; a 32-bit
// float add retires about a third of a lane per cycle, and a
// compare-and-swap loop on a 32-bit word about 1.9 on distinct rows but half
// a lane once hub rows make lanes retry.  So plus-times accumulates every
// row in fp64 and rounds it to fp32 once, when y is written: faster, and the
// rounding error no longer grows with the number of terms of a row (fp32
// sums of a few hundred thousand terms in arbitrary order drift past 1e-5).
// An fp64 cell starts at -0.0, which only a sum whose every term is -0.0
// reproduces: such a product also sets the row's bitmap bit, and every other
// touched row is the one whose cell is no longer -0.0 (a ballot pass after
// the accumulation sets its bit).  min and or use their native integer
// atomics and set the bitmap bit with every entry.
constexpr uint64_t kNegZero64 = 0x8000000000000000ull;

// mark: plus-times sets every entry's bitmap bit here (a bucket with few
// entries, where one atomic per entry is cheaper than the ballot pass over
// the whole tile); otherwise only -0.0 products set it and touched_bits64
// finds the rest.
template <int SR, int K>
__device__ __forceinline__ void add_rows(const uint32_t (&r)[K], const uint32_t (&v)[K], const bool (&ok)[K],
                                         uint32_t* spa, uint32_t* bm, bool mark = false) {
    if constexpr (SR == SR_PLUS_TIMES) {
        double* spa64 = reinterpret_cast<double*>(spa);
#pragma unroll
        for (int u = 0; u < K; ++u) {
            if (ok[u]) {
                atomicAdd(&spa64[r[u]], (double)__uint_as_float(v[u]));
                if (mark || v[u] == 0x80000000u) atomicOr(&bm[r[u] >> 5], 1u << (r[u] & 31u));
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < K; ++u) {
            if (ok[u]) {
                atomicOr(&bm[r[u] >> 5], 1u << (r[u] & 31u));
                accumulate<SR>(&spa[r[u]], v[u]);
            }
        }
    }
}

// Bitmap bits of the fp64 cells a plus-times entry reached (cell no longer
// -0.0), 64 consecutive cells per wave and step: conflict-free 8-byte LDS
// reads, one ballot, and lane 0 merges the two bitmap words (nothing else
// writes them after the accumulation).
template <int BLOCK>
__device__ __forceinline__ void touched_bits64(const uint32_t* spa, uint32_t* bm, int rows) {
    const uint64_t* c64 = reinterpret_cast<const uint64_t*>(spa);
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    for (int c0 = wid * kWave; c0 < rows; c0 += BLOCK) {
        const int c = c0 + lane;
        const bool t = c < rows && c64[c] != kNegZero64;
        const uint64_t b = __ballot(t);
        if (lane == 0) {
            const int w = c0 >> 5;
            bm[w] |= (uint32_t)b;
            if (c0 + 32 < rows) bm[w + 1] |= (uint32_t)(b >> 32);
        }
    }
}

}  // namespace spv
