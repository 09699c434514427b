// Direction (and selector class) of a BFS level, shared by the decision
// kernels (k_decide, k_select) and by the scan, which takes the decision
// itself when the previous level ran pull and its emit left the new
// frontier's column sums behind.  Not installed.
#pragma once

#include "internal.h"

namespace spv {

// Selector MLP parameter layout (flat): W1[64][6], b1[64], W2[64][64],
// b2[64], W3[10][64], b3[10].
constexpr int kMI = kMlpIn, kMH1 = kMlpH1, kMH2 = kMlpH2, kMO = kMlpOut;
constexpr int kOW1 = 0, kOB1 = kOW1 + kMH1 * kMI, kOW2 = kOB1 + kMH1, kOB2 = kOW2 + kMH2 * kMH1,
              kOW3 = kOB2 + kMH2, kOB3 = kOW3 + kMO * kMH2;
static_assert(kOB3 + kMO == kMlpParams, "parameter layout");

__device__ __forceinline__ int32_t dc_ld(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t dc_ld64(const int64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void dc_st(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void dc_st64(int64_t* p, int64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Beamer, Asanovic and Patterson's direction-optimizing rule for a frontier
// of f vertices whose columns hold W stored entries: push -> pull when W
// exceeds edges_left / 14, pull -> push when f < n / 24.  Called by one
// thread; updates edges_left and ctrl->dir and returns the direction.
__device__ inline int heuristic_step(Ctrl* ctrl, int32_t n, int32_t f, int32_t W) {
    const int32_t prev = dc_ld(&ctrl->dir);
    const int32_t policy = dc_ld(&ctrl->policy);
    int64_t left = dc_ld64(&ctrl->edges_left);
    int dir = 0;
    if (policy == 1) {
        if (prev == 0) dir = ((int64_t)W * 14 > left) ? 1 : 0;
        else dir = ((int64_t)f * 24 < (int64_t)n) ? 0 : 1;
    }
    left -= W;
    if (left < 0) left = 0;
    dc_st64(&ctrl->edges_left, left);
    dc_st(&ctrl->dir, dir);
    return dir;
}

// The selector's step for a frontier of f vertices, W stored entries in its
// columns, longest column mx and fnz non-empty columns.  Features (log2(1 +
// v), standardised): f, W, mx, n, mean column length nnz / n, vertices not
// yet reached.  Writes the features and the class to the control block,
// with set_dir also the direction (pull = the last class, when a pull form
// exists and f > 0); forced >= 0 replaces the network's class.  When pull is
// chosen, mx / W / fnz become the call's reported figures (the scatter does
// that on the push path).  Every thread of the calling workgroup (at least
// 64) calls it; returns the direction in every thread.
__device__ inline int select_step(Ctrl* ctrl, const float* sel, int32_t n, int64_t nnz, int has_pull, int set_dir,
                                  int forced, int32_t f, int32_t W, int32_t mx, int32_t fnz) {
    __shared__ float feat[kMI], h1[kMH1], h2[kMH2], z[kMO];
    __shared__ int s_dir;
    const int tid = threadIdx.x;
    if (tid == 0) {
        int64_t seen = dc_ld64(&ctrl->seen);
        seen += ctrl->bfs_mode ? f : 0;
        dc_st64(&ctrl->seen, seen);
        const double unvisited = ctrl->bfs_mode ? (double)(n - seen) : (double)n;
        const double raw[kMI] = {(double)f, (double)W, (double)mx, (double)n, (double)nnz / (double)n, unvisited};
        for (int c = 0; c < kMI; ++c)
            feat[c] = ((float)log2(1.0 + raw[c]) - sel[kMlpParams + c]) / sel[kMlpParams + kMI + c];
    }
    __syncthreads();
    if (tid < kMH1) {
        float t = sel[kOB1 + tid];
        for (int c = 0; c < kMI; ++c) t = fmaf(sel[kOW1 + tid * kMI + c], feat[c], t);
        h1[tid] = t > 0.f ? t : 0.f;
    }
    __syncthreads();
    if (tid < kMH2) {
        float t = sel[kOB2 + tid];
        for (int i = 0; i < kMH1; ++i) t = fmaf(sel[kOW2 + tid * kMH1 + i], h1[i], t);
        h2[tid] = t > 0.f ? t : 0.f;
    }
    __syncthreads();
    if (tid < kMO) {
        float t = sel[kOB3 + tid];
        for (int j = 0; j < kMH2; ++j) t = fmaf(sel[kOW3 + tid * kMH2 + j], h2[j], t);
        z[tid] = t;
    }
    __syncthreads();
    if (tid == 0) {
        int best = 0;
        for (int k = 1; k < kMO; ++k)
            if (z[k] > z[best]) best = k;
        if (forced >= 0 && forced < kMO) best = forced;
        for (int c = 0; c < kMI; ++c) ctrl->features[c] = feat[c];
        const bool pull = best == kMO - 1 && has_pull && f > 0;
        if (set_dir) dc_st(&ctrl->dir, pull ? 1 : 0);
        if (pull) {
            atomicExch(&ctrl->maxlen, 0);
            dc_st(&ctrl->maxlen_last, mx);
            dc_st(&ctrl->W_last, W);
            dc_st(&ctrl->fnz_last, fnz);
        }
        dc_st(&ctrl->cls, best);
        s_dir = pull ? 1 : 0;
    }
    __syncthreads();
    return s_dir;
}

// Called first by the decision kernels of a direction-switching BFS level:
// when the scan already decided (chain_word = 2 | direction), consume that
// decision (a push level ends the chain) and return true.
__device__ inline bool consume_chain(Ctrl* ctrl) {
    const uint32_t w = __hip_atomic_load(&ctrl->chain_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!(w & 2u)) return false;
    if (!(w & 1u)) __hip_atomic_store(&ctrl->chain_ready, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctrl->chain_word, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

}  // namespace spv
