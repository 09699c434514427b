// Persistent BFS levels for small frontiers on low-degree graphs.
//
// A high-diameter graph (a 3-D grid: hundreds of levels, frontiers of a few
// thousand vertices) spends almost all of a level's time in launch and
// phase latency of the three bucketing kernels.  While the frontier stays
// at or below kTinyFrontier vertices, this kernel runs level after level in
// one cooperative launch, with two grid-wide barriers per level:
//   expand:  every (u, v) with u in the frontier and v not yet visited
//            records min(u) for v (min-select2nd: the parent rule of the
//            level-synchronous SpMSpV, select2nd with x value = vertex id)
//            and the first lane to set v's bit in the discovered bitmap
//            appends v to the next frontier;
//   commit:  every discovered v gets its level, parent and visited bit, and
//            the scratch state is reset.
// Results are those of the bucketing path (same levels, same minimum
// parents); only the order of the frontier list differs.  The kernel stops
// when the frontier empties or outgrows kTinyFrontier, leaving the frontier
// in front[0] and its length in the control block for the bucketing path.

#include "internal.h"

namespace spv {

namespace {

constexpr int kPBlock = 256;
constexpr int kSpinLimit = 1 << 22;

__device__ __forceinline__ int32_t ldc(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sense-counting grid barrier (all workgroups are resident: cooperative
// launch).  bar[0] counts arrivals, bar[1] is the generation.  A wait past
// kSpinLimit polls sets ERR_SPIN and proceeds, so no wave can hang.
__device__ void grid_sync(uint32_t* bar, uint32_t& gen, uint32_t* err) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t g = gen;
        const uint32_t arrived = atomicAdd(&bar[0], 1u) + 1u;
        if (arrived == gridDim.x) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            __hip_atomic_store(&bar[1], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            int spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (++spins > kSpinLimit) {
                    atomicOr(err, ERR_SPIN);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        gen = g + 1u;
        __threadfence();
    }
    __syncthreads();
}

template <bool MIN>
__global__ __launch_bounds__(kPBlock) void k_bfs_persistent(PersistArgs a) {
    const int lane = threadIdx.x & 63;
    uint32_t gen = 0;
    if (threadIdx.x == 0) gen = __hip_atomic_load(&a.bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    int32_t* cur = a.front0;
    int32_t* nxt = a.front1;
    int32_t f = ldc(&a.ctrl->f);
    int32_t lvl = ldc(&a.ctrl->level);
    int32_t* const level = reinterpret_cast<int32_t*>(
        __hip_atomic_load(reinterpret_cast<const uint64_t*>(&a.ctrl->bfs_level), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT));
    int32_t* const parent = reinterpret_cast<int32_t*>(
        __hip_atomic_load(reinterpret_cast<const uint64_t*>(&a.ctrl->bfs_parent), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT));
    const int64_t stride = (int64_t)gridDim.x * kPBlock;
    bool swapped = false;
    while (f > 0 && f <= kTinyFrontier) {
        ++lvl;   // the level being discovered (the frontier's level + 1)
        // expand: lanes step through their vertices' neighbour lists together
        // (degrees are small here), so each step's discoveries are appended
        // with one counter update per wave
        for (int64_t base = (int64_t)blockIdx.x * kPBlock; base < f; base += stride) {
            const int64_t p = base + threadIdx.x;
            const int32_t u = p < f ? ldc(&cur[p]) : -1;
            int32_t q = 0, len = 0;
            if (u >= 0) {
                q = a.colptr[u];
                len = a.colptr[u + 1] - q;
            }
            int32_t mx = len;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d, 64));
            for (int k = 0; k < mx; ++k) {
                bool claim = false;
                int32_t v = 0;
                if (k < len) {
                    v = a.rowids[q + k];
                    const uint32_t bit = 1u << (v & 31);
                    const uint32_t vis = __hip_atomic_load(&a.visited[v >> 5], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                    if (!(vis & bit)) {
                        if (MIN) atomicMin(&a.pmin[v], u);
                        claim = !(atomicOr(&a.disc[v >> 5], bit) & bit);
                    }
                }
                const uint64_t vote = __ballot(claim);
                if (vote) {
                    int32_t first = 0;
                    if (lane == 0) first = atomicAdd(&a.ctrl->gen_count, (int32_t)__popcll(vote));
                    first = __shfl(first, 0, 64);
                    if (claim) nxt[first + (int)__popcll(vote & ((1ull << lane) - 1ull))] = v;
                }
            }
        }
        grid_sync(a.bar, gen, &a.ctrl->err);
        const int32_t fn = ldc(&a.ctrl->gen_count);
        // commit
        for (int64_t p = (int64_t)blockIdx.x * kPBlock + threadIdx.x; p < fn; p += stride) {
            const int32_t v = ldc(&nxt[p]);
            level[v] = lvl;
            if (MIN) {
                if (parent) parent[v] = ldc(&a.pmin[v]);
                a.pmin[v] = 0x7fffffff;
            }
            atomicOr(&a.visited[v >> 5], 1u << (v & 31));
            a.disc[v >> 5] = 0u;   // every bit of this word was discovered at this level
        }
        grid_sync(a.bar, gen, &a.ctrl->err);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            __hip_atomic_store(&a.ctrl->gen_count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.ctrl->f, fn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.ctrl->level, lvl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        grid_sync(a.bar, gen, &a.ctrl->err);
        f = fn;
        int32_t* t = cur;
        cur = nxt;
        nxt = t;
        swapped = !swapped;
    }
    // Hand the frontier back in front0.
    if (swapped) {
        for (int64_t p = (int64_t)blockIdx.x * kPBlock + threadIdx.x; p < f; p += stride) a.front0[p] = ldc(&cur[p]);
    }
}

}  // namespace

int persistent_grid(int num_cu) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bfs_persistent<true>, kPBlock, 0) != hipSuccess ||
        per_cu < 1)
        return 0;
    int per_cu2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, k_bfs_persistent<false>, kPBlock, 0) != hipSuccess ||
        per_cu2 < 1)
        return 0;
    if (per_cu2 < per_cu) per_cu = per_cu2;
    if (per_cu > 2) per_cu = 2;
    return per_cu * num_cu;
}

hipError_t launch_bfs_persistent(const PersistArgs& a, bool min_semiring, int grid, hipStream_t s) {
    void* args[] = {const_cast<PersistArgs*>(&a)};
    const void* fn = min_semiring ? reinterpret_cast<const void*>(k_bfs_persistent<true>)
                                  : reinterpret_cast<const void*>(k_bfs_persistent<false>);
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kPBlock), args, 0, s);
}

}  // namespace spv
