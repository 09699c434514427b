// Persistent BFS levels for small frontiers on low-degree graphs.
//
// A high-diameter graph (a 3-D grid: hundreds of levels, frontiers of a few
// thousand vertices) spends almost all of a level's time in launch and
// phase latency of the three bucketing kernels.  While the frontier stays
// at or below kTinyFrontier vertices, this kernel runs level after level in
// one cooperative launch, with two grid-wide barriers per level (the two
// append counters alternate between levels, so the one a level fills is
// never the one being reset):
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

__device__ __forceinline__ void stc(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stcu(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Counting grid barrier (all workgroups are resident: cooperative launch).
// bar[0] counts arrivals, bar[1] is the generation.  Every value that
// crosses workgroups in this kernel is written and read with device-scope
// atomics, which are coherent without cache maintenance, so the barrier
// only has to wait for this workgroup's own memory operations to complete:
// no L2 write-back or invalidation (which on a multi-die GPU would touch the
// whole L2 of a die at every barrier).  A wait past kSpinLimit polls sets
// ERR_SPIN and proceeds, so no wave can hang.
__device__ void grid_sync(uint32_t* bar, uint32_t& gen, uint32_t* err) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t g = gen;
        const uint32_t arrived = atomicAdd(&bar[0], 1u) + 1u;
        if (arrived == gridDim.x) {
            stcu(&bar[0], 0u);
            stcu(&bar[1], g + 1u);
        } else {
            int spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (++spins > kSpinLimit) {
                    atomicOr(err, ERR_SPIN);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        gen = g + 1u;
    }
    __syncthreads();
}

template <bool MIN>
__global__ __launch_bounds__(kPBlock) void k_bfs_persistent(PersistArgs a) {
    constexpr int K = 8;   // neighbours per lane in flight
    const int lane = threadIdx.x & 63;
    uint32_t gen = 0;
    if (threadIdx.x == 0) gen = __hip_atomic_load(&a.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    int slot = 0;   // append counter of the level being discovered: gen_count, then gen_count2, ...
    while (f > 0 && f <= kTinyFrontier) {
        ++lvl;   // the level being discovered (the frontier's level + 1)
        int32_t* const cnt = slot ? &a.ctrl->gen_count2 : &a.ctrl->gen_count;
        int32_t* const other = slot ? &a.ctrl->gen_count : &a.ctrl->gen_count2;
        // expand: lanes step through their vertices' neighbour lists together
        // (degrees are small here), K neighbours per lane in flight, and each
        // step's discoveries are appended with one counter update per wave
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
            for (int k0 = 0; k0 < mx; k0 += K) {
                int32_t v[K];
                uint32_t vis[K];
                bool claim[K];
#pragma unroll
                for (int j = 0; j < K; ++j) v[j] = k0 + j < len ? a.rowids[q + k0 + j] : -1;
#pragma unroll
                for (int j = 0; j < K; ++j)
                    vis[j] = v[j] >= 0 ? __hip_atomic_load(&a.visited[v[j] >> 5], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT)
                                       : 0xffffffffu;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    claim[j] = false;
                    const uint32_t bit = 1u << (v[j] & 31);
                    if (v[j] >= 0 && !(vis[j] & bit)) {
                        if (MIN) atomicMin(&a.pmin[v[j]], u);
                        claim[j] = !(atomicOr(&a.disc[v[j] >> 5], bit) & bit);
                    }
                }
                uint64_t vote[K];
                int total = 0;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    vote[j] = __ballot(claim[j]);
                    total += (int)__popcll(vote[j]);
                }
                if (total) {
                    int32_t first = 0;
                    if (lane == 0) first = atomicAdd(cnt, total);
                    first = __shfl(first, 0, 64);
                    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        if (claim[j]) stc(&nxt[first + (int)__popcll(vote[j] & below)], v[j]);
                        first += (int)__popcll(vote[j]);
                    }
                }
            }
        }
        grid_sync(a.bar, gen, &a.ctrl->err);
        const int32_t fn = ldc(cnt);
        // commit
        for (int64_t p = (int64_t)blockIdx.x * kPBlock + threadIdx.x; p < fn; p += stride) {
            const int32_t v = ldc(&nxt[p]);
            level[v] = lvl;
            if (MIN) {
                if (parent) parent[v] = ldc(&a.pmin[v]);
                stc(&a.pmin[v], 0x7fffffff);
            }
            atomicOr(&a.visited[v >> 5], 1u << (v & 31));
            stcu(&a.disc[v >> 5], 0u);   // every bit of this word was discovered at this level
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            stc(other, 0);   // the next level appends there; nobody reads it now
            stc(&a.ctrl->f, fn);
            stc(&a.ctrl->level, lvl);
        }
        grid_sync(a.bar, gen, &a.ctrl->err);
        f = fn;
        int32_t* t = cur;
        cur = nxt;
        nxt = t;
        swapped = !swapped;
        slot ^= 1;
    }
    // Hand the frontier back in front0, and leave gen_count at zero.
    if (swapped) {
        for (int64_t p = (int64_t)blockIdx.x * kPBlock + threadIdx.x; p < f; p += stride) stc(&a.front0[p], ldc(&cur[p]));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        stc(&a.ctrl->gen_count, 0);
        stc(&a.ctrl->gen_count2, 0);
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
    if (per_cu > 1) per_cu = 1;   // fewer arrivals per barrier; small frontiers need few threads
    return per_cu * num_cu;
}

hipError_t launch_bfs_persistent(const PersistArgs& a, bool min_semiring, int grid, hipStream_t s) {
    void* args[] = {const_cast<PersistArgs*>(&a)};
    const void* fn = min_semiring ? reinterpret_cast<const void*>(k_bfs_persistent<true>)
                                  : reinterpret_cast<const void*>(k_bfs_persistent<false>);
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kPBlock), args, 0, s);
}

}  // namespace spv
