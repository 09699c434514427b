// Persistent BFS levels for small frontiers on low-degree graphs.
//
// A high-diameter graph (a 3-D grid: hundreds of levels, frontiers of a few
// thousand vertices) spends almost all of a level's time in launch and
// phase latency of the three bucketing kernels.  While the frontier stays
// at or below kTinyFrontier vertices, this kernel runs level after level in
// one cooperative launch, with ONE grid-wide barrier per level.
//
// min-select2nd (parents: select2nd with x value = vertex id, so a new
// vertex's parent is its smallest frontier in-neighbour, as in the
// level-synchronous SpMSpV).  The phase that expands F(L) also finishes
// F(L) itself:
//   expand:  every (u, v) with u in F(L) and v neither visited nor in F(L)
//            lowers pmin[v] to u, and the first lane to set v's bit in the
//            bitmap of F(L+1) appends v to the list of F(L+1);
//   commit:  every u in F(L) gets its level, parent and visited bit (the
//            expansion tests F(L)'s own bitmap, so it does not need them);
//   reset:   the bitmap of F(L-1) is cleared over F(L-1)'s list.
// Three frontier lists, three bitmaps and three append counters rotate, so
// within a phase nothing that is read is also reset.
//
// or-and (levels only): the lane whose atomic OR first sets v's visited
// bit owns v, writes its level and appends it; no bitmaps, no commit.
//
// Results are those of the bucketing path (same levels, same minimum
// parents); only the order of the frontier list differs.  The kernel stops
// when the frontier empties or outgrows kTinyFrontier, commits it, and
// leaves it in front[0] with its length and level in the control block for
// the bucketing path.

#include "internal.h"

namespace spv {

namespace {

constexpr int kPBlock = 256;
constexpr int kSpinLimit = 1 << 22;
// Barrier words, each on a cache line of its own (workgroups that wait poll
// the generation while others update the append counters): arrivals, the
// three append counters, completed barriers.
constexpr int kLine = 32;   // 128-byte L2 line in 32-bit words
constexpr int kArrive = 0, kCount = kLine, kGen = 4 * kLine;

__device__ __forceinline__ int32_t ldc(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ldu(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stcu(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Counting grid barrier (all workgroups are resident: cooperative launch).
// bar[kArrive] counts every arrival of the launch and is never reset inside
// it: barrier k is complete at arrival (k+1)*grid (mod 2^32, a window of
// grid arrivals matches it only once), and the last arrival publishes k+1
// in bar[kGen].  Every value that crosses workgroups in this kernel is
// written and read with device-scope atomics, which are coherent without
// cache maintenance, so the barrier only has to wait for this workgroup's
// own memory operations to complete: no L2 write-back or invalidation (which
// on a multi-die GPU would touch the whole L2 of a die at every barrier).
// That wait is explicit: a workgroup-scope fence does not wait for vector
// memory operations on gfx950 (the waves of a workgroup share one CU), so
// every wave waits for its own outstanding loads, stores and atomics
// (s_waitcnt vmcnt(0)) before the workgroup barrier, and only then does
// thread 0 publish the arrival.
// A wait past kSpinLimit polls sets ERR_SPIN and returns false; the caller
// then leaves the kernel, so every later barrier of the others times out
// too and no wave can hang.
__device__ bool grid_sync(uint32_t* bar, uint32_t& gen, uint32_t* err) {
    __shared__ int s_ok;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    wait_vmem();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const uint32_t target = (gen + 1u) * gridDim.x;
        if (atomicAdd(&bar[kArrive], 1u) + 1u == target) {
            stcu(&bar[kGen], gen + 1u);
        } else {
            int spins = 0;
            while (ldu(&bar[kGen]) == gen) {
                if (++spins > kSpinLimit) {
                    atomicOr(err, ERR_SPIN);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        s_ok = ok;
        ++gen;
    }
    __syncthreads();
    return s_ok != 0;
}

// Level, parent (pm = the smallest frontier in-neighbour) and visited bit of
// a vertex discovered under min-select2nd, and its pmin slot back to
// INT32_MAX.
__device__ __forceinline__ void commit_vertex(int32_t u, int32_t lvl, int32_t pm, int32_t* level, int32_t* parent,
                                              int32_t* pmin, uint32_t* visited) {
    level[u] = lvl;
    if (parent) parent[u] = pm;
    stc(&pmin[u], 0x7fffffff);
    atomicOr(&visited[u >> 5], 1u << (u & 31));
}

template <bool MIN>
__global__ __launch_bounds__(kPBlock) void k_bfs_persistent(PersistArgs a) {
    constexpr int K = 8;   // neighbours per lane in flight
    int32_t f = ldc(&a.ctrl->f);
    if (f <= 0 || f > kTinyFrontier) return;   // the same value in every workgroup
    int32_t lvl = ldc(&a.ctrl->level);         // level of the frontier in front[0]
    const int lane = threadIdx.x & 63;
    int32_t* const level = reinterpret_cast<int32_t*>(
        __hip_atomic_load(reinterpret_cast<const uint64_t*>(&a.ctrl->bfs_level), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT));
    int32_t* const parent = reinterpret_cast<int32_t*>(
        __hip_atomic_load(reinterpret_cast<const uint64_t*>(&a.ctrl->bfs_parent), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT));
    uint32_t* const err = &a.ctrl->err;
    const int64_t stride = (int64_t)gridDim.x * kPBlock;
    const int64_t p0 = (int64_t)blockIdx.x * kPBlock + threadIdx.x;   // first list slot of this thread
    uint32_t gen = 0;
    int cur = 0;           // slot of F(L): list front[cur], bitmap disc[cur], count bar[kCount + kLine * cur]
    int32_t f_prev = 0;    // length of F(L-1), in the previous slot
    bool fresh = false;    // F(L) was discovered by this launch and is not committed yet
    int32_t u0 = p0 < f ? ldc(&a.front[0][p0]) : -1;   // this thread's first frontier vertex
    for (;;) {
        const int nx = cur == 2 ? 0 : cur + 1;
        const int pv = cur == 0 ? 2 : cur - 1;
        const int32_t* const fr = a.front[cur];
        const int32_t* const fp = a.front[pv];
        int32_t* const out = a.front[nx];
        const uint32_t* const dcur = a.disc[cur];
        uint32_t* const dnext = a.disc[nx];
        uint32_t* const dprev = a.disc[pv];
        int32_t* const cnt = reinterpret_cast<int32_t*>(&a.bar[kCount + kLine * nx]);   // zero: reset a phase ago
        const int32_t span = MIN && f_prev > f ? f_prev : f;
        // Lanes step through their vertices' neighbour lists together
        // (degrees are small here), K neighbours per lane in flight, and each
        // step's discoveries are appended with one counter update per wave.
        for (int64_t p = p0; p - threadIdx.x < span; p += stride) {
            const int32_t u = p == p0 ? u0 : p < f ? ldc(&fr[p]) : -1;
            const int32_t w = MIN && p < f_prev ? ldc(&fp[p]) : -1;
            int32_t q = 0, len = 0, pm = 0;
            if (u >= 0) {
                q = a.colptr[u];
                len = a.colptr[u + 1] - q;
                if (MIN && fresh) pm = ldc(&a.pmin[u]);
            }
            int32_t mx = len;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d, 64));
            for (int k0 = 0; k0 < mx; k0 += K) {
                int32_t v[K];
                bool claim[K];
#pragma unroll
                for (int j = 0; j < K; ++j) v[j] = k0 + j < len ? a.rowids[q + k0 + j] : -1;
                if (MIN) {
                    // v is new if neither visited nor in F(L); every frontier
                    // in-neighbour of a new v takes part in the minimum, the
                    // first to set its bit in F(L+1)'s bitmap appends it.
                    uint32_t vis[K];
#pragma unroll
                    for (int j = 0; j < K; ++j)
                        vis[j] = v[j] >= 0 ? ldu(&a.visited[v[j] >> 5]) | ldu(&dcur[v[j] >> 5]) : 0xffffffffu;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        claim[j] = false;
                        const uint32_t bit = 1u << (v[j] & 31);
                        if (v[j] >= 0 && !(vis[j] & bit)) {
                            atomicMin(&a.pmin[v[j]], u);
                            claim[j] = !(atomicOr(&dnext[v[j] >> 5], bit) & bit);
                        }
                    }
                } else {
                    // Levels only: the first lane to set v's visited bit owns
                    // v and writes its level at once.
#pragma unroll
                    for (int j = 0; j < K; ++j)
                        claim[j] = v[j] >= 0 && !(atomicOr(&a.visited[v[j] >> 5], 1u << (v[j] & 31)) &
                                                  (1u << (v[j] & 31)));
#pragma unroll
                    for (int j = 0; j < K; ++j)
                        if (claim[j]) level[v[j]] = lvl + 1;
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
                        if (claim[j]) stc(&out[first + (int)__popcll(vote[j] & below)], v[j]);
                        first += (int)__popcll(vote[j]);
                    }
                }
            }
            // Writes last: the in-order memory counter would otherwise make
            // the expansion's loads wait for them.
            if (MIN) {
                if (fresh && u >= 0) commit_vertex(u, lvl, pm, level, parent, a.pmin, a.visited);
                if (w >= 0) stcu(&dprev[w >> 5], 0u);   // every bit set there belongs to F(L-1)
            }
        }
        // F(L-1)'s counter starts F(L+2) next phase; every workgroup read it
        // right after the previous barrier.
        if (blockIdx.x == 0 && threadIdx.x == 0) stc(reinterpret_cast<int32_t*>(&a.bar[kCount + kLine * pv]), 0);
        if (!grid_sync(a.bar, gen, err)) return;
        f_prev = f;
        f = ldc(cnt);
        // Loaded with the count, before it is known (the list holds n slots).
        u0 = p0 < a.n ? ldc(&out[p0]) : -1;
        cur = nx;
        ++lvl;
        fresh = true;
        if (f == 0 || f > kTinyFrontier) break;
        if (p0 >= f) u0 = -1;
    }
    // Commit the last frontier and clear the two bitmaps still set.
    if (MIN) {
        const int pv = cur == 0 ? 2 : cur - 1;
        const int32_t* const fr = a.front[cur];
        const int32_t* const fp = a.front[pv];
        const int32_t span = f > f_prev ? f : f_prev;
        for (int64_t p = p0; p - threadIdx.x < span; p += stride) {
            if (p < f) {
                const int32_t u = ldc(&fr[p]);
                commit_vertex(u, lvl, ldc(&a.pmin[u]), level, parent, a.pmin, a.visited);
                stcu(&a.disc[cur][u >> 5], 0u);
            }
            if (p < f_prev) {
                const int32_t w = ldc(&fp[p]);
                stcu(&a.disc[pv][w >> 5], 0u);
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        stc(&a.ctrl->f, f);
        stc(&a.ctrl->level, lvl);
    }
    // Hand the frontier back in front[0] once nobody reads the other lists.
    if (cur != 0 && f > 0) {
        if (!grid_sync(a.bar, gen, err)) return;
        const int32_t* const fr = a.front[cur];
        for (int64_t p = p0; p < f; p += stride) stc(&a.front[0][p], ldc(&fr[p]));
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
