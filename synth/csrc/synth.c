/*
 * Seeded synthetic inputs for the SpMSpV library and its oracle.
 *
 * This file builds input data only: R-MAT and grid graphs in CSC form,
 * fp32 values on the 2^-24 grid, sparse vectors with distinct indices,
 * BFS roots and log-uniform frontier sizes.  It performs none of the
 * sparse matrix-sparse vector arithmetic; both the GPU path and the CPU
 * oracle consume what it produces.
 *
 * Random numbers come from the SplitMix64 output function (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
 * used as a counter-based generator: draw i of stream s under seed k is
 * mix(key(k, s) + (i + 1) * gamma), with gamma = 0x9e3779b97f4a7c15.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return mix64(seed * GAMMA + mix64(stream + 0x632be59bd9b4e019ULL));
}

static inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GAMMA); }

/* Uniform integer in [0, bound) by the multiply-shift reduction (Lemire 2019). */
static inline uint64_t below(uint64_t r, uint64_t bound) {
    return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

uint64_t synth_draw(uint64_t seed, uint64_t stream, uint64_t i) {
    return draw(stream_key(seed, stream), i);
}

/* ------------------------------------------------------------------ */
/* R-MAT tuples.  Each tuple descends `scale` levels; at every level one
 * 32-bit uniform picks a quadrant with probabilities a, b, c, d (row bit,
 * column bit) = (0,0), (0,1), (1,0), (1,1).  Tuple e uses draws
 * [e * ceil(scale/2), ...) of stream 1.                                  */
void synth_rmat_tuples(int scale, int64_t ntuples, double a, double b, double c, uint64_t seed,
                       int32_t* rows, int32_t* cols) {
    const uint64_t key = stream_key(seed, 1);
    const uint64_t ta = (uint64_t)(a * 4294967296.0);
    const uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
    const uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
    const int64_t per = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ntuples; ++e) {
        uint32_t i = 0, j = 0;
        for (int l = 0; l < scale; ++l) {
            uint64_t r64 = draw(key, (uint64_t)e * per + (l >> 1));
            uint64_t r = (l & 1) ? (r64 >> 32) : (r64 & 0xffffffffULL);
            uint32_t ib = 0, jb = 0;
            if (r < ta) { ib = 0; jb = 0; }
            else if (r < tb) { ib = 0; jb = 1; }
            else if (r < tc) { ib = 1; jb = 0; }
            else { ib = 1; jb = 1; }
            i = (i << 1) | ib;
            j = (j << 1) | jb;
        }
        rows[e] = (int32_t)i;
        cols[e] = (int32_t)j;
    }
}

/* Seeded uniform permutation of [0, n) (Fisher-Yates, stream 2). */
void synth_permutation(int64_t n, uint64_t seed, int32_t* perm) {
    const uint64_t key = stream_key(seed, 2);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t k = (int64_t)below(draw(key, (uint64_t)i), (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[k]; perm[k] = t;
    }
}

static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

static void sort_i32(int32_t* v, int64_t len) {
    if (len < 32) {
        for (int64_t i = 1; i < len; ++i) {
            int32_t t = v[i];
            int64_t k = i - 1;
            while (k >= 0 && v[k] > t) { v[k + 1] = v[k]; --k; }
            v[k + 1] = t;
        }
    } else {
        qsort(v, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/*
 * COO -> CSC.  Tuples (rows[e], cols[e]) for e < nt are relabelled by perm
 * (if non-NULL, applied to both coordinates), mirrored when `symmetrize`,
 * stripped of self loops when `drop_self`, bucketed by column, sorted by row
 * within each column and de-duplicated.  colptr has n+1 entries; rowids must
 * hold (symmetrize ? 2 : 1) * nt entries.  Returns nnz.
 */
int64_t synth_coo_to_csc(int64_t m, int64_t n, int64_t nt, const int32_t* rows, const int32_t* cols,
                         const int32_t* perm, int symmetrize, int drop_self, int32_t* colptr,
                         int32_t* rowids) {
    const int64_t cap = symmetrize ? 2 * nt : nt;
    int64_t* cnt = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    /* counting pass */
    for (int64_t e = 0; e < nt; ++e) {
        int32_t i = rows[e], j = cols[e];
        if (perm) { i = perm[i]; j = perm[j]; }
        if (drop_self && i == j) continue;
        cnt[j + 1]++;
        if (symmetrize) cnt[i + 1]++;
    }
    for (int64_t j = 0; j < n; ++j) cnt[j + 1] += cnt[j];
    int64_t* pos = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    memcpy(pos, cnt, (size_t)(n + 1) * sizeof(int64_t));
    (void)cap;
    for (int64_t e = 0; e < nt; ++e) {
        int32_t i = rows[e], j = cols[e];
        if (perm) { i = perm[i]; j = perm[j]; }
        if (drop_self && i == j) continue;
        rowids[pos[j]++] = i;
        if (symmetrize) rowids[pos[i]++] = j;
    }
    free(pos);
    /* sort + dedup each column in place; new column lengths into len[] */
    int64_t* len = (int64_t*)malloc((size_t)n * sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t j = 0; j < n; ++j) {
        int32_t* v = rowids + cnt[j];
        int64_t l = cnt[j + 1] - cnt[j];
        sort_i32(v, l);
        int64_t u = 0;
        for (int64_t k = 0; k < l; ++k)
            if (u == 0 || v[k] != v[u - 1]) v[u++] = v[k];
        len[j] = u;
    }
    /* compact */
    int64_t out = 0;
    colptr[0] = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t src = cnt[j];
        if (out != src) memmove(rowids + out, rowids + src, (size_t)len[j] * sizeof(int32_t));
        out += len[j];
        colptr[j + 1] = (int32_t)out;
    }
    (void)m;
    free(len);
    free(cnt);
    return out;
}

/* fp32 values (u + 1) * 2^-24 with u uniform in [0, 2^24): exact in fp32, in (0, 1]. */
void synth_values(int64_t count, uint64_t seed, uint64_t stream, float* out) {
    const uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < count; ++q) {
        uint64_t u = draw(key, (uint64_t)q) >> 40;
        out[q] = (float)((double)(u + 1) * (1.0 / 16777216.0));
    }
}

/* f distinct indices of [0, n), uniformly chosen (Floyd's sampling), then
 * put in a uniformly random order (Fisher-Yates).  Stream 3 + 16 * tag.  */
int synth_distinct(int64_t n, int64_t f, uint64_t seed, uint64_t tag, int32_t* out) {
    if (f < 0 || f > n) return -1;
    const uint64_t key = stream_key(seed, 3 + 16 * tag);
    uint64_t* seen = (uint64_t*)calloc((size_t)(n / 64 + 1), sizeof(uint64_t));
    int64_t k = 0;
    uint64_t ctr = 0;
    for (int64_t j = n - f; j < n; ++j) {
        int64_t t = (int64_t)below(draw(key, ctr++), (uint64_t)(j + 1));
        int64_t pick = (seen[t >> 6] >> (t & 63)) & 1 ? j : t;
        seen[pick >> 6] |= 1ULL << (pick & 63);
        out[k++] = (int32_t)pick;
    }
    for (int64_t i = f - 1; i > 0; --i) {
        int64_t r = (int64_t)below(draw(key, ctr++), (uint64_t)(i + 1));
        int32_t t = out[i]; out[i] = out[r]; out[r] = t;
    }
    free(seen);
    return 0;
}

/* 2-D 5-point / 3-D 7-point grid in CSC, diagonal optional.  Vertex
 * v = x + nx*y + nx*ny*z; rows in each column ascending.  Returns nnz.   */
int64_t synth_grid_csc(int64_t nx, int64_t ny, int64_t nz, int diag, int32_t* colptr, int32_t* rowids) {
    const int64_t n = nx * ny * nz;
    const int64_t sy = nx, sz = nx * ny;
    int64_t q = 0;
    colptr[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t x = v % nx, y = (v / nx) % ny, z = v / sz;
        if (z > 0) rowids[q++] = (int32_t)(v - sz);
        if (y > 0) rowids[q++] = (int32_t)(v - sy);
        if (x > 0) rowids[q++] = (int32_t)(v - 1);
        if (diag) rowids[q++] = (int32_t)v;
        if (x + 1 < nx) rowids[q++] = (int32_t)(v + 1);
        if (y + 1 < ny) rowids[q++] = (int32_t)(v + sy);
        if (z + 1 < nz) rowids[q++] = (int32_t)(v + sz);
        colptr[v + 1] = (int32_t)q;
    }
    return q;
}

/* count roots uniformly drawn among vertices with a non-empty column. */
int synth_roots(int64_t n, const int32_t* colptr, int count, uint64_t seed, int32_t* out) {
    const uint64_t key = stream_key(seed, 5);
    uint64_t ctr = 0;
    for (int r = 0; r < count; ++r) {
        for (int tries = 0;; ++tries) {
            if (tries > 1000000) return -1;
            int64_t v = (int64_t)below(draw(key, ctr++), (uint64_t)n);
            if (colptr[v + 1] > colptr[v]) { out[r] = (int32_t)v; break; }
        }
    }
    return 0;
}

/* count sizes round(exp(U * ln(hi))) with U uniform in [0,1): log-uniform in [1, hi]. */
void synth_log_uniform(int count, double hi, uint64_t seed, int64_t* out) {
    const uint64_t key = stream_key(seed, 6);
    for (int r = 0; r < count; ++r) {
        double u = (double)(draw(key, (uint64_t)r) >> 11) * (1.0 / 9007199254740992.0);
        double v = floor(exp(u * log(hi)) + 0.5);
        if (v < 1) v = 1;
        if (v > hi) v = hi;
        out[r] = (int64_t)v;
    }
}
