/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct implementation of what the GPU library
 * computes.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header, table or helper with the
 * GPU library; the two meet only on inputs produced by the seeded generators.
 *
 * Contents
 *   oracle_spmspv        y <- A x over a semiring, dense accumulator
 *                        (fp64 for plus-times), structural output pattern.
 *   oracle_spmspv_f32seq the same product folded in fp32 in product order
 *                        (the deterministic mode's reference).
 *   oracle_bfs           FIFO-queue breadth-first search levels, parents by
 *                        the minimum-parent rule.
 *   oracle_spmspv_graphblas  masked multiply with accumulate / replace.
 *   oracle_cc            connected components (smallest reaching vertex).
 *   oracle_spmspv_left   left multiplication y' <- x' A, column-driven.
 *   oracle_spmspv_dcsc   y <- A x with A in DCSC (non-empty columns only).
 *   oracle_pagerank      data-driven (delta) PageRank in fp64.
 *   oracle_mlp_*         fp64 forward / backward of the schedule-selector MLP.
 *
 * Definitions followed (paper: Azad and Bulu\c{c}, "A work-efficient parallel
 * sparse matrix-sparse vector multiplication algorithm"):
 *   - y <- A x with A m-by-n in CSC and x, y sparse lists (Background,
 *     Notation; Sparse matrix and vector data structures).
 *   - The output holds exactly the rows reached from the selected columns,
 *     one entry per unique row; the number of unique indices over all
 *     buckets is nnz(y) (Time and space complexity), so the pattern is
 *     structural: a row is present even if its value equals the semiring
 *     zero.
 *   - Multiplication applies Mult to the x entry and the matrix entry, and
 *     repeated rows combine with Add (Algorithm 1).  For min-select2nd the
 *     operand order is the GraphBLAS one, select2nd(A(i,j), x(j)) = x(j).
 *   - Sorted output lists indices in strictly ascending order (SpMSpV-bucket
 *     section, sorted variant).
 *
 * Parity pins live in tests/test_oracle_pins.py.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

enum { OR_PLUS_TIMES = 0, OR_MIN_SELECT2ND = 1, OR_OR_AND = 2 };

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/*
 * Validate CSC + x.  Returns 0 if valid, else a negative code:
 *   -1 colptr[0] != 0 or not monotone, -2 row id out of range,
 *   -3 x index out of range, -4 duplicate x index.
 */
int oracle_validate(int64_t m, int64_t n, const int32_t* colptr, const int32_t* rowids, int64_t f,
                    const int32_t* x_idx) {
    if (colptr[0] != 0) return -1;
    for (int64_t j = 0; j < n; ++j)
        if (colptr[j + 1] < colptr[j]) return -1;
    for (int64_t q = 0; q < colptr[n]; ++q)
        if (rowids[q] < 0 || rowids[q] >= m) return -2;
    unsigned char* used = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    int rc = 0;
    for (int64_t p = 0; p < f; ++p) {
        int32_t j = x_idx[p];
        if (j < 0 || j >= n) { rc = -3; break; }
        if (used[j]) { rc = -4; break; }
        used[j] = 1;
    }
    free(used);
    return rc;
}

/*
 * y <- A x over `semiring`.
 *   values  : float[nnz] or NULL (pattern: every stored entry is 1 / true).
 *   x_val   : plus-times float[f]; min-select2nd int32[f]; or-and uint8[f].
 *   mask    : NULL or uint8[m]; rows with mask[i] != 0 are dropped from y
 *             (applied after the multiply).
 *   y_val   : plus-times double[m]; min-select2nd int32[m]; or-and uint8[m].
 *   y_idx   : int32[m].  Output order: first-touch order when !sorted,
 *             ascending when sorted.
 *   *W      : products formed = sum over x entries of their column lengths.
 * Every stored x entry selects its column, whatever its value.
 */
int oracle_spmspv(int semiring, int64_t m, int64_t n, const int32_t* colptr, const int32_t* rowids,
                  const float* values, int64_t f, const int32_t* x_idx, const void* x_val,
                  const uint8_t* mask, int sorted, int32_t* y_idx, void* y_val, int64_t* nnz_y,
                  int64_t* W) {
    (void)n;
    unsigned char* seen = (unsigned char*)calloc((size_t)(m > 0 ? m : 1), 1);
    double* acc_d = NULL;
    int32_t* acc_i = NULL;
    uint8_t* acc_b = NULL;
    if (semiring == OR_PLUS_TIMES) acc_d = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    else if (semiring == OR_MIN_SELECT2ND) acc_i = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    else if (semiring == OR_OR_AND) acc_b = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
    else { free(seen); return -5; }

    int64_t count = 0, work = 0;
    for (int64_t p = 0; p < f; ++p) {
        int32_t j = x_idx[p];
        for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {
            int32_t i = rowids[q];
            work++;
            if (semiring == OR_PLUS_TIMES) {
                double a = values ? (double)values[q] : 1.0;
                double t = a * (double)((const float*)x_val)[p];
                if (!seen[i]) { seen[i] = 1; acc_d[i] = t; y_idx[count++] = i; }
                else acc_d[i] = acc_d[i] + t;
            } else if (semiring == OR_MIN_SELECT2ND) {
                int32_t t = ((const int32_t*)x_val)[p];
                if (!seen[i]) { seen[i] = 1; acc_i[i] = t; y_idx[count++] = i; }
                else if (t < acc_i[i]) acc_i[i] = t;
            } else {
                uint8_t a = values ? (values[q] != 0.0f) : 1;
                uint8_t t = (uint8_t)(a && ((const uint8_t*)x_val)[p] != 0);
                if (!seen[i]) { seen[i] = 1; acc_b[i] = t; y_idx[count++] = i; }
                else acc_b[i] = (uint8_t)(acc_b[i] || t);
            }
        }
    }
    if (mask) {
        int64_t k = 0;
        for (int64_t r = 0; r < count; ++r)
            if (!mask[y_idx[r]]) y_idx[k++] = y_idx[r];
        count = k;
    }
    if (sorted) qsort(y_idx, (size_t)count, sizeof(int32_t), cmp_i32);
    for (int64_t r = 0; r < count; ++r) {
        int32_t i = y_idx[r];
        if (semiring == OR_PLUS_TIMES) ((double*)y_val)[r] = acc_d[i];
        else if (semiring == OR_MIN_SELECT2ND) ((int32_t*)y_val)[r] = acc_i[i];
        else ((uint8_t*)y_val)[r] = acc_b[i];
    }
    *nnz_y = count;
    *W = work;
    free(seen); free(acc_d); free(acc_i); free(acc_b);
    return 0;
}

/*
 * Masked multiply with accumulation, w<mask, replace> = w (accum) (A x): the
 * generalisation of the BFS visited mask that the paper's conclusions name
 * as future work, with the mask, accumulate and replace rules of the
 * GraphBLAS standard.
 *   t = A x, structural pattern (oracle_spmspv, no mask).
 *   Mask: has_mask = 0 means every row is in the mask.  Otherwise row i is
 *     in it when it is listed in mask_idx[0..mask_count) and, for a value
 *     mask (mask_val != NULL), its listed value is nonzero; `complement`
 *     inverts membership (with has_mask = 0: no row is in the mask).
 *   w: w_idx[0..w_count) distinct rows, any order, values w_val (plus-times
 *     double, min-select2nd int32, or-and uint8).
 *   accum: 0 none, 1 the semiring's Add, 2 first (w wins), 3 second (t wins).
 *   z(i) = accum(w(i), t(i)) where both are present and accum != 0;
 *          t(i) where t(i) is present (accum == 0 or w(i) absent);
 *          w(i) where only w(i) is present and accum != 0; else absent.
 *   result(i) = z(i) for rows in the mask; for the other rows w(i) when
 *     replace == 0, absent when replace != 0.
 * Output ascending in y_idx / y_val (value type as w's).  Returns 0, or
 * -1 for an index out of range.
 */
int oracle_spmspv_graphblas(int semiring, int64_t m, int64_t n, const int32_t* colptr, const int32_t* rowids,
                            const float* values, int64_t f, const int32_t* x_idx, const void* x_val, int has_mask,
                            const int32_t* mask_idx, const uint8_t* mask_val, int64_t mask_count, int complement,
                            int accum, const int32_t* w_idx, const void* w_val, int64_t w_count, int replace,
                            int32_t* y_idx, void* y_val, int64_t* nnz_y) {
    const size_t M = (size_t)(m > 0 ? m : 1);
    int32_t* t_idx = (int32_t*)malloc(M * sizeof(int32_t));
    void* t_val = malloc(M * 8);
    unsigned char* t_has = (unsigned char*)calloc(M, 1);
    unsigned char* w_has = (unsigned char*)calloc(M, 1);
    unsigned char* in_mask = (unsigned char*)calloc(M, 1);
    double* td = (double*)calloc(M, sizeof(double));
    double* wd = (double*)calloc(M, sizeof(double));
    int32_t* ti = (int32_t*)calloc(M, sizeof(int32_t));
    int32_t* wi = (int32_t*)calloc(M, sizeof(int32_t));
    int rc = 0;
    int64_t nt = 0, W = 0, count = 0;
    if (oracle_spmspv(semiring, m, n, colptr, rowids, values, f, x_idx, x_val, NULL, 1, t_idx, t_val, &nt, &W)) {
        rc = -1;
        goto done;
    }
    for (int64_t r = 0; r < nt; ++r) {
        const int32_t i = t_idx[r];
        t_has[i] = 1;
        if (semiring == OR_PLUS_TIMES) td[i] = ((const double*)t_val)[r];
        else if (semiring == OR_MIN_SELECT2ND) ti[i] = ((const int32_t*)t_val)[r];
        else ti[i] = ((const uint8_t*)t_val)[r];
    }
    for (int64_t r = 0; r < w_count; ++r) {
        const int32_t i = w_idx[r];
        if (i < 0 || i >= m) { rc = -1; goto done; }
        w_has[i] = 1;
        if (semiring == OR_PLUS_TIMES) wd[i] = ((const double*)w_val)[r];
        else if (semiring == OR_MIN_SELECT2ND) wi[i] = ((const int32_t*)w_val)[r];
        else wi[i] = ((const uint8_t*)w_val)[r];
    }
    if (has_mask) {
        for (int64_t r = 0; r < mask_count; ++r) {
            const int32_t i = mask_idx[r];
            if (i < 0 || i >= m) { rc = -1; goto done; }
            if (!mask_val || mask_val[r] != 0) in_mask[i] = 1;
        }
    } else {
        for (int64_t i = 0; i < m; ++i) in_mask[i] = 1;
    }
    if (complement)
        for (int64_t i = 0; i < m; ++i) in_mask[i] = (unsigned char)!in_mask[i];
    for (int64_t i = 0; i < m; ++i) {
        int zp = 0;          /* z(i) present */
        double zd = 0.0;     /* z(i), plus-times */
        int32_t zi = 0;      /* z(i), min-select2nd and or-and */
        if (t_has[i] && w_has[i] && accum != 0) {
            zp = 1;
            if (accum == 2) { zd = wd[i]; zi = wi[i]; }
            else if (accum == 3) { zd = td[i]; zi = ti[i]; }
            else if (semiring == OR_PLUS_TIMES) zd = wd[i] + td[i];
            else if (semiring == OR_MIN_SELECT2ND) zi = wi[i] < ti[i] ? wi[i] : ti[i];
            else zi = (wi[i] || ti[i]) ? 1 : 0;
        } else if (t_has[i]) {
            zp = 1; zd = td[i]; zi = ti[i];
        } else if (w_has[i] && accum != 0) {
            zp = 1; zd = wd[i]; zi = wi[i];
        }
        int out = 0;
        double od = 0.0;
        int32_t oi = 0;
        if (in_mask[i]) {
            if (zp) { out = 1; od = zd; oi = zi; }
        } else if (!replace && w_has[i]) {
            out = 1; od = wd[i]; oi = wi[i];
        }
        if (out) {
            y_idx[count] = (int32_t)i;
            if (semiring == OR_PLUS_TIMES) ((double*)y_val)[count] = od;
            else if (semiring == OR_MIN_SELECT2ND) ((int32_t*)y_val)[count] = oi;
            else ((uint8_t*)y_val)[count] = (uint8_t)(oi != 0);
            ++count;
        }
    }
    *nnz_y = count;
done:
    free(t_idx); free(t_val); free(t_has); free(w_has); free(in_mask); free(td); free(wd); free(ti); free(wi);
    return rc;
}

/*
 * Connected components as the paper's introduction lists them among the
 * data-driven uses of SpMSpV: label(v) = the smallest vertex u from which v
 * is reachable along edges j -> i (every stored A(i,j)), u = v included.
 * For a symmetric A that is the smallest vertex of v's component.  Plain
 * definition: vertices in increasing order; an unlabelled one labels every
 * unlabelled vertex it reaches (FIFO queue), so each vertex is labelled by
 * the first, i.e. smallest, vertex that reaches it (a vertex reached only
 * through an already labelled one is reached by that one's smaller label
 * too).  Returns the number of components (distinct labels).
 */
int64_t oracle_cc(int64_t n, const int32_t* colptr, const int32_t* rowids, int32_t* label) {
    int32_t* queue = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t v = 0; v < n; ++v) label[v] = -1;
    int64_t comps = 0;
    for (int64_t u = 0; u < n; ++u) {
        if (label[u] >= 0) continue;
        ++comps;
        int64_t head = 0, tail = 0;
        label[u] = (int32_t)u;
        queue[tail++] = (int32_t)u;
        while (head < tail) {
            const int32_t j = queue[head++];
            for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {
                const int32_t i = rowids[q];
                if (label[i] < 0) {
                    label[i] = (int32_t)u;
                    queue[tail++] = i;
                }
            }
        }
    }
    free(queue);
    return comps;
}

/*
 * Left multiplication y' <- x' A (Background, Notation: the row-vector case,
 * which the paper leaves to symmetry with the column-vector one).  x' is a
 * sparse row vector over A's m rows and y' one over its n columns:
 *   y'(j) = Add over the stored A(i,j) whose row i is in x' of
 *           Mult(A(i,j), x'(i)),
 * in the operand order of oracle_spmspv (select2nd yields the x entry), so
 * y' equals A^T x' entry for entry.  Column-driven, unlike oracle_spmspv:
 * x' is spread into a dense array and every column of A is walked; column j
 * is in y' exactly when one of its stored rows is in x' (structural
 * pattern).  Output ascending in y_idx [n] / y_val (plus-times double,
 * min-select2nd int32, or-and uint8).  Returns 0, -3 for an x index out of
 * range, -4 for a duplicate x index.
 */
int oracle_spmspv_left(int semiring, int64_t m, int64_t n, const int32_t* colptr, const int32_t* rowids,
                       const float* values, int64_t f, const int32_t* x_idx, const void* x_val, int32_t* y_idx,
                       void* y_val, int64_t* nnz_y) {
    unsigned char* has = (unsigned char*)calloc((size_t)(m > 0 ? m : 1), 1);
    double* xd = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    int32_t* xi = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int rc = 0;
    for (int64_t p = 0; p < f && rc == 0; ++p) {
        const int32_t i = x_idx[p];
        if (i < 0 || i >= m) rc = -3;
        else if (has[i]) rc = -4;
        else {
            has[i] = 1;
            if (semiring == OR_PLUS_TIMES) xd[i] = (double)((const float*)x_val)[p];
            else if (semiring == OR_MIN_SELECT2ND) xi[i] = ((const int32_t*)x_val)[p];
            else xi[i] = ((const uint8_t*)x_val)[p] != 0;
        }
    }
    int64_t count = 0;
    for (int64_t j = 0; j < n && rc == 0; ++j) {
        int hit = 0;
        double sd = 0.0;
        int32_t si = 0;
        for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {
            const int32_t i = rowids[q];
            if (!has[i]) continue;
            if (semiring == OR_PLUS_TIMES) {
                const double t = (values ? (double)values[q] : 1.0) * xd[i];
                sd = hit ? sd + t : t;
            } else if (semiring == OR_MIN_SELECT2ND) {
                si = (!hit || xi[i] < si) ? xi[i] : si;
            } else {
                const int32_t t = (values ? (values[q] != 0.0f) : 1) && xi[i];
                si = hit ? (si || t) : t;
            }
            hit = 1;
        }
        if (!hit) continue;
        y_idx[count] = (int32_t)j;
        if (semiring == OR_PLUS_TIMES) ((double*)y_val)[count] = sd;
        else if (semiring == OR_MIN_SELECT2ND) ((int32_t*)y_val)[count] = si;
        else ((uint8_t*)y_val)[count] = (uint8_t)si;
        ++count;
    }
    *nnz_y = count;
    free(has); free(xd); free(xi);
    return rc;
}

/*
 * y <- A x with A in DCSC (Background, Sparse matrix and vector data
 * structures): only the nzc non-empty columns are stored, their ids
 * ascending in jc[0..nzc) and their entries at [cp[k], cp[k+1]) of rowids /
 * values.  Each x entry's column is looked up in jc by binary search; a
 * column absent from jc is empty and selects nothing.  The product is then
 * formed as in oracle_spmspv (dense accumulator, fp64 for plus-times,
 * structural pattern), output ascending.  *W = products formed.  Returns 0,
 * or -3 for an x index outside [0, n).
 */
int oracle_spmspv_dcsc(int semiring, int64_t m, int64_t n, int64_t nzc, const int32_t* jc, const int32_t* cp,
                       const int32_t* rowids, const float* values, int64_t f, const int32_t* x_idx,
                       const void* x_val, int32_t* y_idx, void* y_val, int64_t* nnz_y, int64_t* W) {
    unsigned char* seen = (unsigned char*)calloc((size_t)(m > 0 ? m : 1), 1);
    double* acc_d = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    int32_t* acc_i = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int64_t work = 0;
    int rc = 0;
    for (int64_t p = 0; p < f; ++p) {
        const int32_t j = x_idx[p];
        if (j < 0 || j >= n) { rc = -3; break; }
        int64_t lo = 0, hi = nzc;   /* first k with jc[k] >= j */
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (jc[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        if (lo == nzc || jc[lo] != j) continue;   /* empty column */
        for (int64_t q = cp[lo]; q < cp[lo + 1]; ++q) {
            const int32_t i = rowids[q];
            ++work;
            if (semiring == OR_PLUS_TIMES) {
                const double t = (values ? (double)values[q] : 1.0) * (double)((const float*)x_val)[p];
                acc_d[i] = seen[i] ? acc_d[i] + t : t;
            } else if (semiring == OR_MIN_SELECT2ND) {
                const int32_t t = ((const int32_t*)x_val)[p];
                acc_i[i] = (!seen[i] || t < acc_i[i]) ? t : acc_i[i];
            } else {
                const int32_t t = (values ? (values[q] != 0.0f) : 1) && ((const uint8_t*)x_val)[p] != 0;
                acc_i[i] = seen[i] ? (acc_i[i] || t) : t;
            }
            seen[i] = 1;
        }
    }
    int64_t count = 0;
    for (int64_t i = 0; i < m && rc == 0; ++i) {
        if (!seen[i]) continue;
        y_idx[count] = (int32_t)i;
        if (semiring == OR_PLUS_TIMES) ((double*)y_val)[count] = acc_d[i];
        else if (semiring == OR_MIN_SELECT2ND) ((int32_t*)y_val)[count] = acc_i[i];
        else ((uint8_t*)y_val)[count] = (uint8_t)acc_i[i];
        ++count;
    }
    *nnz_y = count;
    *W = work;
    free(seen); free(acc_d); free(acc_i);
    return rc;
}

/* Plus-times in fp32, the reference of the deterministic mode: each
 * product is rounded to fp32 (Mult), and each row's products are added one
 * at a time in fp32 in product order -- x order, then the column's storage
 * order (Algorithm 1's Add in the order the products are formed).
 * y_val float[m], y_idx in first-touch order.                             */
int oracle_spmspv_f32seq(int64_t m, const int32_t* colptr, const int32_t* rowids, const float* values,
                         int64_t f, const int32_t* x_idx, const float* x_val, int32_t* y_idx,
                         float* y_val, int64_t* nnz_y) {
    unsigned char* seen = (unsigned char*)calloc((size_t)(m > 0 ? m : 1), 1);
    float* acc = (float*)malloc((size_t)(m > 0 ? m : 1) * sizeof(float));
    int64_t count = 0;
    for (int64_t p = 0; p < f; ++p) {
        int32_t j = x_idx[p];
        for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {
            int32_t i = rowids[q];
            volatile float t = (values ? values[q] : 1.0f) * x_val[p];
            if (!seen[i]) { seen[i] = 1; acc[i] = t; y_idx[count++] = i; }
            else { volatile float s = acc[i] + t; acc[i] = s; }
        }
    }
    for (int64_t r = 0; r < count; ++r) y_val[r] = acc[y_idx[r]];
    *nnz_y = count;
    free(seen); free(acc);
    return 0;
}

/*
 * Breadth-first search from `root`, edges j -> i for every stored A(i,j)
 * (x over columns reaches rows).  FIFO queue.  level[v] = hop count or -1;
 * parent[v] = the smallest u with A(v,u) stored and level[u] = level[v]-1,
 * parent[root] = root, -1 when unreached.  Returns the number of levels
 * (max level + 1).
 */
int oracle_bfs(int64_t n, const int32_t* colptr, const int32_t* rowids, int32_t root, int32_t* level,
               int32_t* parent) {
    for (int64_t v = 0; v < n; ++v) { level[v] = -1; if (parent) parent[v] = -1; }
    int32_t* queue = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t head = 0, tail = 0;
    level[root] = 0;
    queue[tail++] = root;
    int32_t maxl = 0;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t q = colptr[u]; q < colptr[u + 1]; ++q) {
            int32_t v = rowids[q];
            if (level[v] < 0) {
                level[v] = level[u] + 1;
                if (level[v] > maxl) maxl = level[v];
                queue[tail++] = v;
            }
        }
    }
    if (parent) {
        for (int64_t u = 0; u < n; ++u) {
            if (level[u] < 0) continue;
            for (int64_t q = colptr[u]; q < colptr[u + 1]; ++q) {
                int32_t v = rowids[q];
                if (level[v] == level[u] + 1 && (parent[v] < 0 || u < parent[v])) parent[v] = (int32_t)u;
            }
        }
        parent[root] = root;
    }
    free(queue);
    return maxl + 1;
}

/*
 * Schedule-selector MLP in fp64: 6 inputs -> 64 ReLU -> 64 ReLU -> 10 logits,
 * softmax cross-entropy, mean over the batch.  Parameter layout (flat):
 *   W1[h1][in], b1[h1], W2[h2][h1], b2[h2], W3[out][h2], b3[out].
 * oracle_mlp_forward writes logits[B][out]; oracle_mlp_loss_grad writes the
 * gradient of the mean loss (same layout as the parameters) and returns the
 * mean loss.  Plain loops, no blocking.
 */
static void mlp_layers(int in, int h1, int h2, int out, const double* p, const double* x, double* a1, double* a2,
                       double* z3) {
    const double* W1 = p;
    const double* b1 = W1 + h1 * in;
    const double* W2 = b1 + h1;
    const double* b2 = W2 + h2 * h1;
    const double* W3 = b2 + h2;
    const double* b3 = W3 + out * h2;
    for (int i = 0; i < h1; ++i) {
        double z = b1[i];
        for (int c = 0; c < in; ++c) z += W1[i * in + c] * x[c];
        a1[i] = z > 0 ? z : 0;
    }
    for (int j = 0; j < h2; ++j) {
        double z = b2[j];
        for (int i = 0; i < h1; ++i) z += W2[j * h1 + i] * a1[i];
        a2[j] = z > 0 ? z : 0;
    }
    for (int k = 0; k < out; ++k) {
        double z = b3[k];
        for (int j = 0; j < h2; ++j) z += W3[k * h2 + j] * a2[j];
        z3[k] = z;
    }
}

void oracle_mlp_forward(int in, int h1, int h2, int out, int B, const double* p, const double* X, double* logits,
                        double* unused0, double* unused1, double* unused2, double* unused3) {
    (void)unused0; (void)unused1; (void)unused2; (void)unused3;
    double* a1 = (double*)malloc(sizeof(double) * h1);
    double* a2 = (double*)malloc(sizeof(double) * h2);
    for (int s = 0; s < B; ++s) mlp_layers(in, h1, h2, out, p, X + s * in, a1, a2, logits + s * out);
    free(a1); free(a2);
}

double oracle_mlp_loss_grad(int in, int h1, int h2, int out, int B, const double* p, const double* X,
                            const int* labels, double* grad, double* unused0, double* unused1, double* unused2,
                            double* unused3) {
    (void)unused0; (void)unused1; (void)unused2; (void)unused3;
    const int np = h1 * in + h1 + h2 * h1 + h2 + out * h2 + out;
    for (int q = 0; q < np; ++q) grad[q] = 0;
    const double* W2 = p + h1 * in + h1;
    const double* W3 = W2 + h2 * h1 + h2;
    double* gW1 = grad;
    double* gb1 = gW1 + h1 * in;
    double* gW2 = gb1 + h1;
    double* gb2 = gW2 + h2 * h1;
    double* gW3 = gb2 + h2;
    double* gb3 = gW3 + out * h2;
    double* a1 = (double*)malloc(sizeof(double) * h1);
    double* a2 = (double*)malloc(sizeof(double) * h2);
    double* z3 = (double*)malloc(sizeof(double) * out);
    double* d3 = (double*)malloc(sizeof(double) * out);
    double* d2 = (double*)malloc(sizeof(double) * h2);
    double* d1 = (double*)malloc(sizeof(double) * h1);
    double loss = 0;
    for (int s = 0; s < B; ++s) {
        const double* x = X + s * in;
        mlp_layers(in, h1, h2, out, p, x, a1, a2, z3);
        double mx = z3[0];
        for (int k = 1; k < out; ++k) if (z3[k] > mx) mx = z3[k];
        double se = 0;
        for (int k = 0; k < out; ++k) se += exp(z3[k] - mx);
        loss += -(z3[labels[s]] - mx - log(se));
        /* d(mean loss)/d z3 = (softmax - onehot) / B */
        for (int k = 0; k < out; ++k) d3[k] = (exp(z3[k] - mx) / se - (k == labels[s] ? 1.0 : 0.0)) / B;
        for (int k = 0; k < out; ++k) {
            gb3[k] += d3[k];
            for (int j = 0; j < h2; ++j) gW3[k * h2 + j] += d3[k] * a2[j];
        }
        for (int j = 0; j < h2; ++j) {
            double t = 0;
            for (int k = 0; k < out; ++k) t += W3[k * h2 + j] * d3[k];
            d2[j] = a2[j] > 0 ? t : 0;
        }
        for (int j = 0; j < h2; ++j) {
            gb2[j] += d2[j];
            for (int i = 0; i < h1; ++i) gW2[j * h1 + i] += d2[j] * a1[i];
        }
        for (int i = 0; i < h1; ++i) {
            double t = 0;
            for (int j = 0; j < h2; ++j) t += W2[j * h1 + i] * d2[j];
            d1[i] = a1[i] > 0 ? t : 0;
        }
        for (int i = 0; i < h1; ++i) {
            gb1[i] += d1[i];
            for (int c = 0; c < in; ++c) gW1[i * in + c] += d1[i] * x[c];
        }
    }
    free(a1); free(a2); free(z3); free(d3); free(d2); free(d1);
    return loss / B;
}

/*
 * Data-driven (delta) PageRank in fp64.  The paper cites PageRank as a
 * data-driven SpMSpV customer whose vertices stop sending updates once
 * their value has converged (Introduction); it gives no formula, so this
 * is the reading the GPU library implements:
 *   outdeg(j) = stored entries of column j; A_n(i, j) = 1 / outdeg(j) for
 *   every stored A(i, j) (edge j -> i); columns with no entries send
 *   nothing (their mass is dropped).
 *   p = 0; delta = (1 - d) / n at every vertex; every vertex active.
 *   repeat:  p += delta;
 *            stop when no vertex is active or max_iter multiplies are done;
 *            delta' = d * A_n * (delta restricted to active vertices), as a
 *              sparse product: its pattern is the rows reached (structural);
 *            active = { v in pattern(delta') : delta'(v) > tol * p(v) }
 *              (p before adding delta'); delta = delta'.
 * rank[n] receives p.  active_counts (nullable, max_iter + 1 entries)
 * receives the number of active vertices before each multiply.  Returns
 * the number of multiplies performed.
 */
int oracle_pagerank(int64_t n, const int32_t* colptr, const int32_t* rowids, double damping, double tol,
                    int max_iter, double* rank, int32_t* active_counts) {
    double* delta = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double* next = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    unsigned char* active = (unsigned char*)malloc((size_t)(n > 0 ? n : 1));
    unsigned char* reached = (unsigned char*)malloc((size_t)(n > 0 ? n : 1));
    for (int64_t v = 0; v < n; ++v) {
        rank[v] = 0.0;
        delta[v] = (1.0 - damping) / (double)n;
        active[v] = 1;
    }
    int it = 0;
    for (;;) {
        int64_t nact = 0;
        for (int64_t v = 0; v < n; ++v) {
            rank[v] += delta[v];
            nact += active[v];
        }
        if (active_counts) active_counts[it] = (int32_t)nact;
        if (nact == 0 || it == max_iter) break;
        for (int64_t v = 0; v < n; ++v) {
            next[v] = 0.0;
            reached[v] = 0;
        }
        for (int64_t j = 0; j < n; ++j) {
            const int64_t len = colptr[j + 1] - colptr[j];
            if (!active[j] || len == 0) continue;
            const double c = damping * delta[j] / (double)len;
            for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {
                next[rowids[q]] += c;
                reached[rowids[q]] = 1;
            }
        }
        for (int64_t v = 0; v < n; ++v) {
            active[v] = reached[v] && next[v] > tol * rank[v];
            delta[v] = next[v];
        }
        ++it;
    }
    free(delta); free(next); free(active); free(reached);
    return it;
}
