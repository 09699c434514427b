"""Pins for the CPU oracle: checks against things other than the oracle itself.

Brute force on tiny dense inputs, scipy.sparse products, closed forms
(x = e_j, permutation matrices, grid BFS levels), the paper's invariants
(products counted = sum of selected column lengths; unique indices over all
buckets = nnz(y) <= products) and a hand-computed fixture built on the
structure of the paper's Figure 1 caption.
"""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    synth.build(force=False)
    oracle.build(force=False)


def random_csc(rng, m, n, density, unsorted=True, with_values=True):
    """Random CSC with optional shuffled row order inside columns."""
    P = rng.random((m, n)) < density
    colptr = np.zeros(n + 1, np.int32)
    rows = []
    for j in range(n):
        r = np.nonzero(P[:, j])[0].astype(np.int32)
        if unsorted:
            rng.shuffle(r)
        rows.append(r)
        colptr[j + 1] = colptr[j] + r.size
    rowids = np.concatenate(rows) if rows else np.zeros(0, np.int32)
    vals = None
    if with_values:
        vals = ((rng.integers(0, 1 << 24, rowids.size) + 1) / float(1 << 24)).astype(np.float32)
    return synth.CSC(m, n, colptr, rowids.astype(np.int32), vals)


def dense_of(A):
    P = np.zeros((A.m, A.n), bool)
    D = np.zeros((A.m, A.n), np.float64)
    for j in range(A.n):
        for q in range(A.colptr[j], A.colptr[j + 1]):
            P[A.rowids[q], j] = True
            D[A.rowids[q], j] = 1.0 if A.values is None else float(A.values[q])
    return P, D


def as_dict(idx, val):
    return {int(i): v for i, v in zip(idx.tolist(), val.tolist())}


# ---------------------------------------------------------------- brute force
@settings(max_examples=60, deadline=None)
@given(m=st.integers(1, 24), n=st.integers(1, 24), dens=st.floats(0.0, 0.6), fx=st.floats(0.0, 1.0),
       seed=st.integers(0, 10**6), sorted_out=st.booleans())
def test_brute_force_all_semirings(m, n, dens, fx, seed, sorted_out):
    rng = np.random.default_rng(seed)
    A = random_csc(rng, m, n, dens)
    f = int(round(fx * n))
    S = rng.permutation(n)[:f].astype(np.int32)
    xv = ((rng.integers(0, 1 << 24, f) + 1) / float(1 << 24)).astype(np.float32)
    P, D = dense_of(A)
    present = P[:, S].any(axis=1)
    expect_rows = np.nonzero(present)[0]

    # plus-times: dense fp64 mat-vec over the selected columns
    yi, yv, W = oracle.spmspv(A, S, xv, oracle.PLUS_TIMES, sorted_output=sorted_out)
    assert W == int(np.diff(A.colptr)[S].sum())
    assert sorted(yi.tolist()) == expect_rows.tolist()
    ref = D[:, S] @ xv.astype(np.float64)
    got = as_dict(yi, yv)
    for i in expect_rows:
        assert abs(got[int(i)] - ref[i]) <= 1e-14 * max(1.0, abs(ref[i]))
    if sorted_out:
        assert np.all(np.diff(yi) > 0)

    # min-select2nd with arbitrary int values
    xi = rng.integers(-1000, 1000, f).astype(np.int32)
    yi, yv, _ = oracle.spmspv(A, S, xi, oracle.MIN_SELECT2ND, sorted_output=sorted_out)
    got = as_dict(yi, yv)
    assert sorted(got) == expect_rows.tolist()
    for i in expect_rows:
        assert got[int(i)] == min(int(xi[k]) for k in range(f) if P[i, S[k]])

    # or-and with explicit false entries in x and zeros in A
    xb = (rng.random(f) < 0.5).astype(np.uint8)
    yi, yv, _ = oracle.spmspv(A, S, xb, oracle.OR_AND, sorted_output=sorted_out)
    got = as_dict(yi, yv)
    assert sorted(got) == expect_rows.tolist()
    for i in expect_rows:
        assert got[int(i)] == int(any(P[i, S[k]] and D[i, S[k]] != 0 and xb[k] for k in range(f)))


def test_mask_drops_rows():
    rng = np.random.default_rng(5)
    A = random_csc(rng, 30, 20, 0.3)
    S = np.arange(0, 20, 3, dtype=np.int32)
    xv = np.ones(S.size, np.float32)
    mask = (rng.random(30) < 0.5).astype(np.uint8)
    yi, _, _ = oracle.spmspv(A, S, xv, mask=None)
    ym, _, _ = oracle.spmspv(A, S, xv, mask=mask)
    assert sorted(ym.tolist()) == sorted(i for i in yi.tolist() if not mask[i])


# ------------------------------------------------------------ library routine
def test_scipy_plus_times_rmat_s14():
    A = synth.rmat(14, seed=1)
    S, xv = synth.sparse_x(A.n, 164, seed=1000)
    yi, yv, W = oracle.spmspv(A, S, xv)
    sp = A.to_scipy()
    ref = sp[:, S] @ xv.astype(np.float64)
    nz = np.nonzero(ref)[0]   # values are in (0, 1]: no cancellation, pattern = nonzeros
    assert sorted(yi.tolist()) == nz.tolist()
    got = np.zeros(A.m)
    got[yi] = yv
    np.testing.assert_allclose(got[nz], ref[nz], rtol=1e-13)
    assert W == int(A.degrees()[S].sum())


# ------------------------------------------------------------------ invariants
def test_invariants_rmat_s14():
    A = synth.rmat(14, seed=1)
    S, xv = synth.sparse_x(A.n, 164, seed=1001)
    deg = A.degrees()
    yi, yv, W = oracle.spmspv(A, S, xv)
    # I1: products = sum of selected column lengths (work bound)
    assert W == int(deg[S].sum())
    # I2: nnz(y) = size of the union of selected column patterns <= W
    union = set()
    for j in S:
        union.update(A.rowids[A.colptr[j]:A.colptr[j + 1]].tolist())
    assert yi.size == len(union) <= W
    # I3: 1^T (A x) = (1^T A) x
    colsum = np.add.reduceat(np.r_[A.values.astype(np.float64), 0.0], A.colptr[:-1].astype(np.int64))
    colsum[deg == 0] = 0.0
    assert abs(yv.sum() - float((colsum[S] * xv.astype(np.float64)).sum())) <= 1e-12 * yv.sum()
    # I4: min-select2nd with x_val = column index gives the minimum selected in-neighbour
    yi2, yv2, _ = oracle.spmspv(A, S, S.copy(), oracle.MIN_SELECT2ND)
    best = {}
    for j in S.tolist():
        for i in A.rowids[A.colptr[j]:A.colptr[j + 1]].tolist():
            best[i] = min(best.get(i, 1 << 30), j)
    assert as_dict(yi2, yv2) == best
    # I5: or-and with all-true x: every value true
    yi3, yv3, _ = oracle.spmspv(A, S, np.ones(S.size, np.uint8), oracle.OR_AND)
    assert set(yi3.tolist()) == union and np.all(yv3 == 1)
    # I6: sorted output strictly increasing, same set
    yi4, yv4, _ = oracle.spmspv(A, S, xv, sorted_output=True)
    assert np.all(np.diff(yi4) > 0) and set(yi4.tolist()) == union
    assert np.array_equal(yv4, np.array([as_dict(yi, yv)[i] for i in yi4.tolist()]))
    # output order of x does not matter (sortedness of x does not affect correctness)
    order = np.argsort(S)
    yi5, yv5, _ = oracle.spmspv(A, S[order], xv[order], sorted_output=True)
    assert np.array_equal(yi5, yi4)
    np.testing.assert_allclose(yv5, yv4, rtol=1e-15)


# --------------------------------------------------------- special-case pins
def test_unit_vector_is_a_column():
    A = synth.rmat(12, seed=3)
    for j in [0, 5, int(np.argmax(A.degrees()))]:
        S = np.array([j], np.int32)
        one = np.ones(1, np.float32)
        yi, yv, W = oracle.spmspv(A, S, one, sorted_output=True)
        col = A.rowids[A.colptr[j]:A.colptr[j + 1]]
        order = np.argsort(col)
        assert np.array_equal(yi, col[order])
        assert np.array_equal(yv, A.values[A.colptr[j]:A.colptr[j + 1]][order].astype(np.float64))
        yi32, yv32 = oracle.spmspv_f32seq(A, S, one)
        assert np.array_equal(yi32, col) and np.array_equal(yv32, A.values[A.colptr[j]:A.colptr[j + 1]])


def test_permutation_matrix_single_products():
    rng = np.random.default_rng(11)
    n = 500
    perm = rng.permutation(n).astype(np.int32)
    A = synth.CSC(n, n, np.arange(n + 1, dtype=np.int32), perm, synth.values(n, 9))
    S, xv = synth.sparse_x(n, 120, seed=4)
    yi, yv = oracle.spmspv_f32seq(A, S, xv)
    assert np.array_equal(yi, perm[S])
    assert np.array_equal(yv, (A.values[S] * xv).astype(np.float32))   # RN32(a*x), bit-exact
    yi64, yv64, _ = oracle.spmspv(A, S, xv)
    assert np.array_equal(yi64, perm[S])
    assert np.array_equal(yv64, A.values[S].astype(np.float64) * xv.astype(np.float64))


def test_f32_two_contributions_order_free():
    # column j holds rows j and j+1 (mod n): every row gets exactly two products, and
    # RN32(RN32(p1) + RN32(p2)) does not depend on their order
    n = 64
    colptr = np.arange(0, 2 * n + 1, 2, dtype=np.int32)
    rowids = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).ravel().astype(np.int32)
    A = synth.CSC(n, n, colptr, rowids, synth.values(2 * n, 2))
    S = np.arange(n, dtype=np.int32)
    xv = synth.values(n, 3, stream=99)
    yi, yv = oracle.spmspv_f32seq(A, S, xv)
    yi_r, yv_r = oracle.spmspv_f32seq(A, S[::-1].copy(), xv[::-1].copy())
    a, b = as_dict(yi, yv), as_dict(yi_r, yv_r)
    assert a == b
    for i, v in a.items():
        p1 = np.float32(A.values[2 * i] * xv[i])
        j = (i - 1) % n
        p2 = np.float32(A.values[2 * j + 1] * xv[j])
        assert v == np.float32(p1 + p2)


# ------------------------------------------------------------------ golden
def test_figure1_structure_fixture():
    g = json.load(open(os.path.join(GOLDEN, "figure1_structure.json")))
    ent = sorted(g["entries"], key=lambda e: (e[1], e[0]))
    colptr = np.zeros(g["n"] + 1, np.int32)
    for _, j, _ in ent:
        colptr[j + 1] += 1
    colptr = np.cumsum(colptr).astype(np.int32)
    A = synth.CSC(g["m"], g["n"], colptr, np.array([e[0] for e in ent], np.int32),
                  np.array([e[2] for e in ent], np.float32))
    S = np.array(g["x_idx"], np.int32)
    yi, yv, W = oracle.spmspv(A, S, np.array(g["x_val"], np.float32))
    assert W == g["expected_W"] and yi.size == g["expected_unique"]
    assert as_dict(yi, yv) == {int(k): v for k, v in g["expected_plus_times"].items()}
    yi, yv, _ = oracle.spmspv(A, S, S.copy(), oracle.MIN_SELECT2ND)
    assert as_dict(yi, yv) == {int(k): v for k, v in g["expected_min_select2nd_xval_is_index"].items()}
    # bucket sizes with rows split evenly over 4 buckets
    per = g["m"] // g["nbuckets"]
    sizes = [0] * g["nbuckets"]
    for j in S:
        for q in range(colptr[j], colptr[j + 1]):
            sizes[A.rowids[q] // per] += 1
    assert sizes == g["expected_bucket_sizes_rows_per_bucket_2"]


# --------------------------------------------------------------------- BFS
def test_bfs_levels_vs_scipy_directed():
    from scipy.sparse.csgraph import shortest_path
    A = synth.rmat(10, seed=7)   # directed
    root = int(synth.roots(A, 1, 2000)[0])
    lev, par, nl = oracle.bfs(A, root)
    # edges j -> i for stored A(i, j): scipy's graph[u, v] is an edge u -> v, so pass A^T
    d = shortest_path(A.to_scipy().T.tocsr(), unweighted=True, indices=root)
    ref = np.where(np.isinf(d), -1, d).astype(np.int64)
    assert np.array_equal(lev.astype(np.int64), ref)
    assert nl == int(ref.max()) + 1
    # minimum-parent rule by brute force
    P, _ = dense_of(A)
    for v in range(A.n):
        if lev[v] <= 0:
            assert par[v] == (root if v == root else -1)
            continue
        cand = [u for u in range(A.n) if P[v, u] and lev[u] == lev[v] - 1]
        assert par[v] == min(cand)


def test_bfs_grid_closed_form():
    nx = ny = nz = 12
    G = synth.grid(nx, ny, nz, diag=True)
    lev, par, nl = oracle.bfs(G, 0)
    v = np.arange(G.n)
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    assert np.array_equal(lev, (x + y + z).astype(np.int32))
    assert nl == (nx - 1) + (ny - 1) + (nz - 1) + 1
    expect_par = np.where(z > 0, v - nx * ny, np.where(y > 0, v - nx, v - 1))
    expect_par[0] = 0
    assert np.array_equal(par, expect_par.astype(np.int32))


def test_grid_256_layer_sizes_closed_form():
    # level sizes of the 256^3 corner BFS: lattice points with x+y+z = L
    n = 256
    L = np.arange(3 * (n - 1) + 1)
    cnt = np.zeros(L.size, np.int64)
    s = np.arange(n)
    for x in range(n):
        yz = x + s[:, None] + s[None, :]
        cnt += np.bincount(yz.ravel(), minlength=L.size)[: L.size]
    assert L.size == 766 and cnt.sum() == n ** 3 and cnt.max() == 49152 and cnt.argmax() == 382


def test_validate_codes():
    A = synth.rmat(8, seed=1)
    assert oracle.validate(A.m, A.n, A.colptr, A.rowids, np.array([1, 2, 3])) == 0
    assert oracle.validate(A.m, A.n, A.colptr, A.rowids, np.array([1, 1])) == -4
    assert oracle.validate(A.m, A.n, A.colptr, A.rowids, np.array([A.n])) == -3
    bad = A.rowids.copy()
    bad[0] = A.m
    assert oracle.validate(A.m, A.n, A.colptr, bad, np.array([0])) == -2
    # colptr: must start at 0 and never decrease (the CSC definition)
    cp = A.colptr.copy()
    cp[0] = 1
    assert oracle.validate(A.m, A.n, cp, A.rowids, np.array([0])) == -1
    j = int(np.argmax(np.diff(A.colptr) > 0))      # a non-empty column: make its end fall below its start
    cp = A.colptr.copy()
    cp[j + 1] = cp[j] - 1
    assert oracle.validate(A.m, A.n, cp, A.rowids, np.array([0])) == -1
    # a valid colptr with an empty column passes
    cp = np.concatenate([[0], A.colptr]).astype(np.int32)
    assert oracle.validate(A.m, A.n + 1, cp, A.rowids, np.array([0, A.n])) == 0
