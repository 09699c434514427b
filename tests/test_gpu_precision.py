"""fp32 plus-times accuracy on rows with hundreds of thousands of terms, the
widest plus-times tile, signed zeros, and the held-out scale-24 graph's
PageRank multiplies.

Contract (products rounded to fp32, any summation order):
|y - y64| <= 1e-5 * sum|terms|, with y64 the oracle's fp64 sum of exact
products.  The merge sums each row in fp64 and rounds once, so the error
is at most the products' own rounding (2^-24 each) plus the final rounding
(2^-24) plus k 2^-53 sum|terms| for k terms: the tests also assert that
tighter bound, which a row summed sequentially in fp32 misses once it has
about 10^5 terms (u sqrt(k) growth)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare, rmat24_pattern, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def spv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_07902_amd as spv
    spv.load_library()
    oracle.build(force=False)
    synth.build(force=False)
    return spv


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def tight_bound(terms_abs, k):
    """fp32 rounding of each product and of the sum, fp64 accumulation."""
    return (2.0 ** -23 + np.maximum(k, 1) * 2.0 ** -53) * terms_abs


def hub_matrix(n, m, seed):
    """Every column holds row 0 (the hub) and one other row, so selecting all
    n columns gives row 0 exactly n terms; row m-1 is a second hub fed by
    every third column."""
    rng = np.random.default_rng(seed)
    other = rng.integers(1, m - 1, n)
    cols = np.arange(n)
    extra = cols[cols % 3 == 0]
    rows = np.concatenate([np.zeros(n, np.int64), other, np.full(extra.size, m - 1)])
    cc = np.concatenate([cols, cols, extra])
    colptr, rowids = synth.coo_to_csc(m, n, rows.astype(np.int32), cc.astype(np.int32), drop_self=False)
    return synth.CSC(m, n, colptr, rowids, synth.values(rowids.size, seed + 1))


def row_terms(A, S, xv):
    """Per-row sum of |a * x| and term counts (fp64), for the bounds."""
    cols = np.repeat(np.arange(A.n), np.diff(A.colptr))
    xd = np.zeros(A.n)
    xd[S] = np.abs(xv.astype(np.float64))
    sel = np.zeros(A.n, bool)
    sel[S] = True
    keep = sel[cols]
    av = np.abs(A.values.astype(np.float64)) if A.values is not None else np.ones(A.nnz)
    t = np.zeros(A.m)
    k = np.zeros(A.m)
    np.add.at(t, A.rowids[keep], av[keep] * xd[cols[keep]])
    np.add.at(k, A.rowids[keep], 1.0)
    return t, k


@pytest.mark.parametrize("tile", [8, 13, 14])
def test_hub_row_with_450k_terms(spv, tile):
    """One row with 450,000 terms and one with 150,000, through the merge's
    streamed (large-bucket) path at three tile widths."""
    n, m = 450_000, 70_000
    A = hub_matrix(n, m, seed=81)
    M = spv.Matrix.from_csc(A)
    s = M.schedule
    s.tile_log2 = tile
    M.schedule = s
    S = np.arange(n, dtype=np.int32)
    xv = synth.values(n, 82)
    gi, gv, nnz = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True)
    oi, ov, W = oracle.spmspv(A, S, xv, 0, sorted_output=True)
    t, k = row_terms(A, S, xv)
    compare(0, gi, gv, oi, ov, sorted_output=True, terms_abs=t[oi])
    err = np.abs(to_np(gv).astype(np.float64) - ov)
    assert np.all(err <= tight_bound(t[oi], k[oi])), f"worst {np.max(err / t[oi]):.3e}"
    assert k[0] == n and oi[0] == 0
    M.close()


def test_hub_rows_in_a_batch(spv):
    """Two vectors that both select every column: each vector's hub row gets
    450,000 terms through the batched (keyed) merge."""
    n, m = 450_000, 70_000
    A = hub_matrix(n, m, seed=83)
    M = spv.Matrix.from_csc(A)
    S = np.arange(n, dtype=np.int32)
    xs = [(S, synth.values(n, 84)), (S[::-1].copy(), synth.values(n, 85))]
    off = np.array([0, n, 2 * n], np.int64)
    idx = np.concatenate([x[0] for x in xs])
    val = np.concatenate([x[1] for x in xs])
    M.attach_batch(2, max_f=2 * n, max_products=2 * A.nnz)
    y_off, y_idx, y_val, total = M.spmspv_batch(dev(off), dev(idx), dev(val), semiring=0)
    yo = to_np(y_off)
    for b, (Sb, xb) in enumerate(xs):
        oi, ov, _ = oracle.spmspv(A, Sb, xb, 0, sorted_output=True)
        t, k = row_terms(A, Sb, xb)
        gi, gv = y_idx[yo[b]:yo[b + 1]], y_val[yo[b]:yo[b + 1]]
        compare(0, gi, gv, oi, ov, sorted_output=True, terms_abs=t[oi])
        err = np.abs(to_np(gv).astype(np.float64) - ov)
        assert np.all(err <= tight_bound(t[oi], k[oi]))
    M.close()


@pytest.mark.parametrize("tile", [14, 15])
def test_widest_plus_times_tile_walks_in_two_rounds(spv, tile):
    """Tile 2^14 (the widest plus-times tile; a schedule asking for 2^15 runs
    as 2^14): every row of a 16,384-row bucket is touched, more than the
    8,192 rows one round of the ordered walk stages, so y is written in two
    rounds per bucket and must stay ascending across them."""
    n = m = 40_000
    rng = np.random.default_rng(86)
    rows = rng.integers(0, m, n * 20).astype(np.int32)
    cols = np.repeat(np.arange(n), 20).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(m, n, rows, cols, drop_self=False)
    A = synth.CSC(m, n, colptr, rowids, synth.values(rowids.size, 87))
    M = spv.Matrix.from_csc(A)
    s = M.schedule
    s.tile_log2 = tile
    M.schedule = s
    for f in (n, n // 2):
        S, xv = synth.sparse_x(n, f, seed=88 + f)
        gi, gv, nnz = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True)
        oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
        compare(0, gi, gv, oi, ov, sorted_output=True)
        if f == n:
            assert np.count_nonzero(oi < 16384) > 8192
    M.close()


def test_signed_zero_rows(spv):
    """Rows whose every product is -0.0 are in y with value -0.0; rows whose
    products cancel or mix +0.0 and -0.0 hold +0.0 (IEEE sums, whatever the
    order).  A values are +-1 or +-0, x values +-1 or +-0."""
    m, n = 5000, 3000
    rng = np.random.default_rng(89)
    rows = rng.integers(0, m, n * 6).astype(np.int32)
    cols = np.repeat(np.arange(n), 6).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(m, n, rows, cols, drop_self=False)
    av = rng.choice(np.array([1.0, -1.0, 0.0, -0.0], np.float32), rowids.size)
    A = synth.CSC(m, n, colptr, rowids, av)
    M = spv.Matrix.from_csc(A)
    S = rng.permutation(n)[:2500].astype(np.int32)
    xv = rng.choice(np.array([1.0, -1.0, 0.0, -0.0], np.float32), S.size)
    gi, gv, _ = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True)
    oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
    assert np.array_equal(to_np(gi), oi)
    g = to_np(gv).astype(np.float64)
    assert np.array_equal(g, ov)                                   # small integers: exact in any order
    z = ov == 0.0
    assert z.sum() > 100 and np.signbit(ov[z]).sum() > 10
    assert np.array_equal(np.signbit(g[z]), np.signbit(ov[z]))
    M.close()


# ---------------------------------------------------------------- scale 24
def pagerank_x(A, delta, active, d=0.85):
    """x of one data-driven PageRank multiply: (j, d * delta(j) / outdeg(j))
    for active j with outdeg(j) > 0, as fp32."""
    deg = np.diff(A.colptr)
    S = np.nonzero(active & (deg > 0))[0].astype(np.int32)
    return S, (d * delta[S] / deg[S]).astype(np.float32)


def test_rmat24_pagerank_first_multiplies(spv):
    """The first three multiplies of data-driven PageRank on the held-out
    scale-24 graph (f = 8.87M columns, 521M products in the first: the
    406,317-entry hub row gets every one of its entries as a term), each
    compared element by element with the oracle on identical x.  x of the
    next multiply comes from the oracle's result."""
    A = rmat24_pattern()
    M = spv.Matrix.from_csc(A, pattern=True)
    n, d, tol = A.n, 0.85, 1e-6
    deg = np.diff(A.colptr)
    rank = np.zeros(n)
    delta = np.full(n, (1 - d) / n)
    active = np.ones(n, bool)
    worst = 0.0
    for step in range(3):
        rank += delta
        S, xv = pagerank_x(A, delta, active, d)
        gi, gv, nnz = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True)
        oi, ov, W = oracle.spmspv(A, S, xv, 0, sorted_output=True)
        if step == 0:
            assert S.size == 8871018 and W == A.nnz
        # pattern matrix and positive x: sum|terms| = y64
        compare(0, gi, gv, oi, ov, sorted_output=True)
        g = to_np(gv).astype(np.float64)
        if step == 0:
            hub = int(np.argmax(deg))
            assert deg[hub] == 406317 and oi[np.searchsorted(oi, hub)] == hub
        err = np.abs(g - ov)
        assert np.all(err <= tight_bound(ov, deg[oi])), f"step {step}: worst {np.max(err / ov):.3e}"
        worst = max(worst, float(np.max(err / ov)))
        nd = np.zeros(n)
        nd[oi] = ov
        active = nd > tol * rank
        delta = nd
    assert worst < 1.2e-7
    M.close()


def pagerank_bound(ref, it_ref, tol):
    return (2 * max(it_ref, 1) * tol + 2e-5) * np.max(ref)


def test_rmat24_pagerank_three_steps(spv):
    """Three PageRank steps on the device (one pagerank_run, max_iter 3)
    against the oracle's, under the activity-threshold bound."""
    A = rmat24_pattern()
    M = spv.Matrix.from_csc(A, pattern=True)
    r, it = M.pagerank(0.85, 1e-6, 3)
    ref, it_ref, _ = oracle.pagerank(A, 0.85, 1e-6, 3)
    assert it == it_ref == 3
    g = to_np(r).astype(np.float64)
    err = np.max(np.abs(g - ref))
    assert err <= pagerank_bound(ref, it_ref, 1e-6), err
    assert np.max(np.abs(g - ref) / ref) < 1e-5
    M.close()


def test_rmat24_pagerank_converged_residual(spv):
    """The converged device PageRank on the scale-24 graph satisfies the
    fixed-point equation p = (1-d)/n + d A_n p up to the activity threshold
    (a property that holds at any size; checked with scipy's fp64 product)."""
    import scipy.sparse as sp
    A = rmat24_pattern()
    M = spv.Matrix.from_csc(A, pattern=True)
    tol = 1e-6
    r, it = M.pagerank(0.85, tol, 200)
    assert 10 < it < 200
    g = to_np(r).astype(np.float64)
    M.close()
    deg = np.diff(A.colptr).astype(np.float64)
    w = np.where(deg > 0, 0.85 * g / np.maximum(deg, 1), 0.0)
    An = sp.csc_matrix((np.ones(A.nnz, np.float32), A.rowids, A.colptr), shape=(A.n, A.n))
    push = An @ w
    res = g - 0.15 / A.n - push
    assert np.max(np.abs(res)) <= 4 * it * tol * np.max(g)
