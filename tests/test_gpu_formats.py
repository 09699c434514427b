"""GPU parity of the format variants (Background: Notation, and Sparse
matrix and vector data structures) against the oracle:

* left multiplication y' = x'A (SPMSPV_LEFT) on handles with a transpose
  (WITH_TRANSPOSE, SYMMETRIC), square and rectangular, plain, masked and
  with the GraphBLAS rules; against oracle_spmspv_left, and the masked and
  GraphBLAS forms against the oracle on the transpose scipy builds;
* DCSC input (spmspv_create_dcsc): hypersparse and ordinary matrices, x
  naming absent columns, batched calls, BFS and the GraphBLAS rules, the
  benchmark's scale-22 graph; against oracle_spmspv_dcsc and the CSC oracle;
* bitvector x and y (spmspv_run_bitvector): every semiring, empty and full
  x, lengths that are not multiples of 32, LEFT and DCSC handles, against
  the oracle's list result in bitvector form.

Index sets and int32 / bool values bit-exact; fp32 within 1e-5 of the fp64
oracle (all values positive)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VDT = {0: np.float32, 1: np.int32, 2: np.uint8}


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


def xvals(rng, semiring, k):
    if semiring == 0:
        return ((rng.integers(0, 1 << 24, k) + 1) / float(1 << 24)).astype(np.float32)
    if semiring == 1:
        return rng.integers(-(1 << 30), 1 << 30, k).astype(np.int32)
    return (rng.random(k) < 0.7).astype(np.uint8)


def transpose(A):
    T = A.to_scipy().T.tocsc()
    T.sort_indices()
    vals = None if A.values is None else T.data.astype(np.float32)
    return synth.CSC(A.n, A.m, T.indptr.astype(np.int32), T.indices.astype(np.int32), vals)


def rect(m, n, k, seed):
    rng = np.random.default_rng(seed)
    colptr, rowids = synth.coo_to_csc(m, n, rng.integers(0, m, k).astype(np.int32),
                                      rng.integers(0, n, k).astype(np.int32), drop_self=False)
    return synth.CSC(m, n, colptr, rowids, synth.values(rowids.size, seed))


# ------------------------------------------------------------ left multiply

@pytest.fixture(scope="module")
def left_cases(spv):
    out = {}
    A = synth.rmat(14, 16, seed=31)                      # directed: A != A^T
    out["rmat14"] = (A, spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE))
    W = rect(3000, 90000, 400000, 2)                     # wide: A^T has 90000 rows
    out["wide"] = (W, spv.Matrix.from_csc(W, flags=spv.WITH_TRANSPOSE))
    T = rect(90000, 3000, 400000, 3)                     # tall
    out["tall"] = (T, spv.Matrix.from_csc(T, flags=spv.WITH_TRANSPOSE))
    yield out
    for _, M in out.values():
        M.close()


@pytest.mark.parametrize("case", ["rmat14", "wide", "tall"])
@pytest.mark.parametrize("semiring", [0, 1, 2])
def test_left_against_oracle(spv, left_cases, case, semiring):
    A, M = left_cases[case]
    rng = np.random.default_rng(semiring * 7 + len(case))
    for f in (1, max(1, A.m // 100), A.m // 3, A.m):
        S = synth.distinct_indices(A.m, f, seed=int(rng.integers(1 << 30)))
        xv = xvals(rng, semiring, f)
        fl = spv.LEFT
        gi, gv, nnz = M.spmspv(dev(S), dev(xv), semiring=semiring, sorted_output=True, flags=fl)
        oi, ov = oracle.spmspv_left(A, S, xv, semiring)
        assert nnz == oi.size
        compare(semiring, gi, gv, oi, ov, sorted_output=True)
    assert M.last_stats()["err"] == 0


def test_left_on_symmetric_handle_equals_right(spv):
    """SYMMETRIC states A == A^T, values included: a pattern matrix."""
    A0 = synth.rmat(13, 8, seed=4, symmetrize=True)
    A = synth.CSC(A0.m, A0.n, A0.colptr, A0.rowids, None)
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC)
    S, xv = synth.sparse_x(A.n, 500, seed=5)
    gl, vl, _ = M.spmspv(dev(S), dev(xv), sorted_output=True, flags=spv.LEFT)
    gr, vr, _ = M.spmspv(dev(S), dev(xv), sorted_output=True)
    assert np.array_equal(to_np(gl), to_np(gr))
    oi, ov = oracle.spmspv_left(A, S, xv, 0)
    compare(0, gl, vl, oi, ov, sorted_output=True)
    M.close()


def test_left_masked_and_graphblas(spv, left_cases):
    """A bitmap mask over the columns (spmspv_run_masked: masked-out columns
    dropped) and the GraphBLAS rules over the columns, against the oracle on
    the transpose scipy builds."""
    A, M = left_cases["wide"]
    At = transpose(A)
    rng = np.random.default_rng(17)
    S, xv = synth.sparse_x(A.m, 600, seed=18)
    drop = rng.random(A.n) < 0.4
    words = np.zeros((A.n + 31) // 32, np.uint32)
    for j in np.nonzero(drop)[0]:
        words[j >> 5] |= np.uint32(1 << (j & 31))
    y = torch.empty(A.n, dtype=torch.int32, device="cuda")
    yv = torch.empty(A.n, dtype=torch.float32, device="cuda")
    nnz = spv.spmspv_run_masked(M.handle, 0, spv.LEFT | spv.SORTED_OUTPUT, S.size, dev(S), dev(xv),
                                dev(words.view(np.int32)), y, yv, A.n)
    oi, ov, _ = oracle.spmspv(At, S, xv, 0, mask=drop.astype(np.uint8), sorted_output=True)
    compare(0, y[:nnz], yv[:nnz], oi, ov, sorted_output=True)
    # GraphBLAS: value mask over the columns, complement, accumulate Add, replace
    mi = rng.permutation(A.n)[: A.n // 2].astype(np.int32)
    mv = (rng.random(mi.size) < 0.5).astype(np.uint8)
    wi = np.sort(rng.permutation(A.n)[: A.n // 5]).astype(np.int32)
    wv = xvals(rng, 0, wi.size)
    gy = torch.empty(A.n, dtype=torch.int32, device="cuda")
    gyv = torch.empty(A.n, dtype=torch.float32, device="cuda")
    k = spv.spmspv_run_graphblas(M.handle, 0, spv.LEFT, S.size, dev(S), dev(xv), dev(mi), dev(mv), mi.size,
                                 spv.MASK_COMPLEMENT | spv.MASK_REPLACE, spv.ACCUM_ADD, dev(wi), dev(wv), wi.size,
                                 gy, gyv, A.n)
    oi, ov = oracle.spmspv_graphblas(At, S, xv, 0, mask_idx=mi, mask_val=mv, complement=True, w_idx=wi,
                                     w_val=wv.astype(np.float64), accum=oracle.ACCUM_ADD, replace=True)
    assert np.array_equal(to_np(gy[:k]), oi)
    ref = np.zeros(A.n)
    ref[oi] = ov
    got = to_np(gyv[:k]).astype(np.float64)
    assert np.all(np.abs(got - ov) <= 1e-5 * np.abs(ov) + 1e-30)


def test_left_needs_a_transpose(spv):
    A = synth.rmat(10, 4, seed=1)
    M = spv.Matrix.from_csc(A)
    S, xv = synth.sparse_x(A.m, 50, seed=2)
    with pytest.raises(spv.SpmspvError) as e:
        M.spmspv(dev(S), dev(xv), flags=spv.LEFT)
    assert e.value.status == spv.EUNSUPPORTED
    Mt = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE)
    with pytest.raises(spv.SpmspvError) as e:
        Mt.spmspv(dev(np.array([A.m], np.int32)), dev(np.ones(1, np.float32)), flags=spv.LEFT | spv.VALIDATE)
    assert e.value.status == spv.EINVAL
    with pytest.raises(spv.SpmspvError) as e:           # the selector is for the right multiply
        Mt.spmspv(dev(S), dev(xv), flags=spv.LEFT | spv.USE_SELECTOR)
    assert e.value.status == spv.EINVAL
    # the handle still serves right multiplies and BFS afterwards
    gi, gv, _ = Mt.spmspv(dev(S), dev(xv), sorted_output=True)
    oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
    compare(0, gi, gv, oi, ov, sorted_output=True)
    M.close()
    Mt.close()


# --------------------------------------------------------------------- DCSC

@pytest.fixture(scope="module")
def hyper(spv):
    A0 = synth.rmat(16, 8, seed=41)
    A = synth.column_subset(A0, np.random.default_rng(42).random(A0.n) < 1 / 16)
    D = synth.csc_to_dcsc(A)
    M = spv.Matrix.from_dcsc(D, flags=spv.VALIDATE)
    yield A, D, M
    M.close()


@pytest.mark.parametrize("semiring", [0, 1, 2])
def test_dcsc_hypersparse(spv, hyper, semiring):
    A, D, M = hyper
    assert D.nzc < A.n // 10
    rng = np.random.default_rng(100 + semiring)
    present = D.jc
    for f in (1, 100, A.n // 50, A.n // 2, A.n):
        S = synth.distinct_indices(A.n, f, seed=int(rng.integers(1 << 30)))
        xv = xvals(rng, semiring, f)
        gi, gv, nnz = M.spmspv(dev(S), dev(xv), semiring=semiring, sorted_output=True)
        oi, ov, W = oracle.spmspv_dcsc(D, S, xv, semiring)
        assert nnz == oi.size
        compare(semiring, gi, gv, oi, ov, sorted_output=True)
        assert M.last_stats()["W"] == W
    # only stored columns; only absent ones
    S = present[:: max(1, present.size // 500)].copy()
    xv = xvals(rng, semiring, S.size)
    gi, gv, _ = M.spmspv(dev(S), dev(xv), semiring=semiring, sorted_output=True)
    oi, ov, _ = oracle.spmspv_dcsc(D, S, xv, semiring)
    compare(semiring, gi, gv, oi, ov, sorted_output=True)
    absent = np.setdiff1d(np.arange(A.n, dtype=np.int32), present)[:2000]
    gi, gv, nnz = M.spmspv(dev(absent), dev(xvals(rng, semiring, absent.size)), semiring=semiring)
    assert nnz == 0 and M.last_stats()["W"] == 0


def test_dcsc_equals_csc_handle(spv):
    """An ordinary R-MAT (few empty columns): the DCSC handle and the CSC
    handle give the same index sets and int32 values, fp32 both within the
    oracle's bound."""
    A = synth.rmat(15, 16, seed=7)
    D = synth.csc_to_dcsc(A)
    Md = spv.Matrix.from_dcsc(D)
    Mc = spv.Matrix.from_csc(A)
    S, xv = synth.sparse_x(A.n, A.n // 100, seed=8)
    for semiring, v, fl in ((0, xv, 0), (1, None, spv.X_VAL_IS_INDEX)):
        gd = Md.spmspv(dev(S), None if v is None else dev(v), semiring=semiring, sorted_output=True, flags=fl)
        gc = Mc.spmspv(dev(S), None if v is None else dev(v), semiring=semiring, sorted_output=True, flags=fl)
        assert np.array_equal(to_np(gd[0]), to_np(gc[0]))
        oi, ov, _ = oracle.spmspv_dcsc(D, S, xv if semiring == 0 else S.astype(np.int32), semiring)
        compare(semiring, gd[0], gd[1], oi, ov, sorted_output=True)
    Md.close()
    Mc.close()


def test_dcsc_batch_bfs_graphblas(spv):
    # the subgraph induced by 30 % of the vertices of a symmetric R-MAT, in
    # the full id range: the other ids are empty columns (and empty rows)
    A0 = synth.rmat(14, 8, seed=51, symmetrize=True)
    keep = np.random.default_rng(52).random(A0.n) < 0.3
    C = A0.to_scipy().tocoo()
    k = keep[C.row] & keep[C.col]
    colptr, rowids = synth.coo_to_csc(A0.n, A0.n, C.row[k].astype(np.int32), C.col[k].astype(np.int32),
                                      drop_self=False)
    big = synth.CSC(A0.n, A0.n, colptr, rowids, synth.values(rowids.size, 5))
    D = synth.csc_to_dcsc(big)
    assert 0 < D.nzc <= int(keep.sum())
    M = spv.Matrix.from_dcsc(D)
    # batched calls
    xs = [synth.sparse_x(A0.n, f, seed=60 + k, tag=k) for k, f in enumerate((10, 0, 3000, 800, A0.n // 2))]
    off = np.zeros(len(xs) + 1, np.int64)
    off[1:] = np.cumsum([x[0].size for x in xs])
    idx = np.concatenate([x[0] for x in xs]).astype(np.int32)
    val = np.concatenate([x[1] for x in xs]).astype(np.float32)
    M.attach_batch(8, max_f=int(off[-1]), max_products=big.nnz * 8)
    y_off, y_idx, y_val, total = M.spmspv_batch(dev(off), dev(idx), dev(val))
    yo = to_np(y_off)
    for b, (S, xv) in enumerate(xs):
        oi, ov, _ = oracle.spmspv_dcsc(D, S, xv, 0)
        compare(0, y_idx[yo[b]:yo[b + 1]], y_val[yo[b]:yo[b + 1]], oi, ov, sorted_output=True)
    # BFS from a stored vertex (bucketing levels) against the CSC oracle
    P = spv.Matrix.from_dcsc(D, pattern=True)
    root = int(D.jc[D.jc.size // 2])
    lev, par, nl = P.bfs(root, spv.MIN_SELECT2ND_I32)
    olev, opar, onl = oracle.bfs(big, root)
    assert nl == onl and np.array_equal(to_np(lev), olev) and np.array_equal(to_np(par), opar)
    # GraphBLAS rules on the DCSC handle
    rng = np.random.default_rng(3)
    S, xv = xs[2]
    mi = rng.permutation(A0.n)[: A0.n // 3].astype(np.int32)
    wi = np.sort(rng.permutation(A0.n)[: A0.n // 10]).astype(np.int32)
    wv = rng.integers(0, 100, wi.size).astype(np.int32)
    y = torch.empty(A0.n, dtype=torch.int32, device="cuda")
    yv = torch.empty(A0.n, dtype=torch.int32, device="cuda")
    k = spv.spmspv_run_graphblas(M.handle, 1, spv.X_VAL_IS_INDEX, S.size, dev(S), None, dev(mi), None, mi.size, 0,
                                 spv.ACCUM_ADD, dev(wi), dev(wv), wi.size, y, yv, A0.n)
    oi, ov = oracle.spmspv_graphblas(big, S, S.astype(np.int32), 1, mask_idx=mi, w_idx=wi, w_val=wv,
                                     accum=oracle.ACCUM_ADD)
    assert np.array_equal(to_np(y[:k]), oi) and np.array_equal(to_np(yv[:k]), ov)
    # what a DCSC handle refuses
    with pytest.raises(spv.SpmspvError) as e:
        P.connected_components()
    assert e.value.status == spv.EUNSUPPORTED
    with pytest.raises(spv.SpmspvError) as e:
        P.bfs(root, spv.MIN_SELECT2ND_I32, flags=spv.PERSISTENT)
    assert e.value.status == spv.EUNSUPPORTED
    M.close()
    P.close()


def test_dcsc_invalid_and_empty(spv):
    A = synth.rmat(10, 4, seed=3)
    D = synth.csc_to_dcsc(A)
    bad = synth.DCSC(D.m, D.n, D.jc[::-1].copy(), D.cp, D.rowids, D.values)   # ids not ascending
    for fl in (spv.VALIDATE, 0):
        with pytest.raises(spv.SpmspvError) as e:
            spv.Matrix.from_dcsc(bad, flags=fl)
        assert e.value.status == spv.EINVAL
    out = synth.DCSC(D.m, D.n, np.r_[D.jc[:-1], D.n].astype(np.int32), D.cp, D.rowids, D.values)   # id == n
    with pytest.raises(spv.SpmspvError):
        spv.Matrix.from_dcsc(out)
    E = synth.DCSC(500, 700, np.zeros(0, np.int32), np.zeros(1, np.int32), np.zeros(0, np.int32), None)
    M = spv.Matrix.from_dcsc(E)
    S, xv = synth.sparse_x(700, 300, seed=1)
    _, _, nnz = M.spmspv(dev(S), dev(xv))
    assert nnz == 0
    M.close()


def test_dcsc_full_size_rmat22(spv):
    """The benchmark's scale-22 graph (43 % of its vertices isolated: their
    columns are absent from the DCSC form) at 1 % density."""
    A = synth.rmat(22, 16, seed=1, symmetrize=True)
    D = synth.csc_to_dcsc(A)
    M = spv.Matrix.from_dcsc(D)
    S, xv = synth.sparse_x(A.n, synth.density_f(A.n, 0.01), seed=2)
    gi, gv, nnz = M.spmspv(dev(S), dev(xv), sorted_output=True)
    oi, ov, _ = oracle.spmspv_dcsc(D, S, xv, 0)
    compare(0, gi, gv, oi, ov, sorted_output=True)
    M.close()


# ---------------------------------------------------------------- bitvector

def run_bv(spv, M, semiring, bits, vals, length_y, flags=0, cap=None):
    fl = flags
    xv = None
    if semiring == 1 and vals is None:
        fl |= spv.X_VAL_IS_INDEX
    elif semiring == 2 and vals is None:
        fl |= spv.X_ALL_TRUE
    else:
        xv = dev(vals) if vals.size else torch.zeros(1, dtype=torch.float32, device="cuda")
    yb, yv, nnz = M.spmspv_bitvector(dev(bits.view(np.int32)), xv, semiring=semiring, flags=fl, y_capacity=cap)
    return to_np(yb).view(np.uint32)[: (length_y + 31) // 32], to_np(yv), nnz


@pytest.mark.parametrize("semiring", [0, 1, 2])
def test_bitvector_against_oracle(spv, semiring):
    A = synth.rmat(14, 16, seed=61, symmetrize=True)
    M = spv.Matrix.from_csc(A)
    rng = np.random.default_rng(semiring)
    for f in (0, 1, A.n // 100, A.n // 2, A.n):
        S = np.sort(synth.distinct_indices(A.n, f, seed=int(rng.integers(1 << 30))))
        xv = xvals(rng, semiring, f)
        bits, _ = oracle.to_bitvector(S, None, A.n)
        gb, gv, nnz = run_bv(spv, M, semiring, bits, xv, A.m)
        oi, ov, _ = oracle.spmspv(A, S, xv, semiring, sorted_output=True)
        ob, _ = oracle.to_bitvector(oi, None, A.m)
        assert nnz == oi.size and np.array_equal(gb, ob)
        compare(semiring, torch.as_tensor(oi), torch.as_tensor(gv[:nnz]), oi, ov, sorted_output=True)
    # values of min-select2nd taken from the indices, or-and all true
    if semiring:
        S = np.sort(synth.distinct_indices(A.n, 700, seed=9))
        bits, _ = oracle.to_bitvector(S, None, A.n)
        gb, gv, nnz = run_bv(spv, M, semiring, bits, None, A.m)
        ox = S.astype(np.int32) if semiring == 1 else np.ones(S.size, np.uint8)
        oi, ov, _ = oracle.spmspv(A, S, ox, semiring, sorted_output=True)
        assert np.array_equal(gb, oracle.to_bitvector(oi, None, A.m)[0])
        assert np.array_equal(gv[:nnz].astype(np.int64), ov.astype(np.int64))
    M.close()


def test_bitvector_ragged_left_dcsc_and_errors(spv):
    # lengths that are not multiples of 32, left multiplication on a rectangular A
    A = rect(1000 * 32 + 7, 700 * 32 + 19, 200000, 77)
    M = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE)
    rng = np.random.default_rng(4)
    S = np.sort(synth.distinct_indices(A.m, 3000, seed=5))
    S[-1] = A.m - 1
    S = np.unique(S)
    xv = xvals(rng, 0, S.size)
    bits, _ = oracle.to_bitvector(S, None, A.m)
    gb, gv, nnz = run_bv(spv, M, 0, bits, xv, A.n, flags=spv.LEFT)
    oi, ov = oracle.spmspv_left(A, S, xv, 0)
    assert np.array_equal(gb, oracle.to_bitvector(oi, None, A.n)[0])
    compare(0, torch.as_tensor(oi), torch.as_tensor(gv[:nnz]), oi, ov, sorted_output=True)
    # right multiply on the same handle
    S2 = np.sort(synth.distinct_indices(A.n, 2000, seed=6))
    xv2 = xvals(rng, 0, S2.size)
    gb, gv, nnz = run_bv(spv, M, 0, oracle.to_bitvector(S2, None, A.n)[0], xv2, A.m)
    oi, ov, _ = oracle.spmspv(A, S2, xv2, 0, sorted_output=True)
    assert np.array_equal(gb, oracle.to_bitvector(oi, None, A.m)[0])
    # a bit past the length is reported; a short capacity is reported
    stray = oracle.to_bitvector(S2, None, A.n)[0]
    stray[-1] |= np.uint32(1 << 31)
    with pytest.raises(spv.SpmspvError) as e:
        run_bv(spv, M, 0, stray, xv2, A.m)
    assert e.value.status == spv.EDEVICE
    with pytest.raises(spv.SpmspvError) as e:
        run_bv(spv, M, 0, oracle.to_bitvector(S2, None, A.n)[0], xv2, A.m, cap=oi.size - 1)
    assert e.value.status == spv.ECAPACITY
    # with too small a capacity the bitmap still holds every row of y and the
    # values the first capacity rows
    cap = oi.size // 2
    y_bits = torch.full(((A.m + 31) // 32,), -1, dtype=torch.int32, device="cuda")
    y_val = torch.empty(cap, dtype=torch.float32, device="cuda")
    xb = dev(oracle.to_bitvector(S2, None, A.n)[0].view(np.int32))
    spv.spmspv_run_bitvector(M.handle, 0, 0, xb, dev(xv2), y_bits, y_val, cap, sync=False)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(y_bits).view(np.uint32), oracle.to_bitvector(oi, None, A.m)[0])
    compare(0, torch.as_tensor(oi[:cap]), y_val, oi[:cap], ov[:cap], sorted_output=True)
    gb, gv, nnz = run_bv(spv, M, 0, oracle.to_bitvector(S2, None, A.n)[0], xv2, A.m, cap=oi.size)
    assert nnz == oi.size and np.array_equal(gb, oracle.to_bitvector(oi, None, A.m)[0])
    M.close()
    # DCSC handle
    A0 = synth.rmat(13, 8, seed=81)
    H = synth.column_subset(A0, np.random.default_rng(82).random(A0.n) < 0.1)
    D = synth.csc_to_dcsc(H)
    Md = spv.Matrix.from_dcsc(D)
    S = np.sort(synth.distinct_indices(H.n, H.n // 3, seed=83))
    xv = xvals(rng, 1, S.size)
    gb, gv, nnz = run_bv(spv, Md, 1, oracle.to_bitvector(S, None, H.n)[0], xv, H.m)
    oi, ov, _ = oracle.spmspv_dcsc(D, S, xv, 1)
    assert np.array_equal(gb, oracle.to_bitvector(oi, None, H.m)[0])
    assert np.array_equal(gv[:nnz], ov)
    Md.close()


def test_bitvector_full_size_matches_list_call(spv):
    """R-MAT scale 22, 1 % density: the bitvector call's y equals the list
    call's y (same kernels after the conversion) and the oracle's."""
    A = synth.rmat(22, 16, seed=1, symmetrize=True)
    M = spv.Matrix.from_csc(A)
    S, xv = synth.sparse_x(A.n, synth.density_f(A.n, 0.01), seed=3, sort=True)
    bits, _ = oracle.to_bitvector(S, None, A.n)
    gb, gv, nnz = run_bv(spv, M, 0, bits, xv, A.m)
    oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
    assert np.array_equal(oracle.from_bitvector(gb, A.m), oi)
    compare(0, torch.as_tensor(oi), torch.as_tensor(gv[:nnz]), oi, ov, sorted_output=True)
    M.close()
