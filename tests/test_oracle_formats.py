"""Pins for the oracle's format variants (Background: Notation, and Sparse
matrix and vector data structures): left multiplication y' = x' A
(oracle_spmspv_left), y = A x with A in DCSC (oracle_spmspv_dcsc) and the
bitvector form of sparse vectors (oracle.to_bitvector / from_bitvector).

* Left multiplication against scipy's A^T x (plus-times values and the
  structural pattern), against dense brute force on tiny inputs for all
  three semirings, and against the right-multiply oracle on the explicit
  transpose that scipy builds.
* DCSC against the CSC oracle on the same matrix (empty columns selected,
  first and last columns, hypersparse matrices), against dense brute force,
  and a closed form with two non-empty columns.
* Bitvector: a hand-computed word layout, round trips, and a bit set past
  the vector's length refused.
* Planted mistakes in copies of the oracle, each caught by these pins.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
PT, MS, OA = oracle.PLUS_TIMES, oracle.MIN_SELECT2ND, oracle.OR_AND


@pytest.fixture(scope="module", autouse=True)
def _built():
    synth.build(force=False)
    oracle.build(force=False)


def tiny(rng, m, n, density, zero_frac=0.0):
    P = rng.random((m, n)) < density
    colptr = np.r_[0, np.cumsum(P.sum(0))].astype(np.int32)
    rowids = np.concatenate([np.nonzero(P[:, j])[0] for j in range(n)] + [np.zeros(0, np.int64)]).astype(np.int32)
    vals = ((rng.integers(0, 1 << 24, rowids.size) + 1) / float(1 << 24)).astype(np.float32)
    vals[rng.random(rowids.size) < zero_frac] = 0.0
    return synth.CSC(m, n, colptr, rowids, vals)


def dense(A):
    D = np.zeros((A.m, A.n))
    P = np.zeros((A.m, A.n), bool)
    for j in range(A.n):
        r = A.rowids[A.colptr[j]:A.colptr[j + 1]]
        D[r, j] = 1.0 if A.values is None else A.values[A.colptr[j]:A.colptr[j + 1]]
        P[r, j] = True
    return D, P


def xvals(rng, semiring, k):
    if semiring == PT:
        return ((rng.integers(0, 1 << 24, k) + 1) / float(1 << 24)).astype(np.float32)
    if semiring == MS:
        return rng.integers(-50, 50, k).astype(np.int32)
    return (rng.random(k) < 0.6).astype(np.uint8)


def brute_left(A, S, xv, semiring):
    """y'(j) over dense arrays: j present when a stored A(i, j) has i in S."""
    D, P = dense(A)
    Ps = P[S, :]                      # rows of x', all columns
    idx = np.nonzero(Ps.any(0))[0]
    if semiring == PT:
        val = (xv.astype(np.float64) @ D[S, :])[idx]
    elif semiring == MS:
        val = np.array([xv[Ps[:, j]].min() for j in idx], np.int64)
    else:
        val = np.array([bool(((D[S, j] != 0) & (xv != 0) & Ps[:, j]).any()) for j in idx], np.int64)
    return idx, val


def brute_right(A, S, xv, semiring):
    D, P = dense(A)
    Ps = P[:, S]
    idx = np.nonzero(Ps.any(1))[0]
    if semiring == PT:
        val = (D[:, S] @ xv.astype(np.float64))[idx]
    elif semiring == MS:
        val = np.array([xv[Ps[i, :]].min() for i in idx], np.int64)
    else:
        val = np.array([bool(((D[i, S] != 0) & (xv != 0) & Ps[i, :]).any()) for i in idx], np.int64)
    return idx, val


def same(gi, gv, oi, ov, semiring):
    if not np.array_equal(np.asarray(gi, np.int64), np.asarray(oi, np.int64)):
        return False
    if semiring == PT:
        return np.allclose(np.asarray(gv, np.float64), np.asarray(ov, np.float64), rtol=1e-12, atol=0)
    return np.array_equal(np.asarray(gv, np.int64), np.asarray(ov, np.int64))


# ------------------------------------------------------------ left multiply

def left_pins(lib=None):
    rng = np.random.default_rng(11)
    for t in range(24):
        m, n = int(rng.integers(1, 12)), int(rng.integers(1, 12))
        A = tiny(rng, m, n, float(rng.uniform(0.1, 0.6)), zero_frac=0.3)
        S = rng.permutation(m)[: int(rng.integers(0, m + 1))].astype(np.int32)
        for semiring in (PT, MS, OA):
            xv = xvals(rng, semiring, S.size)
            gi, gv = oracle.spmspv_left(A, S, xv, semiring, lib=lib)
            bi, bv = brute_left(A, S, xv, semiring)
            if not same(gi, gv, bi, bv, semiring):
                return False
    return True


def test_left_brute_force():
    assert left_pins()


@pytest.mark.parametrize("scale,ef,seed", [(10, 4, 1), (12, 2, 2)])
def test_left_against_scipy_transpose_product(scale, ef, seed):
    A = synth.rmat(scale, ef, seed=seed)
    S, xv = synth.sparse_x(A.m, A.m // 20, seed=seed + 7)
    gi, gv = oracle.spmspv_left(A, S, xv, PT)
    M = A.to_scipy()
    x = np.zeros(A.m)
    x[S] = xv
    yd = M.T @ x
    pat = (abs(M).T.astype(bool).astype(np.int64) @ (x != 0).astype(np.int64)) > 0
    assert np.array_equal(gi, np.nonzero(pat)[0])
    assert np.allclose(gv, yd[gi], rtol=1e-12, atol=0)


@pytest.mark.parametrize("semiring", [PT, MS, OA])
def test_left_is_right_multiply_by_the_transpose(semiring):
    """Rectangular A (m != n): y' = x' A equals oracle_spmspv on A^T, which
    scipy builds."""
    rng = np.random.default_rng(5 + semiring)
    m, n = 3000, 1700
    rows = rng.integers(0, m, 20000).astype(np.int32)
    cols = rng.integers(0, n, 20000).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(m, n, rows, cols, drop_self=False)
    A = synth.CSC(m, n, colptr, rowids, synth.values(rowids.size, 3))
    T = A.to_scipy().T.tocsc()
    T.sort_indices()
    At = synth.CSC(n, m, T.indptr.astype(np.int32), T.indices.astype(np.int32), T.data.astype(np.float32))
    S = rng.permutation(m)[:400].astype(np.int32)
    xv = xvals(rng, semiring, S.size)
    gi, gv = oracle.spmspv_left(A, S, xv, semiring)
    oi, ov, _ = oracle.spmspv(At, S, xv, semiring, sorted_output=True)
    assert same(gi, gv, oi, ov, semiring)


def test_left_errors():
    A = tiny(np.random.default_rng(1), 5, 4, 0.5)
    with pytest.raises(ValueError):
        oracle.spmspv_left(A, np.array([5], np.int32), np.ones(1, np.float32))
    with pytest.raises(ValueError):
        oracle.spmspv_left(A, np.array([1, 1], np.int32), np.ones(2, np.float32))


# --------------------------------------------------------------------- DCSC

def dcsc_pins(lib=None):
    rng = np.random.default_rng(21)
    for t in range(24):
        m, n = int(rng.integers(1, 12)), int(rng.integers(1, 14))
        A = tiny(rng, m, n, float(rng.uniform(0.05, 0.4)), zero_frac=0.2)
        D = synth.csc_to_dcsc(A)
        S = rng.permutation(n)[: int(rng.integers(0, n + 1))].astype(np.int32)
        for semiring in (PT, MS, OA):
            xv = xvals(rng, semiring, S.size)
            gi, gv, W = oracle.spmspv_dcsc(D, S, xv, semiring, lib=lib)
            bi, bv = brute_right(A, S, xv, semiring)
            if not same(gi, gv, bi, bv, semiring) or W != int(np.diff(A.colptr)[S].sum()):
                return False
    # two non-empty columns (3 and 7) of a 6 x 10 matrix; x selects every column
    rows = np.array([0, 4, 5, 1, 4], np.int32)
    A = synth.CSC(6, 10, np.array([0, 0, 0, 0, 3, 3, 3, 3, 5, 5, 5], np.int32), rows,
                  np.array([0.5, 0.25, 1.0, 2.0, 0.125], np.float32))
    D = synth.csc_to_dcsc(A)
    if D.nzc != 2 or list(D.jc) != [3, 7]:
        return False
    xv = np.arange(1, 11, dtype=np.float32)
    gi, gv, W = oracle.spmspv_dcsc(D, np.arange(10, dtype=np.int32), xv, PT, lib=lib)
    want_i = [0, 1, 4, 5]
    want_v = [0.5 * 4, 2.0 * 8, 0.25 * 4 + 0.125 * 8, 1.0 * 4]
    if list(gi) != want_i or not np.allclose(gv, want_v, rtol=0, atol=0) or W != 5:
        return False
    # only empty columns selected
    gi, gv, W = oracle.spmspv_dcsc(D, np.array([0, 9, 4], np.int32), np.ones(3, np.float32), PT, lib=lib)
    return gi.size == 0 and W == 0


def test_dcsc_brute_force_and_closed_form():
    assert dcsc_pins()


@pytest.mark.parametrize("semiring", [PT, MS, OA])
def test_dcsc_matches_csc_oracle_hypersparse(semiring):
    """R-MAT scale 14 with all but ~1/16 of its columns emptied: x mixes
    present and absent columns, including the first and last ids."""
    A0 = synth.rmat(14, 8, seed=3)
    keep = np.random.default_rng(9).random(A0.n) < 1 / 16
    A = synth.column_subset(A0, keep)
    D = synth.csc_to_dcsc(A)
    assert D.nzc < A.n // 10 and D.nnz == A.nnz
    S = synth.distinct_indices(A.n - 2, 3000, seed=4) + 1
    S = np.concatenate([[0], S, [A.n - 1]]).astype(np.int32)
    rng = np.random.default_rng(semiring)
    xv = xvals(rng, semiring, S.size)
    gi, gv, W = oracle.spmspv_dcsc(D, S, xv, semiring)
    oi, ov, OW = oracle.spmspv(A, S, xv, semiring, sorted_output=True)
    assert W == OW
    assert same(gi, gv, oi, ov, semiring)


def test_csc_to_dcsc_format():
    A = synth.rmat(10, 2, seed=8)
    D = synth.csc_to_dcsc(A)
    lens = np.diff(A.colptr)
    assert np.array_equal(D.jc, np.nonzero(lens)[0])
    assert np.all(np.diff(D.jc) > 0) and np.all(np.diff(D.cp) > 0)
    assert np.array_equal(np.diff(D.cp), lens[lens > 0])
    with pytest.raises(ValueError):
        oracle.spmspv_dcsc(D, np.array([A.n], np.int32), np.ones(1, np.float32))


# ---------------------------------------------------------------- bitvector

def test_bitvector_hand_layout():
    bits, vals = oracle.to_bitvector(np.array([64, 0, 32, 5, 63, 31]), np.array([6, 1, 4, 2, 5, 3]), 70)
    assert bits.dtype == np.uint32 and list(bits) == [0x80000021, 0x80000001, 0x1]
    assert list(vals) == [1, 2, 3, 4, 5, 6]
    assert list(oracle.from_bitvector(bits, 70)) == [0, 5, 31, 32, 63, 64]
    bits, _ = oracle.to_bitvector(np.zeros(0, np.int32), None, 33)
    assert list(bits) == [0, 0] and oracle.from_bitvector(bits, 33).size == 0


def test_bitvector_round_trip():
    rng = np.random.default_rng(3)
    for length in (1, 31, 32, 33, 1000, 4099):
        idx = rng.permutation(length)[: int(rng.integers(0, length + 1))]
        val = rng.random(idx.size)
        bits, v = oracle.to_bitvector(idx, val, length)
        back = oracle.from_bitvector(bits, length)
        assert np.array_equal(back, np.sort(idx))
        assert np.array_equal(v, val[np.argsort(idx)])


def test_bitvector_bit_past_length_refused():
    with pytest.raises(ValueError):
        oracle.from_bitvector(np.array([1 << 5], np.uint32), 5)


# ---------------------------------------------------------- planted mistakes

MUTANTS = {
    "left_no_accumulation": ("left", "sd = hit ? sd + t : t;", "sd = hit ? sd : t;"),
    "left_min_as_max": ("left", "si = (!hit || xi[i] < si) ? xi[i] : si;", "si = (!hit || xi[i] > si) ? xi[i] : si;"),
    "left_skip_first_entry": ("left", "for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {\n            const int32_t i = rowids[q];\n            if (!has[i]) continue;",
                              "for (int64_t q = colptr[j] + 1; q < colptr[j + 1]; ++q) {\n            const int32_t i = rowids[q];\n            if (!has[i]) continue;"),
    "left_drops_false_entries": ("left", "        if (!hit) continue;\n        y_idx[count] = (int32_t)j;",
                                 "        if (!hit || (semiring == OR_OR_AND && si == 0)) continue;\n        y_idx[count] = (int32_t)j;"),
    "left_value_from_matrix": ("left", "si = (!hit || xi[i] < si) ? xi[i] : si;",
                               "si = (!hit || (int32_t)q < si) ? (int32_t)q : si;"),
    "dcsc_no_equality_check": ("dcsc", "if (lo == nzc || jc[lo] != j) continue;", "if (lo == nzc) continue;"),
    "dcsc_search_past_match": ("dcsc", "if (jc[mid] < j) lo = mid + 1;", "if (jc[mid] <= j) lo = mid + 1;"),
    "dcsc_drops_last_entry": ("dcsc", "for (int64_t q = cp[lo]; q < cp[lo + 1]; ++q) {",
                              "for (int64_t q = cp[lo]; q < cp[lo + 1] - 1; ++q) {"),
}


def test_pins_pass_on_the_oracle():
    lib = oracle.load()
    assert left_pins(lib) and dcsc_pins(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    which, old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"oracle_{name}.c"
    path.write_text(src.replace(old, new))
    lib = oracle.load(oracle.build(src=str(path), out=str(tmp_path / f"liboracle_{name}.so")))
    ok = left_pins(lib) if which == "left" else dcsc_pins(lib)
    assert not ok, f"planted mistake {name} passed the pins"
