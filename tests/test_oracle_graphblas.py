"""Pins for the oracle's masked multiply with accumulate / replace
(oracle_spmspv_graphblas: w<mask, replace> = w accum (A x), the masked
SpMSpV the paper's conclusions leave as future work, with the GraphBLAS
standard's rules).

* Dense brute force on tiny random inputs for every combination of mask
  kind (none, structural, value), complement, accumulate operator and
  replace, in all three semirings.
* Identities that reduce it to routes pinned elsewhere: no mask and no w is
  the plain product; the complement of a structural mask with no w is the
  visited-mask product a BFS level computes; w = A x accumulated with Add
  doubles the scipy product (plus-times) or leaves it unchanged (min, or);
  an empty mask, a value mask of zeros and the complement of no mask give
  w (or nothing, with replace).
* Planted mistakes in copies of the oracle, each caught by these pins.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st

import oracle
import synth

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
PT, MS, OA = oracle.PLUS_TIMES, oracle.MIN_SELECT2ND, oracle.OR_AND
NONE, ADD, FIRST, SECOND = oracle.ACCUM_NONE, oracle.ACCUM_ADD, oracle.ACCUM_FIRST, oracle.ACCUM_SECOND


@pytest.fixture(scope="module", autouse=True)
def _built():
    synth.build(force=False)
    oracle.build(force=False)


def tiny(rng, m=14, n=11, density=0.3):
    P = rng.random((m, n)) < density
    colptr = np.r_[0, np.cumsum(P.sum(0))].astype(np.int32)
    rowids = np.concatenate([np.nonzero(P[:, j])[0] for j in range(n)]).astype(np.int32)
    vals = ((rng.integers(0, 1 << 24, rowids.size) + 1) / float(1 << 24)).astype(np.float32)
    return synth.CSC(m, n, colptr, rowids, vals), P


def inputs(rng, A, semiring):
    S = rng.permutation(A.n)[: rng.integers(0, A.n + 1)].astype(np.int32)
    wi = rng.permutation(A.m)[: rng.integers(0, A.m + 1)].astype(np.int32)
    if semiring == PT:
        xv = ((rng.integers(0, 1 << 24, S.size) + 1) / float(1 << 24)).astype(np.float32)
        wv = rng.random(wi.size)
    elif semiring == MS:
        xv = rng.integers(-40, 40, S.size).astype(np.int32)
        wv = rng.integers(-40, 40, wi.size).astype(np.int32)
    else:
        xv = (rng.random(S.size) < 0.6).astype(np.uint8)
        wv = (rng.random(wi.size) < 0.5).astype(np.uint8)
    return S, xv, wi, wv


def brute(A, P, S, xv, semiring, mi, mv, complement, wi, wv, accum, replace):
    """The GraphBLAS rules over dense arrays."""
    m = A.m
    D = np.zeros(P.shape)
    for j in range(A.n):
        D[A.rowids[A.colptr[j]:A.colptr[j + 1]], j] = A.values[A.colptr[j]:A.colptr[j + 1]]
    Ps = P[:, S]
    tp = Ps.any(1)
    if semiring == PT:
        tv = D[:, S] @ xv.astype(np.float64)
    elif semiring == MS:
        tv = np.where(Ps, xv[None, :].astype(np.int64), 1 << 40).min(1) if S.size else np.zeros(m)
    else:
        tv = (Ps & (D[:, S] != 0) & (xv[None, :] != 0)).any(1)
    wp = np.zeros(m, bool)
    wp[wi] = True
    wd = np.zeros(m)
    wd[wi] = wv
    if mi is None:
        M = np.ones(m, bool)
    else:
        M = np.zeros(m, bool)
        M[mi] = True if mv is None else (mv != 0)
    if complement:
        M = ~M
    both = tp & wp & (accum != NONE)
    if accum == ADD:
        comb = wd + tv if semiring == PT else (np.minimum(wd, tv) if semiring == MS else ((wd != 0) | (tv != 0)))
    elif accum == FIRST:
        comb = wd
    else:
        comb = tv
    zp = tp | (wp & (accum != NONE))
    zv = np.where(both, comb, np.where(tp, tv, wd))
    out = np.where(M, zp, wp & (not replace))
    val = np.where(M, zv, wd)
    rows = np.nonzero(out)[0]
    return rows, val[rows].astype(np.float64)


def call(A, S, xv, semiring, mi, mv, complement, wi, wv, accum, replace, lib=None):
    yi, yv = oracle.spmspv_graphblas(A, S, xv, semiring, mask_idx=mi, mask_val=mv, complement=complement,
                                     w_idx=wi, w_val=wv, accum=accum, replace=replace, lib=lib)
    return yi, yv.astype(np.float64)


CASES = [(sr, mk, comp, acc, rep) for sr in (PT, MS, OA) for mk in ("none", "struct", "value")
         for comp in (False, True) for acc in (NONE, ADD, FIRST, SECOND) for rep in (False, True)]


@pytest.mark.parametrize("semiring,mask,complement,accum,replace", CASES)
def test_brute_force_every_combination(semiring, mask, complement, accum, replace):
    rng = np.random.default_rng(hash((semiring, mask, complement, accum, replace)) % (1 << 32))
    for _ in range(6):
        A, P = tiny(rng)
        S, xv, wi, wv = inputs(rng, A, semiring)
        mi = mv = None
        if mask != "none":
            mi = rng.permutation(A.m)[: rng.integers(0, A.m + 1)].astype(np.int32)
            if mask == "value":
                mv = (rng.random(mi.size) < 0.5).astype(np.uint8)
        yi, yv = call(A, S, xv, semiring, mi, mv, complement, wi, wv, accum, replace)
        ri, rv = brute(A, P, S, xv, semiring, mi, mv, complement, wi, wv, accum, replace)
        assert np.array_equal(yi, ri)
        assert np.all(np.diff(yi) > 0)
        if semiring == PT:
            assert np.allclose(yv, rv, rtol=1e-14, atol=0)
        else:
            assert np.array_equal(yv, rv)


@settings(max_examples=40, deadline=None)
@given(seed=st.integers(0, 2 ** 31), semiring=st.sampled_from([PT, MS, OA]))
def test_no_mask_no_w_is_the_plain_product(seed, semiring):
    rng = np.random.default_rng(seed)
    A, P = tiny(rng, 30, 25, 0.2)
    S, xv, _, _ = inputs(rng, A, semiring)
    for accum in (NONE, ADD, FIRST, SECOND):
        for replace in (False, True):
            yi, yv = call(A, S, xv, semiring, None, None, False, None, None, accum, replace)
            oi, ov, _ = oracle.spmspv(A, S, xv, semiring, sorted_output=True)
            assert np.array_equal(yi, oi) and np.array_equal(yv, ov.astype(np.float64))


@pytest.mark.parametrize("semiring", [PT, MS, OA])
def test_complement_of_visited_is_the_bfs_level_product(semiring):
    """The BFS level: rows outside the visited set (complement of a
    structural mask), nothing accumulated; equals the product with the
    visited rows dropped."""
    rng = np.random.default_rng(7 + semiring)
    A = synth.rmat(11, seed=3)
    S, xv, _, _ = inputs(rng, A, semiring)
    visited = rng.permutation(A.m)[: A.m // 3].astype(np.int32)
    drop = np.zeros(A.m, np.uint8)
    drop[visited] = 1
    for replace in (False, True):
        yi, yv = call(A, S, xv, semiring, visited, None, True, None, None, NONE, replace)
        oi, ov, _ = oracle.spmspv(A, S, xv, semiring, mask=drop, sorted_output=True)
        assert np.array_equal(yi, oi) and np.array_equal(yv, ov.astype(np.float64))


def test_accumulating_the_product_into_itself():
    """w = A x (from scipy) accumulated with Add over every row: 2 A x for
    plus-times; A x for min and or (idempotent Add)."""
    rng = np.random.default_rng(11)
    A = synth.rmat(10, seed=5)
    S, xv, _, _ = inputs(rng, A, PT)
    B = sp.csc_matrix((A.values.astype(np.float64), A.rowids, A.colptr), shape=(A.m, A.n))
    ref = np.asarray(B[:, S] @ xv.astype(np.float64)).ravel()
    pres = np.asarray((B[:, S] != 0).sum(1)).ravel() > 0
    rows = np.nonzero(pres)[0].astype(np.int32)
    yi, yv = call(A, S, xv, PT, None, None, False, rows, ref[rows], ADD, False)
    assert np.array_equal(yi, rows) and np.allclose(yv, 2 * ref[rows], rtol=1e-14, atol=0)
    for semiring in (MS, OA):
        _, xs, _, _ = inputs(rng, A, semiring)
        xs = xs[: S.size] if xs.size >= S.size else np.resize(xs, S.size)
        oi, ov, _ = oracle.spmspv(A, S, xs, semiring, sorted_output=True)
        yi, yv = call(A, S, xs, semiring, None, None, False, oi, ov, ADD, False)
        assert np.array_equal(yi, oi) and np.array_equal(yv, ov.astype(np.float64))


@pytest.mark.parametrize("semiring", [PT, MS, OA])
def test_masks_that_select_nothing(semiring):
    """An empty mask, a value mask whose values are all zero and the
    complement of no mask select no row: the result is w, or nothing with
    replace, whatever x and the accumulate operator."""
    rng = np.random.default_rng(13 + semiring)
    A, P = tiny(rng, 40, 30, 0.2)
    S, xv, wi, wv = inputs(rng, A, semiring)
    order = np.argsort(wi)
    for mi, mv, comp in ((np.zeros(0, np.int32), None, False),
                         (np.arange(A.m, dtype=np.int32), np.zeros(A.m, np.uint8), False),
                         (None, None, True)):
        for accum in (NONE, ADD, SECOND):
            yi, yv = call(A, S, xv, semiring, mi, mv, comp, wi, wv, accum, False)
            assert np.array_equal(yi, wi[order]) and np.array_equal(yv, np.asarray(wv, np.float64)[order])
            yi, yv = call(A, S, xv, semiring, mi, mv, comp, wi, wv, accum, True)
            assert yi.size == 0


def test_first_and_second_where_both_are_present():
    rng = np.random.default_rng(17)
    A, P = tiny(rng, 50, 40, 0.15)
    S, xv, wi, wv = inputs(rng, A, MS)
    oi, ov, _ = oracle.spmspv(A, S, xv, MS, sorted_output=True)
    t = dict(zip(oi.tolist(), ov.tolist()))
    w = dict(zip(wi.tolist(), wv.tolist()))
    for accum, pick in ((FIRST, w), (SECOND, t)):
        yi, yv = call(A, S, xv, MS, None, None, False, wi, wv, accum, False)
        got = dict(zip(yi.tolist(), yv.tolist()))
        assert sorted(got) == sorted(set(t) | set(w))
        for i in got:
            want = pick[i] if (i in t and i in w) else (t[i] if i in t else w[i])
            assert got[i] == want


# ------------------------------------------------------------ planted mistakes
MUTANTS = {
    "complement_ignored": ("    if (complement)\n        for (int64_t i = 0; i < m; ++i) in_mask[i] = (unsigned char)!in_mask[i];",
                           ""),
    "replace_ignored": ("} else if (!replace && w_has[i]) {", "} else if (w_has[i]) {"),
    "first_second_swapped": ("if (accum == 2) { zd = wd[i]; zi = wi[i]; }", "if (accum == 2) { zd = td[i]; zi = ti[i]; }"),
    "value_mask_as_structure": ("if (!mask_val || mask_val[r] != 0) in_mask[i] = 1;", "in_mask[i] = 1;"),
    "w_kept_without_accum": ("} else if (w_has[i] && accum != 0) {", "} else if (w_has[i]) {"),
    "min_accum_becomes_max": ("zi = wi[i] < ti[i] ? wi[i] : ti[i];", "zi = wi[i] > ti[i] ? wi[i] : ti[i];"),
    "plus_accum_drops_w": ("else if (semiring == OR_PLUS_TIMES) zd = wd[i] + td[i];",
                           "else if (semiring == OR_PLUS_TIMES) zd = td[i];"),
}


def gb_pin_suite(lib):
    """The brute-force comparison over every combination (one input each);
    returns True when every case matches."""
    rng = np.random.default_rng(99)
    for sr, mk, comp, acc, rep in CASES:
        for _ in range(2):
            A, P = tiny(rng)
            S, xv, wi, wv = inputs(rng, A, sr)
            mi = mv = None
            if mk != "none":
                mi = rng.permutation(A.m)[: rng.integers(1, A.m + 1)].astype(np.int32)
                if mk == "value":
                    mv = (rng.random(mi.size) < 0.5).astype(np.uint8)
            yi, yv = call(A, S, xv, sr, mi, mv, comp, wi, wv, acc, rep, lib=lib)
            ri, rv = brute(A, P, S, xv, sr, mi, mv, comp, wi, wv, acc, rep)
            if not (np.array_equal(yi, ri) and np.allclose(yv, rv, rtol=1e-14, atol=0)):
                return False
    return True


def test_pins_pass_on_the_oracle():
    assert gb_pin_suite(oracle.load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"oracle_{name}.c"
    path.write_text(src.replace(old, new))
    lib = oracle.load(oracle.build(src=str(path), out=str(tmp_path / f"liboracle_{name}.so")))
    assert not gb_pin_suite(lib), f"planted mistake {name} passed the pins"
