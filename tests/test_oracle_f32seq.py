"""Pins for the oracle's sequential fp32 product (oracle_spmspv_f32seq), the
reference of the deterministic plus-times mode: every product is rounded to
fp32 (Mult), and each row's products are added one at a time in fp32 in
product order -- x order, then the column's storage order (Algorithm 1's Add
applied in the order the bucketing produces the products when nothing
reorders them).

* Brute force in numpy float32 arithmetic on small random matrices whose
  rows collect many products (where the order changes the rounding), with
  x in random order and with duplicate (i, j) entries.
* The order matters: on a row built so that the left-to-right fp32 sum and
  the right-to-left one differ, the oracle gives the left-to-right one.
* Planted mistakes in copies of the oracle (x taken in reverse order, the
  first product of each row dropped), each caught.
"""
import os

import numpy as np
import pytest

import oracle
import synth

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")


@pytest.fixture(scope="module", autouse=True)
def _built():
    synth.build(force=False)
    oracle.build(force=False)


def brute(A, S, xv):
    """Rows in first-touch order, values folded left to right in float32."""
    acc, order = {}, []
    for p, j in enumerate(S.tolist()):
        for q in range(int(A.colptr[j]), int(A.colptr[j + 1])):
            i = int(A.rowids[q])
            a = np.float32(1.0) if A.values is None else np.float32(A.values[q])
            t = np.float32(a * np.float32(xv[p]))
            if i in acc:
                acc[i] = np.float32(acc[i] + t)
            else:
                acc[i] = t
                order.append(i)
    return np.array(order, np.int64), np.array([acc[i] for i in order], np.float32)


def dense_rows(rng, m, n, density, dup=False):
    rows, cols = np.nonzero(rng.random((m, n)) < density)
    if dup:   # repeat a fifth of the entries: duplicate (i, j) pairs in their columns
        k = rng.random(rows.size) < 0.2
        rows, cols = np.r_[rows, rows[k]], np.r_[cols, cols[k]]
    order = np.argsort(cols, kind="stable")
    rows, cols = rows[order], cols[order]
    colptr = np.zeros(n + 1, np.int32)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr).astype(np.int32)
    # values spread over many binades so that the order of the adds matters
    vals = (rng.random(rows.size) * 2.0 ** rng.integers(-12, 12, rows.size)).astype(np.float32)
    return synth.CSC(m, n, colptr, rows.astype(np.int32), vals)


def pins(lib=None):
    rng = np.random.default_rng(2024)
    for t in range(30):
        m, n = int(rng.integers(1, 9)), int(rng.integers(1, 40))
        A = dense_rows(rng, m, n, float(rng.uniform(0.3, 0.9)), dup=bool(t % 3 == 0))
        S = rng.permutation(n)[: int(rng.integers(1, n + 1))].astype(np.int32)
        xv = (rng.random(S.size) * 2.0 ** rng.integers(-8, 8, S.size)).astype(np.float32)
        gi, gv = oracle.spmspv_f32seq(A, S, xv, lib=lib)
        bi, bv = brute(A, S, xv)
        if not (np.array_equal(gi, bi) and np.array_equal(gv.view(np.uint32), bv.view(np.uint32))):
            return False
    # one row, three products whose left-to-right and right-to-left sums differ:
    # 1 + 2^-24 + 2^-24 is 1 left to right, 1 + 2^-23 right to left
    A = synth.CSC(1, 3, np.array([0, 1, 2, 3], np.int32), np.zeros(3, np.int32),
                  np.array([1.0, 2.0 ** -24, 2.0 ** -24], np.float32))
    one = np.ones(3, np.float32)
    _, fwd = oracle.spmspv_f32seq(A, np.array([0, 1, 2], np.int32), one, lib=lib)
    _, rev = oracle.spmspv_f32seq(A, np.array([2, 1, 0], np.int32), one, lib=lib)
    return fwd[0] == np.float32(1.0) and rev[0] == np.float32(1.0 + 2.0 ** -23)


def test_sequential_fold_pins():
    assert pins()


MUTANTS = {
    "x_reversed": ("    for (int64_t p = 0; p < f; ++p) {\n        int32_t j = x_idx[p];\n"
                   "        for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {\n            int32_t i = rowids[q];\n"
                   "            volatile float t",
                   "    for (int64_t p = f - 1; p >= 0; --p) {\n        int32_t j = x_idx[p];\n"
                   "        for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {\n            int32_t i = rowids[q];\n"
                   "            volatile float t"),
    "first_product_dropped": ("if (!seen[i]) { seen[i] = 1; acc[i] = t; y_idx[count++] = i; }\n"
                              "            else { volatile float s",
                              "if (!seen[i]) { seen[i] = 1; acc[i] = 0.0f; y_idx[count++] = i; }\n"
                              "            else { volatile float s"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"oracle_{name}.c"
    path.write_text(src.replace(old, new))
    lib = oracle.load(oracle.build(src=str(path), out=str(tmp_path / f"liboracle_{name}.so")))
    assert not pins(lib), f"planted mistake {name} passed the pins"
