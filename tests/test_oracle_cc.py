"""Pins for the oracle's connected components (oracle_cc: label(v) = the
smallest vertex that reaches v; for a symmetric A the smallest vertex of
v's component), the second data-driven SpMSpV workload (the paper's
introduction lists connected components among SpMSpV's uses).

* scipy.sparse.csgraph.connected_components on symmetric R-MAT graphs (weak
  and strong components coincide there): same partition, and every label
  is its component's smallest vertex.
* Boolean transitive closure by repeated squaring on small directed
  graphs: label(v) = min{u : u reaches v}.
* Closed forms: a connected grid (every label 0), disjoint cliques, and
  directed paths in both orientations.
* Planted mistakes in copies of the oracle, each caught by these pins.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle
import synth

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")


@pytest.fixture(scope="module", autouse=True)
def _built():
    synth.build(force=False)
    oracle.build(force=False)


def csc(n, rows, cols):
    colptr, rowids = synth.coo_to_csc(n, n, np.asarray(rows, np.int32), np.asarray(cols, np.int32), drop_self=False)
    return synth.CSC(n, n, colptr, rowids, None)


def check_symmetric(A, lib=None):
    lab, k = oracle.cc(A, lib=lib)
    M = sp.csc_matrix((np.ones(A.nnz), A.rowids, A.colptr), shape=(A.n, A.n))
    kk, comp = connected_components(M, directed=False)
    if k != kk:
        return False
    # same partition, labelled by each component's smallest vertex
    smallest = np.full(kk, A.n)
    np.minimum.at(smallest, comp, np.arange(A.n))
    return np.array_equal(lab, smallest[comp])


def check_directed(A, lib=None):
    lab, _ = oracle.cc(A, lib=lib)
    n = A.n
    R = np.eye(n, dtype=bool)          # R[u, v]: u reaches v
    for j in range(n):
        R[j, A.rowids[A.colptr[j]:A.colptr[j + 1]]] = True
    for _ in range(int(np.ceil(np.log2(max(n, 2)))) + 1):
        R = R | ((R.astype(np.int32) @ R.astype(np.int32)) > 0)
    want = np.array([np.nonzero(R[:, v])[0].min() for v in range(n)], np.int32)
    return np.array_equal(lab, want)


@pytest.mark.parametrize("scale,ef,seed", [(10, 2, 1), (12, 1, 2), (14, 4, 3), (9, 16, 4)])
def test_symmetric_rmat_against_scipy(scale, ef, seed):
    A = synth.rmat(scale, ef, seed=seed, symmetrize=True, with_values=False)
    assert check_symmetric(A)


@pytest.mark.parametrize("seed", range(8))
def test_directed_against_transitive_closure(seed):
    rng = np.random.default_rng(seed)
    n = 40
    k = int(rng.integers(10, 90))
    A = csc(n, rng.integers(0, n, k), rng.integers(0, n, k))
    assert check_directed(A)


def test_closed_forms():
    lab, k = oracle.cc(synth.grid(30, 20, 3))
    assert k == 1 and not lab.any()
    # disjoint cliques of sizes 1..6 laid out consecutively
    rows, cols, start = [], [], 0
    for s in range(1, 7):
        for a in range(start, start + s):
            for b in range(start, start + s):
                if a != b:
                    rows.append(a)
                    cols.append(b)
        start += s
    lab, k = oracle.cc(csc(start, rows, cols))
    assert k == 6
    assert np.array_equal(lab, np.repeat(np.cumsum([0, 1, 2, 3, 4, 5]), np.arange(1, 7)))
    # directed path 0 -> 1 -> ... -> n-1 (A(i+1, i) stored): everything is reached from 0
    n = 50
    lab, k = oracle.cc(csc(n, np.arange(1, n), np.arange(n - 1)))
    assert k == 1 and not lab.any()
    # reversed path n-1 -> ... -> 0: each vertex is reached only from itself and larger ones
    lab, k = oracle.cc(csc(n, np.arange(n - 1), np.arange(1, n)))
    assert np.array_equal(lab, np.arange(n)) and k == n


MUTANTS = {
    "largest_first": ("for (int64_t u = 0; u < n; ++u) {\n        if (label[u] >= 0) continue;",
                      "for (int64_t u = n - 1; u >= 0; --u) {\n        if (label[u] >= 0) continue;"),
    "label_with_parent": ("label[i] = (int32_t)u;\n                    queue[tail++] = i;",
                          "label[i] = j;\n                    queue[tail++] = i;"),
    "one_hop_only": ("queue[tail++] = i;\n                }", "}"),
    "column_off_by_one": ("for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {\n                const int32_t i = rowids[q];\n                if (label[i] < 0) {",
                          "for (int64_t q = colptr[j] + 1; q < colptr[j + 1]; ++q) {\n                const int32_t i = rowids[q];\n                if (label[i] < 0) {"),
}


def pins(lib):
    ok = check_symmetric(synth.rmat(10, 2, seed=1, symmetrize=True, with_values=False), lib)
    rng = np.random.default_rng(5)
    for _ in range(3):
        n, k = 30, int(rng.integers(20, 60))
        ok = ok and check_directed(csc(n, rng.integers(0, n, k), rng.integers(0, n, k)), lib)
    return ok


def test_pins_pass_on_the_oracle():
    assert pins(oracle.load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"oracle_{name}.c"
    path.write_text(src.replace(old, new))
    lib = oracle.load(oracle.build(src=str(path), out=str(tmp_path / f"liboracle_{name}.so")))
    assert not pins(lib), f"planted mistake {name} passed the pins"
