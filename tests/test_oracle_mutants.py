"""Plant plausible mistakes in copies of the oracle and check the pins catch each.

Every mutant is the oracle's C source with one edit (a dropped term, a wrong
comparison, an off-by-one bound, an inverted mask, a swapped operand), built
into a temporary library.  A compact version of the pin checks must fail on
every mutant while passing on the unmodified oracle.
"""
import os

import numpy as np
import pytest

import oracle
import synth

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "dropped_add_term": ("else acc_d[i] = acc_d[i] + t;", "else acc_d[i] = t;"),
    "dropped_x_factor": ("double t = a * (double)((const float*)x_val)[p];", "double t = a;"),
    "min_becomes_max": ("else if (t < acc_i[i]) acc_i[i] = t;", "else if (t > acc_i[i]) acc_i[i] = t;"),
    "column_off_by_one": ("for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {\n            int32_t i = rowids[q];\n            work++;",
                          "for (int64_t q = colptr[j]; q + 1 < colptr[j + 1]; ++q) {\n            int32_t i = rowids[q];\n            work++;"),
    "or_becomes_and": ("else acc_b[i] = (uint8_t)(acc_b[i] || t);", "else acc_b[i] = (uint8_t)(acc_b[i] && t);"),
    "mask_inverted": ("if (!mask[y_idx[r]]) y_idx[k++] = y_idx[r];", "if (mask[y_idx[r]]) y_idx[k++] = y_idx[r];"),
    "transposed_lookup": ("int32_t i = rowids[q];\n            work++;", "int32_t i = (int32_t)(j % m);\n            work++;"),
    "bfs_parent_max": ("(parent[v] < 0 || u < parent[v])", "(parent[v] < 0 || u > parent[v])"),
    "bfs_level_skip": ("level[v] = level[u] + 1;\n                if", "level[v] = level[u] + 2;\n                if"),
}


def pin_suite(lib) -> list:
    """Compact pin checks; returns the names of the checks that failed."""
    failed = []
    rng = np.random.default_rng(123)
    # brute force, three semirings
    m, n = 20, 16
    P = rng.random((m, n)) < 0.35
    colptr = np.r_[0, np.cumsum(P.sum(0))].astype(np.int32)
    rowids = np.concatenate([np.nonzero(P[:, j])[0] for j in range(n)]).astype(np.int32)
    vals = ((rng.integers(0, 1 << 24, rowids.size) + 1) / float(1 << 24)).astype(np.float32)
    A = synth.CSC(m, n, colptr, rowids, vals)
    D = np.zeros((m, n))
    for j in range(n):
        D[rowids[colptr[j]:colptr[j + 1]], j] = vals[colptr[j]:colptr[j + 1]]
    S = np.array([0, 3, 5, 8, 9, 14], np.int32)
    xv = ((rng.integers(0, 1 << 24, S.size) + 1) / float(1 << 24)).astype(np.float32)
    yi, yv, W = oracle.spmspv(A, S, xv, lib=lib)
    ref = D[:, S] @ xv.astype(np.float64)
    rows = np.nonzero(P[:, S].any(1))[0]
    got = dict(zip(yi.tolist(), yv.tolist()))
    if sorted(got) != rows.tolist() or any(not abs(got[i] - ref[i]) <= 1e-14 for i in rows):
        failed.append("plus_times")
    if W != int(np.diff(colptr)[S].sum()):
        failed.append("work")
    xi = rng.integers(-50, 50, S.size).astype(np.int32)
    yi, yv, _ = oracle.spmspv(A, S, xi, oracle.MIN_SELECT2ND, lib=lib)
    got = dict(zip(yi.tolist(), yv.tolist()))
    if sorted(got) != rows.tolist() or any(got[i] != min(int(xi[k]) for k in range(S.size) if P[i, S[k]])
                                           for i in rows):
        failed.append("min_select2nd")
    xb = np.array([1, 0, 1, 0, 1, 1], np.uint8)
    yi, yv, _ = oracle.spmspv(A, S, xb, oracle.OR_AND, lib=lib)
    got = dict(zip(yi.tolist(), yv.tolist()))
    if sorted(got) != rows.tolist() or any(got[i] != int(any(P[i, S[k]] and xb[k] for k in range(S.size)))
                                           for i in rows):
        failed.append("or_and")
    mask = (np.arange(m) % 3 == 0).astype(np.uint8)
    yi, _, _ = oracle.spmspv(A, S, xv, mask=mask, lib=lib)
    if sorted(yi.tolist()) != [i for i in rows.tolist() if not mask[i]]:
        failed.append("mask")
    # grid BFS closed form
    nx = 6
    G = synth.grid(nx, nx, nx)
    lev, par, _ = oracle.bfs(G, 0, lib=lib)
    v = np.arange(G.n)
    x, y, z = v % nx, (v // nx) % nx, v // (nx * nx)
    if not np.array_equal(lev, x + y + z):
        failed.append("bfs_levels")
    ep = np.where(z > 0, v - nx * nx, np.where(y > 0, v - nx, v - 1))
    ep[0] = 0
    if not np.array_equal(par, ep):
        failed.append("bfs_parents")
    return failed


def test_unmodified_oracle_passes():
    assert pin_suite(oracle.load()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = oracle.build(force=True, src=str(path), out=str(tmp_path / "libmutant.so"))
    lib = oracle.load(so)
    assert pin_suite(lib) != [], f"mutant {name} survived the pins"
