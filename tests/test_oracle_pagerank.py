"""Pins of the oracle's data-driven PageRank against closed forms and a
dense linear solve (not against itself), plus planted mistakes that the
pins must catch."""
import os

import numpy as np
import pytest

import oracle
import synth

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")


def dense_normalised(A):
    """A_n(i, j) = 1 / outdeg(j) for stored A(i, j) (edge j -> i)."""
    An = np.zeros((A.n, A.n))
    for j in range(A.n):
        rows = A.rowids[A.colptr[j]:A.colptr[j + 1]]
        if rows.size:
            An[rows, j] += 1.0 / rows.size
    return An


def exact(A, d):
    """Fixed point p = (1-d)/n + d A_n p (dangling mass dropped), by a linear solve."""
    return np.linalg.solve(np.eye(A.n) - d * dense_normalised(A), np.full(A.n, (1 - d) / A.n))


def small_graphs():
    yield synth.rmat(7, 8, seed=5, symmetrize=False)           # directed, with dangling vertices
    yield synth.rmat(7, 8, seed=6, symmetrize=True)
    g = synth.grid(5, 4, 3)
    yield g


def pins(lib) -> list:
    failed = []
    d = 0.85
    for k, A in enumerate(small_graphs()):
        r, it, act = oracle.pagerank(A, d, 0.0, 400, lib=lib)
        if not np.max(np.abs(r - exact(A, d))) <= 1e-12 * max(1.0, np.max(r)):
            failed.append(f"exact{k}")
    # 3-cycle: uniform 1/3
    cyc = synth.CSC(3, 3, np.array([0, 1, 2, 3], np.int32), np.array([1, 2, 0], np.int32), None)
    r, _, _ = oracle.pagerank(cyc, d, 0.0, 400, lib=lib)
    if not np.max(np.abs(r - 1 / 3)) <= 1e-12:
        failed.append("cycle")
    # star 0 -> 1..n-1, leaves dangling: p0 = (1-d)/n, leaves (1-d)/n (1 + d/(n-1))
    n = 9
    star = synth.CSC(n, n, np.array([0] + [n - 1] * n, np.int32), np.arange(1, n, dtype=np.int32), None)
    r, it, _ = oracle.pagerank(star, d, 0.0, 50, lib=lib)
    b = (1 - d) / n
    if not (abs(r[0] - b) <= 1e-15 and np.max(np.abs(r[1:] - b * (1 + d / (n - 1)))) <= 1e-15) or it != 2:
        failed.append("star")
    # tol > 0: never above the exact solution, and within a bound of it
    A = synth.rmat(8, 8, seed=9, symmetrize=True)
    tol = 1e-3
    r, it, act = oracle.pagerank(A, d, tol, 200, lib=lib)
    ex = exact(A, d)
    if not (np.all(r <= ex * (1 + 1e-12)) and np.max(ex - r) <= it * tol * np.max(ex)):
        failed.append("tolerance")
    if not (act[0] == A.n and act[-1] == 0 and it < 200):
        failed.append("termination")
    return failed


def test_oracle_pagerank_pins():
    assert pins(oracle.load()) == []


def test_sum_is_one_without_dangling():
    A = synth.grid(6, 6, 2)
    r, _, _ = oracle.pagerank(A, 0.85, 0.0, 400)
    assert abs(r.sum() - 1.0) < 1e-12


MUTANTS = {
    "no_damping_on_push": ("const double c = damping * delta[j] / (double)len;",
                           "const double c = delta[j] / (double)len;"),
    "wrong_normaliser": ("const double c = damping * delta[j] / (double)len;",
                         "const double c = damping * delta[j] / (double)(len + 1);"),
    "teleport_not_divided": ("delta[v] = (1.0 - damping) / (double)n;", "delta[v] = (1.0 - damping);"),
    "activity_absolute": ("active[v] = reached[v] && next[v] > tol * rank[v];",
                          "active[v] = reached[v] && next[v] > tol;"),
    "pushes_to_source": ("next[rowids[q]] += c;\n                reached[rowids[q]] = 1;",
                         "next[j] += c;\n                reached[j] = 1;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pagerank_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = oracle.build(force=True, src=str(path), out=str(tmp_path / "libmutant.so"))
    assert pins(oracle.load(so)) != [], f"mutant {name} survived the pins"
