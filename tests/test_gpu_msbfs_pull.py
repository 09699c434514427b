"""GPU parity of the direction-switching multi-source BFS (msbfs_run with
SPMSPV_DIRECTION_OPT: push levels through the batched SpMSpV, then pull
levels on one-bit-per-source masks) against the oracle, source by source:
levels and, for min-select2nd, parents (the smallest frontier
in-neighbour) bit for bit; the level count.  Source counts that fill one
64-bit mask word, part of one, and more than one; repeated and isolated
roots; hub rows longer than one thread's scan; a directed graph through the
CSR copy (or-and; min-select2nd there keeps the push direction); a grid
against its closed form; and the benchmark's scale-20 graph with 64
sources."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import to_np

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


def check(spv, M, A, roots, semiring, flags=None):
    flags = spv.DIRECTION_OPT if flags is None else flags
    lev, par, nl = M.msbfs(roots, semiring=semiring, flags=flags)
    lev = to_np(lev)
    maxl = 0
    for k, r in enumerate(roots):
        olev, opar, onl = oracle.bfs(A, int(r))
        assert np.array_equal(lev[k], olev), f"levels of source {k} (root {r})"
        if semiring == 1:
            assert np.array_equal(to_np(par[k]), opar), f"parents of source {k} (root {r})"
        maxl = max(maxl, onl)
    assert nl == maxl
    return nl


@pytest.fixture(scope="module")
def r15(spv):
    A = synth.rmat(15, 16, seed=41, symmetrize=True)
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    M.attach_batch(130, msbfs=True)
    yield A, M
    M.close()


@pytest.mark.parametrize("nsrc", [1, 5, 64, 100, 130])
@pytest.mark.parametrize("semiring", [1, 2])
def test_matches_oracle(spv, r15, nsrc, semiring):
    A, M = r15
    assert int(A.degrees().max()) > 64          # some rows take the wave-wide scan
    roots = [int(r) for r in synth.roots(A, nsrc, seed=nsrc * 7 + semiring)]
    if nsrc >= 5:
        roots[3] = roots[1]                     # the same root twice
        iso = np.nonzero(A.degrees() == 0)[0]
        if iso.size:
            roots[4] = int(iso[0])              # an isolated root
    check(spv, M, A, roots, semiring)


def test_same_results_as_push_only(spv, r15):
    A, M = r15
    roots = [int(r) for r in synth.roots(A, 64, seed=3)]
    a = [to_np(t) for t in M.msbfs(roots, semiring=1, flags=0)[:2]]
    b = [to_np(t) for t in M.msbfs(roots, semiring=1, flags=spv.DIRECTION_OPT)[:2]]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_directed_graph_through_the_csr_copy(spv):
    A = synth.rmat(14, 16, seed=42)                      # directed
    M = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE, pattern=True)
    M.attach_batch(70, msbfs=True)
    roots = [int(r) for r in synth.roots(A, 70, seed=5)]
    check(spv, M, A, roots, 2)
    check(spv, M, A, roots, 1)                           # rows not ascending: push only, same answer
    M.close()


def test_grid_closed_form(spv):
    nx, ny, nz = 40, 30, 20
    A = synth.grid(nx, ny, nz)
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    M.attach_batch(4, msbfs=True)
    corners = [0, nx - 1, nx * ny * nz - 1, nx * (ny - 1)]
    lev, par, nl = M.msbfs(corners, semiring=1, flags=spv.DIRECTION_OPT)
    lev = to_np(lev)
    v = np.arange(nx * ny * nz)
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    assert np.array_equal(lev[0], x + y + z)
    assert np.array_equal(lev[1], (nx - 1 - x) + y + z)
    assert np.array_equal(lev[2], (nx - 1 - x) + (ny - 1 - y) + (nz - 1 - z))
    assert np.array_equal(lev[3], x + (ny - 1 - y) + z)
    assert nl == nx + ny + nz - 2
    for k, r in enumerate(corners):
        assert np.array_equal(to_np(par[k]), oracle.bfs(A, r)[1])
    M.close()


def test_full_size_rmat20_64_sources(spv):
    A = synth.rmat(20, 16, seed=2, symmetrize=True)
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    M.attach_batch(64, msbfs=True)
    roots = [int(r) for r in synth.roots(A, 64, seed=11)]
    lev, par, nl = M.msbfs(roots, semiring=1, flags=spv.DIRECTION_OPT)
    lev, par = to_np(lev), to_np(par)
    rng = np.random.default_rng(0)
    for k in sorted(rng.choice(64, 12, replace=False)):
        olev, opar, _ = oracle.bfs(A, roots[k])
        assert np.array_equal(lev[k], olev), f"levels of source {k}"
        assert np.array_equal(par[k], opar), f"parents of source {k}"
    M.close()
