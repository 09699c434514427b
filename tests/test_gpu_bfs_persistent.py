"""GPU parity of the persistent small-frontier BFS levels (cooperative
kernel) and their hand-off to the bucketing levels, against the oracle."""
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


def random_graph(n, avg_deg, seed):
    rng = np.random.default_rng(seed)
    k = n * avg_deg // 2
    r = rng.integers(0, n, k).astype(np.int32)
    c = rng.integers(0, n, k).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(n, n, np.concatenate([r, c]), np.concatenate([c, r]))
    return synth.CSC(n, n, colptr, rowids, None, f"er{n}")


def check(spv, M, A, root, semiring, flags):
    lev, par, nl = M.bfs(int(root), semiring=semiring, parents=semiring == 1, flags=flags)
    olev, opar, onl = oracle.bfs(A, int(root))
    assert nl == onl
    assert np.array_equal(to_np(lev), olev)
    if semiring == 1:
        assert np.array_equal(to_np(par), opar)


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("semiring", [1, 2])
def test_persistent_grid_closed_form(spv, graph, semiring):
    nx, ny, nz = 40, 30, 20
    A = synth.grid(nx, ny, nz)
    M = spv.Matrix.from_csc(A, pattern=True)
    fl = spv.PERSISTENT | (spv.USE_GRAPH if graph else 0)
    for root in (0, nx * ny * nz - 1, 12345):
        check(spv, M, A, root, semiring, fl)


def test_persistent_hands_off_large_frontiers(spv):
    """Frontiers grow ~8x per level past 65536 vertices (bucketing levels),
    then shrink again (persistent levels)."""
    A = random_graph(1 << 20, 8, 5)
    assert int(np.diff(A.colptr).max()) <= 64
    M = spv.Matrix.from_csc(A, pattern=True)
    for root in synth.roots(A, 3, seed=4):
        check(spv, M, A, root, 1, spv.PERSISTENT | spv.USE_GRAPH)
        check(spv, M, A, root, 2, spv.PERSISTENT)


def test_persistent_ignored_on_high_degree(spv):
    A = synth.rmat(14, 16, seed=3, symmetrize=True)
    M = spv.Matrix.from_csc(A, pattern=True)
    for root in synth.roots(A, 2, seed=6):
        check(spv, M, A, root, 1, spv.PERSISTENT | spv.USE_GRAPH)


def test_persistent_repeated_runs_and_isolated_root(spv):
    A = random_graph(50000, 3, 9)
    M = spv.Matrix.from_csc(A, pattern=True)
    deg = np.diff(A.colptr)
    iso = np.nonzero(deg == 0)[0]
    roots = list(synth.roots(A, 4, seed=2)) + ([int(iso[0])] if iso.size else [])
    for _ in range(2):
        for r in roots:
            check(spv, M, A, r, 1, spv.PERSISTENT)


@pytest.mark.parametrize("tail", [0, 1, 2])
def test_persistent_hand_off_from_every_slot(spv, tail):
    """The kernel rotates three frontier lists; a frontier that outgrows the
    persistent range is copied back to the first list unless it already
    lies there.  A path of `tail` extra vertices in front of an expander
    shifts the level of the hand-off by one per vertex, so the three cases
    cover every list the frontier can end in.  The same handle then runs
    again without the persistent levels and with them, to show the kernel
    left its scratch state clean."""
    n0 = 1 << 19
    rng = np.random.default_rng(11)
    k = n0 * 8 // 2
    r = rng.integers(0, n0, k).astype(np.int64)
    c = rng.integers(0, n0, k).astype(np.int64)
    # chain n0+tail - ... - n0 - 0 (edges (n0+i, n0+i+1) and (n0, 0))
    pr = np.concatenate([np.arange(n0, n0 + tail), [n0]]).astype(np.int64)
    pc = np.concatenate([np.arange(n0 + 1, n0 + tail + 1), [0]]).astype(np.int64)
    n = n0 + tail + 1
    rows = np.concatenate([r, c, pr, pc]).astype(np.int32)
    cols = np.concatenate([c, r, pc, pr]).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(n, n, rows, cols)
    A = synth.CSC(n, n, colptr, rowids, None, f"tail{tail}")
    assert int(np.diff(A.colptr).max()) <= 64
    M = spv.Matrix.from_csc(A, pattern=True)
    root = n0 + tail
    check(spv, M, A, root, 1, spv.PERSISTENT)
    check(spv, M, A, root, 2, 0)
    check(spv, M, A, root, 1, spv.PERSISTENT | spv.USE_GRAPH)
    check(spv, M, A, int(synth.roots(A, 1, seed=tail)[0]), 2, spv.PERSISTENT)
