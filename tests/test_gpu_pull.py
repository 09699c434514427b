"""GPU parity of the pull (matrix-driven) direction and of the
direction-optimizing BFS, against the CPU oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare

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


def pull_schedule(spv, M):
    s = M.schedule
    s.direction = 1
    M.schedule = s


def run_pair(spv, M, A, S, semiring, xval, flags=0):
    gi, gv, nnz = M.spmspv(dev(S), None if xval is None else dev(xval), semiring=semiring, flags=flags)
    if semiring == 1 and xval is None:
        oxv = S.astype(np.int32)
    elif semiring == 2 and xval is None:
        oxv = np.ones(S.size, np.uint8)
    else:
        oxv = xval
    oi, ov, W = oracle.spmspv(A, S, oxv, semiring, sorted_output=True)
    compare(semiring, gi, gv, oi, ov, sorted_output=True)
    assert M.last_stats()["err"] == 0


@pytest.mark.parametrize("shape", [(5000, 3000), (1200, 4000), (4096, 4096)])
def test_pull_with_transpose_all_semirings(spv, shape):
    m, n = shape
    rng = np.random.default_rng(m + n)
    nt = 10 * max(m, n)
    rows = np.concatenate([rng.integers(0, m, nt), np.full(n, 7)]).astype(np.int32)        # row 7: a hub
    cols = np.concatenate([rng.integers(0, n, nt), np.arange(n)]).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(m, n, rows, cols, drop_self=False)
    A = synth.CSC(m, n, colptr, rowids, synth.values(rowids.size, 5))
    M = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE)
    pull_schedule(spv, M)
    assert M.schedule.direction == 1
    for f in (1, n // 50, n // 3, n):
        S, xv = synth.sparse_x(n, f, seed=f)
        run_pair(spv, M, A, S, 0, xv)
        run_pair(spv, M, A, S, 1, rng.integers(-500, 500, f).astype(np.int32))
        run_pair(spv, M, A, S, 1, None, flags=spv.X_VAL_IS_INDEX)
        run_pair(spv, M, A, S, 2, (rng.random(f) < 0.6).astype(np.uint8))
        run_pair(spv, M, A, S, 2, None, flags=spv.X_ALL_TRUE)


@pytest.mark.parametrize("flag", ["WITH_TRANSPOSE", "SYMMETRIC"])
def test_pull_many_columns(spv, flag):
    """More than 2^20 columns (an x bitmap larger than any LDS slice) and a
    hub row spanning many merge-path chunks."""
    rng = np.random.default_rng(11)
    if flag == "SYMMETRIC":
        n = m = 1_300_000
        nt = 3 * n
        r = rng.integers(0, n, nt)
        c = rng.integers(0, n, nt)
        hub = np.arange(0, n, 5)
        rows = np.concatenate([r, c, np.full(hub.size, 7), hub]).astype(np.int32)
        cols = np.concatenate([c, r, hub, np.full(hub.size, 7)]).astype(np.int32)
    else:
        m, n = 30000, 1_500_000
        nt = 3_000_000
        hub = np.arange(0, n, 3)
        rows = np.concatenate([rng.integers(0, m, nt), np.full(hub.size, 7)]).astype(np.int32)
        cols = np.concatenate([rng.integers(0, n, nt), hub]).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(m, n, rows, cols, drop_self=False)
    # a symmetric handle reads A's columns as its rows: pattern only there
    A = synth.CSC(m, n, colptr, rowids, None if flag == "SYMMETRIC" else synth.values(rowids.size, 6))
    M = spv.Matrix.from_csc(A, flags=getattr(spv, flag))
    pull_schedule(spv, M)
    for f in (50, 20000, 400000):
        S, xv = synth.sparse_x(n, f, seed=f + 3)
        run_pair(spv, M, A, S, 0, xv)
        run_pair(spv, M, A, S, 1, None, flags=spv.X_VAL_IS_INDEX)
        run_pair(spv, M, A, S, 2, None, flags=spv.X_ALL_TRUE)


def test_pull_symmetric_pattern(spv):
    A = synth.rmat(15, seed=3, symmetrize=True, with_values=False)
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC)
    pull_schedule(spv, M)
    for f in (10, 3000, 30000):
        S, xv = synth.sparse_x(A.n, f, seed=f + 1)
        run_pair(spv, M, A, S, 0, xv)
        run_pair(spv, M, A, S, 1, None, flags=spv.X_VAL_IS_INDEX)
        run_pair(spv, M, A, S, 2, None, flags=spv.X_ALL_TRUE)
    # push and pull give the same bits for int / bool
    S, _ = synth.sparse_x(A.n, 5000, seed=9)
    a = M.spmspv(dev(S), None, semiring=1, flags=spv.X_VAL_IS_INDEX)
    M.schedule = None
    b = M.spmspv(dev(S), None, semiring=1, flags=spv.X_VAL_IS_INDEX, sorted_output=True)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_pull_rejected_without_rows(spv):
    A = synth.rmat(10, seed=1)
    M = spv.Matrix.from_csc(A)
    s = M.schedule
    s.direction = 1
    with pytest.raises(spv.SpmspvError):
        M.schedule = s


@pytest.mark.parametrize("create_flag", ["SYMMETRIC", "WITH_TRANSPOSE"])
@pytest.mark.parametrize("graph", [False, True])
def test_direction_optimizing_bfs(spv, create_flag, graph):
    A = synth.rmat(16, seed=1, symmetrize=True, with_values=False)
    M = spv.Matrix.from_csc(A, flags=getattr(spv, create_flag))
    fl = spv.DIRECTION_OPT | (spv.USE_GRAPH if graph else 0)
    for root in synth.roots(A, 3, seed=2000):
        lev, par, nl = M.bfs(int(root), spv.MIN_SELECT2ND_I32, flags=fl)
        olev, opar, onl = oracle.bfs(A, int(root))
        assert nl == onl
        assert np.array_equal(lev.cpu().numpy(), olev)
        assert np.array_equal(par.cpu().numpy(), opar)
        lev2, _, nl2 = M.bfs(int(root), spv.OR_AND_BOOL, flags=fl)
        assert nl2 == onl and np.array_equal(lev2.cpu().numpy(), olev)


def test_direction_optimizing_grid(spv):
    nx = 48
    G = synth.grid(nx, nx, nx, diag=True)
    M = spv.Matrix.from_csc(G, flags=spv.SYMMETRIC)
    lev, par, nl = M.bfs(0, spv.MIN_SELECT2ND_I32, flags=spv.DIRECTION_OPT | spv.USE_GRAPH)
    v = np.arange(G.n)
    x, y, z = v % nx, (v // nx) % nx, v // (nx * nx)
    assert nl == 3 * (nx - 1) + 1 and np.array_equal(lev.cpu().numpy(), x + y + z)
    ep = np.where(z > 0, v - nx * nx, np.where(y > 0, v - nx, v - 1))
    ep[0] = 0
    assert np.array_equal(par.cpu().numpy(), ep)


def test_pull_identity_kept_across_bfs_graph_replays(spv):
    """The pull multiply combines rows that straddle two workgroups into a
    dense buffer that holds the semiring's identity between calls.  Captured
    BFS level graphs (with min-select2nd pull levels) replayed between
    plus-times pull calls must leave that buffer as the next call expects."""
    A = synth.rmat(15, seed=5, symmetrize=True, with_values=False)
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC)
    roots = synth.roots(A, 2, seed=3)
    S, xv = synth.sparse_x(A.n, 20000, seed=8)

    def bfs_check(r):
        lev, par, nl = M.bfs(int(r), spv.MIN_SELECT2ND_I32, flags=spv.USE_GRAPH | spv.DIRECTION_OPT)
        olev, opar, onl = oracle.bfs(A, int(r))
        assert nl == onl
        assert np.array_equal(lev.cpu().numpy(), olev) and np.array_equal(par.cpu().numpy(), opar)

    pull_schedule(spv, M)
    run_pair(spv, M, A, S, 0, xv)   # plus-times pull: identity 0
    bfs_check(roots[0])             # captures the level graph
    run_pair(spv, M, A, S, 0, xv)
    bfs_check(roots[1])             # replays it
    run_pair(spv, M, A, S, 0, xv)
    run_pair(spv, M, A, S, 1, None, flags=spv.X_VAL_IS_INDEX)
    bfs_check(roots[0])
    run_pair(spv, M, A, S, 0, xv)


def _two_clusters(nc=20000, deg=32, path=40, seed=13):
    """Two random clusters joined by a path: a BFS from the first cluster
    goes push, pull (the cluster), push (the path), pull (the second
    cluster)."""
    rng = np.random.default_rng(seed)
    k = nc * deg // 2
    parts = []
    for base in (0, nc + path):
        r = rng.integers(0, nc, k) + base
        c = rng.integers(0, nc, k) + base
        parts.append((r, c))
    pr = np.arange(nc, nc + path)                       # path vertices
    parts.append((np.concatenate([[0], pr]), np.concatenate([pr, [nc + path]])))
    rows = np.concatenate([p[0] for p in parts] + [p[1] for p in parts]).astype(np.int32)
    cols = np.concatenate([p[1] for p in parts] + [p[0] for p in parts]).astype(np.int32)
    n = 2 * nc + path
    colptr, rowids = synth.coo_to_csc(n, n, rows, cols)
    return synth.CSC(n, n, colptr, rowids, None, "two-clusters")


def _heuristic_directions(A, olev):
    """The frontier-edge rule (push -> pull when 14 W > edges left, pull ->
    push when 24 f < n) replayed on the oracle's levels."""
    deg = np.diff(A.colptr).astype(np.int64)
    left, prev, dirs = int(A.nnz), 0, []
    for L in range(int(olev.max()) + 1):
        F = np.nonzero(olev == L)[0]
        f, W = F.size, int(deg[F].sum())
        d = (1 if W * 14 > left else 0) if prev == 0 else (0 if f * 24 < A.n else 1)
        left = max(left - W, 0)
        dirs.append(d)
        prev = d
    return dirs


@pytest.mark.parametrize("graph", [False, True])
def test_direction_switches_back_and_forth(spv, graph):
    """Pull levels in a row, then push levels, then pull again in one BFS:
    the scan-free pull chain, its hand-back to push (tables rebuilt, x bits
    cleared) and a fresh pull phase."""
    A = _two_clusters()
    root = 5
    olev, opar, onl = oracle.bfs(A, root)
    dirs = "".join(map(str, _heuristic_directions(A, olev)))
    assert "11" in dirs and "10" in dirs and dirs.count("01") >= 2, dirs   # the graph does exercise it
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC)
    fl = spv.DIRECTION_OPT | (spv.USE_GRAPH if graph else 0)
    for _ in range(2):
        lev, par, nl = M.bfs(root, spv.MIN_SELECT2ND_I32, flags=fl)
        assert nl == onl
        assert np.array_equal(lev.cpu().numpy(), olev)
        assert np.array_equal(par.cpu().numpy(), opar)
        lev2, _, nl2 = M.bfs(root, spv.OR_AND_BOOL, flags=fl)
        assert nl2 == onl and np.array_equal(lev2.cpu().numpy(), olev)
