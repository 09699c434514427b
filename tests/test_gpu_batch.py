"""GPU parity of batched SpMSpV (many x against one A in one launch
sequence) and of the multi-source BFS built on it, against the oracle
run once per vector / per source."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare, to_np

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


@pytest.fixture(scope="module")
def rmat14():
    return synth.rmat(14, 16, seed=21, symmetrize=True)


def make_batch(A, sizes, seed):
    xs = [synth.sparse_x(A.n, int(f), seed=seed + k, tag=k) for k, f in enumerate(sizes)]
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum([x[0].size for x in xs])
    idx = np.concatenate([x[0] for x in xs]) if off[-1] else np.zeros(0, np.int32)
    val = np.concatenate([x[1] for x in xs]) if off[-1] else np.zeros(0, np.float32)
    return xs, off, idx.astype(np.int32), val.astype(np.float32)


def check_batch(spv, M, A, xs, off, idx, val, semiring, flags=0):
    B = len(xs)
    if semiring == 0:
        xv_d = dev(val) if idx.size else torch.zeros(1, dtype=torch.float32, device="cuda")
        fl = flags
    elif semiring == 1:
        xv_d, fl = None, flags | spv.X_VAL_IS_INDEX
    else:
        xv_d, fl = None, flags | spv.X_ALL_TRUE
    xi_d = dev(idx) if idx.size else torch.zeros(1, dtype=torch.int32, device="cuda")
    y_off, y_idx, y_val, total = M.spmspv_batch(dev(off), xi_d, xv_d, semiring=semiring, flags=fl)
    yo = to_np(y_off)
    assert yo[0] == 0 and yo[-1] == total and np.all(np.diff(yo) >= 0)
    for b in range(B):
        S, xv = xs[b]
        if semiring == 1:
            oxv = S.astype(np.int32)
        elif semiring == 2:
            oxv = np.ones(S.size, np.uint8)
        else:
            oxv = xv
        oi, ov, _ = oracle.spmspv(A, S, oxv, semiring, sorted_output=True)
        gi = y_idx[yo[b]:yo[b + 1]]
        gv = y_val[yo[b]:yo[b + 1]]
        compare(semiring, gi, gv, oi, ov, sorted_output=True)
    assert M.last_stats()["err"] == 0
    return total


@pytest.mark.parametrize("semiring", [0, 1, 2])
def test_batch_log_uniform_sizes(spv, rmat14, semiring):
    A = rmat14
    M = spv.Matrix.from_csc(A)
    sizes = synth.log_uniform_sizes(64, A.n / 4, seed=semiring + 5)
    sizes[3] = 0                      # an empty vector in the middle
    xs, off, idx, val = make_batch(A, sizes, 100 * semiring)
    M.attach_batch(64, max_f=int(off[-1]), max_products=int(sum(A.degrees()[x[0]].sum() for x in xs)))
    check_batch(spv, M, A, xs, off, idx, val, semiring)


@pytest.mark.parametrize("B", [1, 2, 7, 33])
def test_batch_sizes_and_tiles(spv, rmat14, B):
    A = rmat14
    M = spv.Matrix.from_csc(A)
    rng = np.random.default_rng(B)
    sizes = rng.integers(0, A.n // 8, B)
    xs, off, idx, val = make_batch(A, sizes, 7 * B)
    M.attach_batch(64, max_f=A.n * 8, max_products=A.nnz * 8)
    for tl in (8, 10, 14):
        s = M.schedule
        s.tile_log2 = tl
        spv.spmspv_set_batch_schedule(M.handle, s)
        eff = spv.spmspv_get_batch_schedule(M.handle, B)
        assert eff.tile_log2 >= tl and B * ((A.m + (1 << eff.tile_log2) - 1) >> eff.tile_log2) <= 8192
        check_batch(spv, M, A, xs, off, idx, val, 0)
        check_batch(spv, M, A, xs, off, idx, val, 1)


def test_batch_all_empty_and_rectangular(spv):
    m, n = 3000, 5000
    rng = np.random.default_rng(4)
    rows = rng.integers(0, m, 40000).astype(np.int32)
    cols = rng.integers(0, n, 40000).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(m, n, rows, cols, drop_self=False)
    A = synth.CSC(m, n, colptr, rowids, synth.values(rowids.size, 3))
    M = spv.Matrix.from_csc(A)
    M.attach_batch(16, max_f=n * 4, max_products=A.nnz * 4)
    xs, off, idx, val = make_batch(A, [0, 0, 0], 1)
    assert check_batch(spv, M, A, xs, off, idx, val, 0) == 0
    xs, off, idx, val = make_batch(A, [10, 0, 4999, 5000, 1], 2)
    check_batch(spv, M, A, xs, off, idx, val, 0)
    check_batch(spv, M, A, xs, off, idx, val, 2)


def test_batch_errors(spv, rmat14):
    A = rmat14
    M = spv.Matrix.from_csc(A)
    xs, off, idx, val = make_batch(A, [500, 500], 9)
    with pytest.raises(spv.SpmspvError):                     # no workspace yet
        M.spmspv_batch(dev(off), dev(idx), dev(val))
    M.attach_batch(4, max_f=2000, max_products=100)          # far too few products
    with pytest.raises(spv.SpmspvError) as e:
        M.spmspv_batch(dev(off), dev(idx), dev(val))
    assert e.value.status == spv.ECAPACITY
    M.attach_batch(4, max_f=2000, max_products=A.nnz * 2)
    check_batch(spv, M, A, xs, off, idx, val, 0)             # recovers after the error
    dup = idx.copy()
    dup[1] = dup[0]
    with pytest.raises(spv.SpmspvError) as e:
        M.spmspv_batch(dev(off), dev(dup), dev(val), flags=spv.VALIDATE)
    assert e.value.status == spv.EINVAL
    bad_off = off.copy()
    bad_off[-1] = 5000                                       # beyond max_f
    with pytest.raises(spv.SpmspvError) as e:
        M.spmspv_batch(dev(bad_off), dev(idx), dev(val))
    assert e.value.status == spv.EINVAL
    # a small output capacity is reported, not overrun
    with pytest.raises(spv.SpmspvError) as e:
        M.spmspv_batch(dev(off), dev(idx), dev(val), y_capacity=10)
    assert e.value.status == spv.ECAPACITY


def test_batch_attach_over_stale_memory(spv, rmat14):
    """A batch workspace is used as handed over, whatever it held: every
    word the first call depends on is initialised by the attach or the call
    itself.  0x80 bytes make every 64-bit look-back word read as a complete
    prefix with a huge value."""
    A = rmat14
    M = spv.Matrix.from_csc(A)
    xs, off, idx, val = make_batch(A, [3000, 0, 5000, 200], 13)
    nbytes = spv.spmspv_batch_workspace_size(M.handle, 8, int(off[-1]), A.nnz * 2, 0)
    ws = torch.full((nbytes,), 0x80, dtype=torch.uint8, device="cuda")
    spv.spmspv_batch_attach(M.handle, 8, int(off[-1]), A.nnz * 2, 0, ws, nbytes)
    M.batch_ws = ws
    check_batch(spv, M, A, xs, off, idx, val, 0)
    check_batch(spv, M, A, xs, off, idx, val, 1)
    P = spv.Matrix.from_csc(A, pattern=True)
    nbytes = spv.spmspv_batch_workspace_size(P.handle, 4, 0, 0, spv.MSBFS)
    ws = torch.full((nbytes,), 0x80, dtype=torch.uint8, device="cuda")
    spv.spmspv_batch_attach(P.handle, 4, 0, 0, spv.MSBFS, ws, nbytes)
    P.batch_ws = ws
    roots = [int(r) for r in synth.roots(A, 4, seed=17)]
    lev, _, _ = P.msbfs(roots, semiring=2, parents=False)
    lev = to_np(lev)
    for k, r in enumerate(roots):
        assert np.array_equal(lev[k], oracle.bfs(A, r)[0]), f"source {k} root {r}"


def test_batch_then_single_calls_agree(spv, rmat14):
    """Batched and single calls share the handle's control block."""
    A = rmat14
    M = spv.Matrix.from_csc(A)
    M.attach_batch(8, max_f=A.n, max_products=A.nnz * 4)
    xs, off, idx, val = make_batch(A, [300, 2000, 40], 11)
    check_batch(spv, M, A, xs, off, idx, val, 0)
    S, xv = xs[1]
    gi, gv, _ = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True)
    oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
    compare(0, gi, gv, oi, ov, sorted_output=True)
    check_batch(spv, M, A, xs, off, idx, val, 1)


@pytest.mark.parametrize("semiring", [0, 1, 2])
def test_fixed_and_counted_slices(spv, rmat14, semiring):
    """The same batch through fixed slices (a workspace for B * nnz(A)
    products: one bucketing pass, each (vector, bucket) key in a slice sized
    by its rows' stored entries) and through counted slices (a workspace for
    exactly the batch's products: a counting pass first).  Both match the
    oracle vector by vector, twice in a row."""
    A = rmat14
    M = spv.Matrix.from_csc(A)
    B = 24
    sizes = synth.log_uniform_sizes(B, A.n / 2, seed=60 + semiring)
    sizes[0] = A.n                     # a whole-width vector: every slice filled to the brim
    sizes[9] = 0
    xs, off, idx, val = make_batch(A, sizes, 300 + semiring)
    W = int(sum(A.degrees()[x[0]].sum() for x in xs))
    assert W < B * A.nnz
    for mp in (B * A.nnz, W):
        M.attach_batch(B, max_f=int(off[-1]), max_products=mp)
        for _ in range(2):
            check_batch(spv, M, A, xs, off, idx, val, semiring)


def test_repeated_index_fixed_vs_counted(spv):
    """A repeated x index breaks the distinctness precondition.  On the
    identity matrix, 5000 copies of column 7 put 5000 products into a bucket
    whose rows hold at most 4096 entries: fixed slices report the overflow
    (EDEVICE) and the handle keeps working; counted slices combine the
    repeated products as the oracle does."""
    n = 4096
    A = synth.CSC(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n, np.float32))
    M = spv.Matrix.from_csc(A)
    rng = np.random.default_rng(8)
    S0 = np.full(5000, 7, np.int32)
    S1 = np.arange(0, n, 3, dtype=np.int32)
    xs = [(S0, rng.random(S0.size).astype(np.float32)), (S1, rng.random(S1.size).astype(np.float32))]
    off = np.array([0, S0.size, S0.size + S1.size], np.int64)
    idx = np.concatenate([S0, S1])
    val = np.concatenate([xs[0][1], xs[1][1]])
    M.attach_batch(2, max_f=int(off[-1]), max_products=2 * n)          # fixed slices
    with pytest.raises(spv.SpmspvError) as e:
        M.spmspv_batch(dev(off), dev(idx), dev(val))
    assert e.value.status == spv.EDEVICE
    good = [xs[1], (S1[::2].copy(), xs[1][1][::2].copy())]
    goff = np.array([0, S1.size, S1.size + good[1][0].size], np.int64)
    check_batch(spv, M, A, good, goff, np.concatenate([g[0] for g in good]),
                np.concatenate([g[1] for g in good]), 0)
    M.attach_batch(2, max_f=int(off[-1]), max_products=int(off[-1]))   # counted slices
    check_batch(spv, M, A, xs, off, idx, val, 0)


@pytest.mark.parametrize("semiring", [1, 2])
def test_msbfs_matches_oracle(spv, rmat14, semiring):
    A = rmat14
    M = spv.Matrix.from_csc(A, pattern=True)
    roots = list(synth.roots(A, 16, seed=31))
    roots[5] = roots[2]                                      # the same root twice
    iso = np.nonzero(A.degrees() == 0)[0]
    if iso.size:
        roots[7] = int(iso[0])                               # an isolated root
    M.attach_batch(16, msbfs=True)
    lev, par, nl = M.msbfs(roots, semiring=semiring)
    lev = to_np(lev)
    maxl = 0
    for k, r in enumerate(roots):
        olev, opar, onl = oracle.bfs(A, int(r))
        assert np.array_equal(lev[k], olev), f"source {k} root {r}"
        if semiring == 1:
            assert np.array_equal(to_np(par[k]), opar), f"parents of source {k}"
        maxl = max(maxl, onl)
    assert nl == maxl


def test_msbfs_grid_closed_form(spv):
    A = synth.grid(24, 20, 6)
    M = spv.Matrix.from_csc(A, pattern=True)
    M.attach_batch(3, msbfs=True)
    nx, ny, nz = 24, 20, 6
    corners = [0, nx - 1, nx * ny * nz - 1]
    lev, par, nl = M.msbfs(corners, semiring=2, parents=False)
    lev = to_np(lev)
    v = np.arange(nx * ny * nz)
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    assert np.array_equal(lev[0], x + y + z)
    assert np.array_equal(lev[1], (nx - 1 - x) + y + z)
    assert np.array_equal(lev[2], (nx - 1 - x) + (ny - 1 - y) + (nz - 1 - z))
    assert nl == nx + ny + nz - 2


def test_msbfs_errors(spv, rmat14):
    M = spv.Matrix.from_csc(rmat14, pattern=True)
    with pytest.raises(spv.SpmspvError):
        M.msbfs([0, 1])                                      # no workspace
    M.attach_batch(2, max_f=100, max_products=100)           # attached without MSBFS
    with pytest.raises(spv.SpmspvError):
        M.msbfs([0, 1])
    M.attach_batch(2, msbfs=True)
    with pytest.raises(spv.SpmspvError):
        M.msbfs([0, 1, 2])                                   # more sources than max_batch
    with pytest.raises(spv.SpmspvError):
        M.msbfs([0, rmat14.n])                               # root out of range
