"""GPU parity at the benchmark's full sizes, in the launch configurations the
benchmark times, against the oracle.  Whole outputs are compared: the
oracle's dense accumulator takes tens of milliseconds per multiply here.

* SpMSpV on R-MAT scale 22 (edge factor 16, symmetrised, relabelled;
  n = 4,194,304, nnz = 128,304,750) with the handle the benchmark builds
  (row form for the pull direction) and its default per-call schedule:
  x density 1 % (f = 41,943) for several of the 64 rotating x vectors, run
  back to back on one stream as the timed loop runs them; all three
  semirings, sorted output; the 0.01 % and 10 % ends of the density sweep,
  push and pull.
* BFS on scale 22 from the benchmark's roots, push and direction-optimising
  (captured level graph), against the queue BFS.
* The 256^3 grid BFS (766 levels) against its closed form, through the
  persistent kernel, the captured level graph and the direction-optimising
  loop, with and without parents.
* The batched workload (R-MAT scale 20, 64 x with log-uniform sizes) with
  the autotuned batch schedule, every vector against the oracle, and the
  64-source BFS with sampled sources against the queue BFS.
* BFS on the selector evaluation's held-out R-MAT scale 24 graph through the
  learned (device-gated and host-read) and heuristic level loops.

The tolerances are those of the other parity tests: bit-exact for int32,
bool and every index set; fp32 within 1e-5 of the fp64 sum (all inputs are
positive, so that is 1e-5 relative).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare, rmat24_pattern, to_np

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


@pytest.fixture(scope="module")
def s22(spv):
    A = synth.rmat(22, 16, seed=1, symmetrize=True)
    assert (A.n, A.nnz) == (4194304, 128304750)
    M = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE)
    yield A, M
    M.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def oracle_x(semiring, S, xv):
    if semiring == 1:
        return S.astype(np.int32)
    if semiring == 2:
        return np.ones(S.size, np.uint8)
    return xv


@pytest.mark.parametrize("launch", [0, 2], ids=["default_three_launches", "one_launch"])
def test_headline_multiply_full_size(spv, s22, launch):
    """The benchmark's default schedule (three launches) and the one-launch
    multiply on the same inputs."""
    A, M = s22
    f = synth.density_f(A.n, 0.01)
    assert f == 41943
    xs = [synth.sparse_x(A.n, f, seed=1000 + r) for r in (0, 1, 17, 63)]
    if launch:
        s = M.schedule
        s.launch = launch
        M.schedule = s
    eff = spv.spmspv_effective_schedule(M.handle, f, 0)
    assert eff.direction == 0 and eff.launch == (launch or 1)
    if launch == 0:
        assert eff.scatter_block * eff.scatter_items == 4096
    stream = torch.cuda.current_stream()
    outs = []
    for S, xv in xs:   # back to back on one stream, each into its own output
        y_idx = torch.empty(A.m, dtype=torch.int32, device="cuda")
        y_val = torch.empty(A.m, dtype=torch.float32, device="cuda")
        d_nnz = torch.zeros(1, dtype=torch.int64, device="cuda")
        spv.spmspv_run(M.handle, spv.PLUS_TIMES_F32, 0, f, dev(S), dev(xv), y_idx, y_val, A.m, d_nnz,
                       sync=False, stream=stream)
        outs.append((y_idx, y_val, d_nnz))
    torch.cuda.synchronize()
    assert M.last_stats()["err"] == 0
    M.schedule = None
    for (S, xv), (y_idx, y_val, d_nnz) in zip(xs, outs):
        oi, ov, W = oracle.spmspv(A, S, xv)
        k = int(to_np(d_nnz)[0])
        compare(0, y_idx[:k], y_val[:k], oi, ov)


@pytest.mark.parametrize("semiring", [0, 1, 2])
def test_full_size_semirings_sorted(spv, s22, semiring):
    A, M = s22
    S, xv = synth.sparse_x(A.n, synth.density_f(A.n, 0.01), seed=1005)
    if semiring == 0:
        gi, gv, nnz = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True)
    elif semiring == 1:
        gi, gv, nnz = M.spmspv(dev(S), None, semiring=1, sorted_output=True, flags=spv.X_VAL_IS_INDEX)
    else:
        gi, gv, nnz = M.spmspv(dev(S), None, semiring=2, sorted_output=True, flags=spv.X_ALL_TRUE)
    oi, ov, _ = oracle.spmspv(A, S, oracle_x(semiring, S, xv), semiring, sorted_output=True)
    compare(semiring, gi, gv, oi, ov, sorted_output=True)


@pytest.mark.parametrize("density", [1e-4, 1e-1])
@pytest.mark.parametrize("direction", [0, 1])
def test_full_size_density_sweep_ends(spv, s22, density, direction):
    A, M = s22
    S, xv = synth.sparse_x(A.n, synth.density_f(A.n, density), seed=3000)
    try:
        if direction:
            s = M.schedule
            s.direction = 1
            M.schedule = s
        else:
            M.schedule = None   # the default per-call schedule the sweep times
        for semiring in (0, 1):
            if semiring == 0:
                gi, gv, _ = M.spmspv(dev(S), dev(xv), semiring=0)
            else:
                gi, gv, _ = M.spmspv(dev(S), None, semiring=1, flags=spv.X_VAL_IS_INDEX)
            oi, ov, _ = oracle.spmspv(A, S, oracle_x(semiring, S, xv), semiring)
            compare(semiring, gi, gv, oi, ov)
    finally:
        M.schedule = None


def test_full_size_bfs_roots(spv, s22):
    A, M = s22
    P = spv.Matrix(A.m, A.n, M.colptr, M.rowids, None, flags=spv.SYMMETRIC)
    roots = synth.roots(A, 16, seed=2000)
    for r in (roots[0], roots[9]):
        olev, opar, onl = oracle.bfs(A, int(r))
        for fl in (spv.USE_GRAPH, spv.USE_GRAPH | spv.DIRECTION_OPT):
            lev, par, nl = P.bfs(int(r), spv.MIN_SELECT2ND_I32, flags=fl)
            assert nl == onl
            assert np.array_equal(to_np(lev), olev)
            assert np.array_equal(to_np(par), opar)
    P.close()


@pytest.fixture(scope="module")
def grid256(spv):
    G = synth.grid(256, 256, 256)
    assert G.nnz == 117047296
    P = spv.Matrix.from_csc(G, flags=spv.SYMMETRIC, pattern=True)
    v = np.arange(G.n, dtype=np.int64)
    x, y, z = v % 256, (v // 256) % 256, v // 65536
    expect_par = np.where(z > 0, v - 65536, np.where(y > 0, v - 256, v - 1))
    expect_par[0] = 0
    yield P, (x + y + z).astype(np.int32), expect_par.astype(np.int32)
    P.close()


@pytest.mark.parametrize("variant", ["persistent", "graph", "direction_heuristic"])
def test_full_size_grid_bfs(spv, grid256, variant):
    P, expect_lev, expect_par = grid256
    fl = {"persistent": spv.USE_GRAPH | spv.PERSISTENT, "graph": spv.USE_GRAPH,
          "direction_heuristic": spv.USE_GRAPH | spv.DIRECTION_OPT}[variant]
    lev, _, nl = P.bfs(0, spv.OR_AND_BOOL, parents=False, flags=fl)
    assert nl == 766
    assert np.array_equal(to_np(lev), expect_lev)
    lev, par, nl = P.bfs(0, spv.MIN_SELECT2ND_I32, parents=True, flags=fl)
    assert nl == 766
    assert np.array_equal(to_np(lev), expect_lev)
    assert np.array_equal(to_np(par), expect_par)


@pytest.fixture(scope="module")
def s20(spv):
    A = synth.rmat(20, 16, seed=1, symmetrize=True)
    M = spv.Matrix.from_csc(A)
    yield A, M
    M.close()


def test_full_size_batched_autotuned(spv, s20):
    """The benchmark's batch (64 vectors against R-MAT scale 20) with its
    workspace of 64 * nnz(A) products (fixed slices), autotuned, then with a
    workspace of exactly the batch's products (counted slices): both match
    the oracle vector by vector."""
    A, M = s20
    deg = A.degrees()
    sizes = synth.log_uniform_sizes(64, A.n / 4, seed=4100)
    xs = [synth.sparse_x(A.n, int(f), seed=5000 + k) for k, f in enumerate(sizes)]
    off = np.zeros(65, np.int64)
    off[1:] = np.cumsum(sizes)
    Wt = int(sum(int(deg[x[0]].sum()) for x in xs))
    off_d = dev(off)
    cat_i = dev(np.concatenate([x[0] for x in xs]))
    cat_v = dev(np.concatenate([x[1] for x in xs]))
    cap = int(min(64 * A.m, Wt)) + 1
    by_idx = torch.empty(cap, dtype=torch.int32, device="cuda")
    by_val = torch.empty(cap, dtype=torch.float32, device="cuda")
    by_off = torch.empty(65, dtype=torch.int64, device="cuda")
    ref = [oracle.spmspv(A, S, xv)[:2] for S, xv in xs]
    for mp in (64 * A.nnz, Wt):
        M.attach_batch(64, max_f=int(off[-1]), max_products=mp)
        if mp != Wt:
            spv.spmspv_autotune_batch(M.handle, 0, 0, 64, off_d, cat_i, cat_v, by_off, by_idx, by_val, cap, reps=1)
        total = spv.spmspv_run_batch(M.handle, 0, 0, 64, off_d, cat_i, cat_v, by_off, by_idx, by_val, cap, sync=True)
        yo = to_np(by_off)
        assert yo[0] == 0 and yo[-1] == total
        for b, (oi, ov) in enumerate(ref):
            compare(0, by_idx[yo[b]:yo[b + 1]], by_val[yo[b]:yo[b + 1]], oi, ov)
        assert M.last_stats()["err"] == 0
    M.batch_ws = None


def test_full_size_64_source_bfs(spv, s20):
    A, M = s20
    roots = synth.roots(A, 64, seed=2000)
    P = spv.Matrix(A.m, A.n, M.colptr, M.rowids, None, flags=spv.SYMMETRIC)
    P.attach_batch(64, msbfs=True)
    lev, par, nl = P.msbfs(roots)
    lev, par = to_np(lev), to_np(par)
    onl = 0
    for k in (0, 1, 31, 63):
        olev, opar, n_k = oracle.bfs(A, int(roots[k]))
        onl = max(onl, n_k)
        assert np.array_equal(lev[k], olev)
        assert np.array_equal(par[k], opar)
    assert nl >= onl
    P.close()


def test_full_size_held_out_bfs_learned_and_heuristic(spv):
    """The selector evaluation's held-out graph (R-MAT scale 24, 16.8M
    vertices, 521M stored entries): BFS with the trained selector consuming
    its direction on the device inside the captured level graph, with the
    host-read selector and with the frontier-edge heuristic, against the
    queue BFS from one of the evaluation's roots."""
    from paper_1610_07902_amd import selector
    A = rmat24_pattern()
    P = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    params, mean, std, _ = selector.load_weights()
    P.load_selector(params, mean, std)
    r = int(synth.roots(A, 16, seed=2000)[0])
    olev, opar, onl = oracle.bfs(A, r)
    for fl in (spv.USE_SELECTOR | spv.USE_GRAPH, spv.USE_SELECTOR, spv.USE_GRAPH | spv.DIRECTION_OPT):
        lev, par, nl = P.bfs(r, spv.MIN_SELECT2ND_I32, flags=fl)
        assert nl == onl
        assert np.array_equal(to_np(lev), olev)
        assert np.array_equal(to_np(par), opar)
    P.close()
