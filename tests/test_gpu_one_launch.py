"""GPU parity of the one-launch multiply (schedule launch = 2) against the
oracle, on the shapes its exchanges and chunking have to get right:

* more products than one chunk per workgroup (several chunks per workgroup,
  and more chunk runs than one merge index group holds);
* more buckets than workgroups (several buckets per merge workgroup);
* fewer x entries than workgroups, a single column spanning many chunks, x
  selecting every column (sample strides above one), empty products;
* masks, rectangular matrices, all three semirings;
* long sequences of calls on one handle (the tags advance every call),
  alternating with three-launch calls that share the workspace.

Bit-exact for int32, bool and every index set; fp32 within 1e-5 of the fp64
sum."""
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


def one_launch(spv, A, tile=None, launch=2, **kw):
    M = spv.Matrix.from_csc(A, **kw)
    s = M.schedule
    s.launch = launch
    if tile is not None:
        s.tile_log2 = tile
    M.schedule = s
    return M


def xval_for(semiring, S, xv):
    if semiring == 0:
        return xv
    if semiring == 1:
        return np.random.default_rng(S.size).integers(-(1 << 30), 1 << 30, S.size).astype(np.int32)
    return (np.random.default_rng(S.size + 1).random(S.size) < 0.7).astype(np.uint8)


def check(spv, M, A, S, xv, semiring=0, sorted_output=True, mask=None, mask_np=None):
    xval = xval_for(semiring, S, xv)
    gi, gv, nnz = M.spmspv(dev(S), dev(xval), semiring=semiring, sorted_output=sorted_output, mask=mask)
    oi, ov, W = oracle.spmspv(A, S, xval, semiring, sorted_output=sorted_output, mask=mask_np)
    compare(semiring, gi, gv, oi, ov, sorted_output=sorted_output)
    st = M.last_stats()
    assert st["err"] == 0 and st["W"] == W and nnz == oi.size
    return W


@pytest.fixture(scope="module")
def s20():
    return synth.rmat(20, 16, seed=20, symmetrize=True)


def test_many_chunks_per_workgroup_and_run_groups(spv, s20):
    """40 % of the columns of R-MAT scale 20: about 12.5M products, so 8192-
    product chunks number about 1,500 (six per workgroup) and every merge
    indexes its runs in two groups of 1024."""
    A = s20
    M = one_launch(spv, A)
    S, xv = synth.sparse_x(A.n, int(0.4 * A.n), seed=71)
    W = check(spv, M, A, S, xv, semiring=0)
    assert W > 1024 * 8192
    check(spv, M, A, S, xv, semiring=1)
    M.close()


def test_every_column(spv, s20):
    """x = every column (f = n = 1,048,576 = 4096 per workgroup, the largest
    slice; list sample stride 64): all 31.4M stored entries are products."""
    A = s20
    M = one_launch(spv, A)
    S = np.random.default_rng(5).permutation(A.n).astype(np.int32)
    xv = synth.values(A.n, 72)
    W = check(spv, M, A, S, xv, semiring=0, sorted_output=False)
    assert W == A.nnz
    check(spv, M, A, S, xv, semiring=2)
    M.close()


def test_more_buckets_than_workgroups(spv):
    """m = 2^18 with 256-row buckets: 1024 buckets, four per workgroup."""
    A = synth.rmat(18, 16, seed=73, symmetrize=True)
    M = one_launch(spv, A, tile=8)
    for f, sr in ((2621, 0), (26214, 1), (26214, 2), (100, 0)):
        S, xv = synth.sparse_x(A.n, f, seed=74 + f)
        check(spv, M, A, S, xv, semiring=sr)
    M.close()


@pytest.mark.parametrize("f", [0, 1, 3, 100, 255, 257])
def test_fewer_x_than_workgroups(spv, f):
    A = synth.rmat(16, 16, seed=75, symmetrize=True)
    M = one_launch(spv, A)
    S, xv = synth.sparse_x(A.n, f, seed=76 + f)
    for sr in (0, 1, 2):
        check(spv, M, A, S, xv, semiring=sr)
    M.close()


def test_one_column_spans_many_chunks(spv):
    """x = the longest column alone, then with a few short ones: one source
    workgroup holds every product, and every chunk's columns come from it."""
    A = synth.rmat(18, 16, seed=77, symmetrize=True)
    M = one_launch(spv, A)
    deg = A.degrees()
    hub = int(np.argmax(deg))
    assert deg[hub] > 5000
    S = np.array([hub], np.int32)
    check(spv, M, A, S, synth.values(1, 78), semiring=0)
    rng = np.random.default_rng(79)
    S = np.unique(np.concatenate([[hub], rng.integers(0, A.n, 30)])).astype(np.int32)
    rng.shuffle(S)
    for sr in (0, 1):
        check(spv, M, A, S, synth.values(S.size, 80), semiring=sr)
    empty = np.nonzero(deg == 0)[0][:300].astype(np.int32)
    gi, gv, nnz = M.spmspv(dev(empty), dev(np.ones(empty.size, np.float32)))
    assert nnz == 0 and M.last_stats()["W"] == 0
    M.close()


def test_mask(spv):
    A = synth.rmat(17, 16, seed=81, symmetrize=True)
    M = one_launch(spv, A)
    rng = np.random.default_rng(82)
    drop = rng.random(A.m) < 0.4
    words = np.zeros((A.m + 31) // 32, np.uint32)
    for i in np.nonzero(drop)[0]:
        words[i >> 5] |= np.uint32(1) << np.uint32(i & 31)
    S, xv = synth.sparse_x(A.n, 3000, seed=83)
    for sr in (0, 1, 2):
        check(spv, M, A, S, xv, semiring=sr, mask=dev(words.view(np.int32)), mask_np=drop.astype(np.uint8))
    M.close()


@pytest.mark.parametrize("shape", [(300000, 5000), (5000, 300000)])
def test_rectangular(spv, shape):
    m, n = shape
    rng = np.random.default_rng(m)
    k = 2_000_000
    rows = rng.integers(0, m, k).astype(np.int32)
    cols = rng.integers(0, n, k).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(m, n, rows, cols, drop_self=False)
    A = synth.CSC(m, n, colptr, rowids, synth.values(rowids.size, 84))
    M = one_launch(spv, A)
    for f in (1, min(n, 4000), n):
        S, xv = synth.sparse_x(n, f, seed=85 + f)
        check(spv, M, A, S, xv, semiring=0)
        check(spv, M, A, S, xv, semiring=1, sorted_output=False)
    M.close()


def test_call_sequences_share_the_workspace(spv):
    """200 calls on one handle with sizes from 0 to 30,000 x entries,
    alternating one-launch and three-launch calls on the same stream; the
    last dozen outputs of each kind are checked."""
    A = synth.rmat(17, 16, seed=86, symmetrize=True)
    M1 = one_launch(spv, A)
    rng = np.random.default_rng(87)
    sizes = rng.integers(0, 30000, 200)
    sizes[::17] = 0
    keep = []
    for c, f in enumerate(sizes):
        mode = 2 if c % 3 else 1
        s = M1.schedule
        s.launch = mode
        M1.schedule = s
        S, xv = synth.sparse_x(A.n, int(f), seed=1000 + c)
        out = (torch.empty(A.m, dtype=torch.int32, device="cuda"), torch.empty(A.m, dtype=torch.float32,
                                                                               device="cuda"))
        _, _, d = M1.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True, out=out, sync=False)
        if c >= 176:
            keep.append((S, xv, out, d.clone()))
    torch.cuda.synchronize()
    assert M1.last_stats()["err"] == 0
    for S, xv, (yi, yv), d in keep:
        k = int(to_np(d)[0])
        oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
        compare(0, yi[:k], yv[:k], oi, ov, sorted_output=True)
    M1.close()


def test_unsupported_forced_one_launch(spv):
    """launch = 2 on a call it cannot take (more buckets than a row of run
    offsets holds) is refused with EUNSUPPORTED; the default runs it."""
    A = synth.rmat(19, 8, seed=88, symmetrize=True)
    M = one_launch(spv, A, tile=8)            # 2048 buckets
    S, xv = synth.sparse_x(A.n, 500, seed=89)
    with pytest.raises(spv.SpmspvError) as e:
        M.spmspv(dev(S), dev(xv))
    assert e.value.status == spv.EUNSUPPORTED
    s = M.schedule
    s.launch = 0
    M.schedule = s
    assert spv.spmspv_effective_schedule(M.handle, 500).launch == 1
    check(spv, M, A, S, xv, semiring=0)
    M.close()
