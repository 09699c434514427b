"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact for min-select2nd int32, or-and bool and every output index set;
fp32 plus-times within 1e-5 relative of the oracle's fp64 sums.  Sizes span
many buckets and scatter chunks with ragged tails; the edge cases cover
empty input, empty columns, rectangular matrices, unit vectors, permutation
matrices, a hub row, bucket sizes above the register-resident limit,
unsorted row ids, small output capacity and invalid input.

Every test runs twice: with the three-launch pipeline (scan, bucketing,
merge) and with the one-launch cooperative kernel (schedule field launch =
1 and 2).
"""
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


LAUNCH = {"mode": 1}


@pytest.fixture(scope="module", autouse=True, params=[1, 2], ids=["three_launches", "one_launch"])
def launch(request):
    LAUNCH["mode"] = request.param
    yield request.param
    LAUNCH["mode"] = 1


def make(spv, A, **kw):
    """Matrix handle whose push calls take the module's launch mode."""
    M = spv.Matrix.from_csc(A, **kw)
    set_launch(M)
    return M


def set_launch(M):
    s = M.schedule
    s.launch = LAUNCH["mode"]
    M.schedule = s


@pytest.fixture(scope="module")
def c1(spv, launch):
    """R-MAT scale 14, edge factor 16, directed, fp32 values (0, 1]."""
    A = synth.rmat(14, seed=1)
    return A, make(spv, A)


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def run_and_compare(spv, M, A, S, semiring, xval, sorted_output=False, flags=0, mask=None):
    x_idx = dev(S, torch.int32)
    x_val = None if xval is None else dev(xval)
    gi, gv, nnz = M.spmspv(x_idx, x_val, semiring=semiring, sorted_output=sorted_output, flags=flags)
    if semiring == spv.MIN_SELECT2ND_I32 and xval is None:
        oxv = S.astype(np.int32)
    elif semiring == spv.OR_AND_BOOL and xval is None:
        oxv = np.ones(S.size, np.uint8)
    else:
        oxv = xval
    oi, ov, W = oracle.spmspv(A, S, oxv, semiring, sorted_output=sorted_output)
    compare(semiring, gi, gv, oi, ov, sorted_output)
    st = M.last_stats()
    assert st["W"] == W and st["nnz_y"] == nnz == oi.size and st["err"] == 0
    return nnz, W


@pytest.mark.parametrize("sorted_output", [False, True])
def test_c1_plus_times(spv, c1, sorted_output):
    A, M = c1
    S, xv = synth.sparse_x(A.n, 164, seed=1000)
    run_and_compare(spv, M, A, S, spv.PLUS_TIMES_F32, xv, sorted_output)


@pytest.mark.parametrize("f", [1, 7, 164, 1638, 8000, 16384])
@pytest.mark.parametrize("semiring", [0, 1, 2])
def test_c1_densities_all_semirings(spv, c1, f, semiring):
    A, M = c1
    S, xv = synth.sparse_x(A.n, f, seed=1100 + f)
    if semiring == 0:
        xval = xv
    elif semiring == 1:
        xval = np.random.default_rng(f).integers(-(1 << 30), 1 << 30, f).astype(np.int32)
    else:
        xval = (np.random.default_rng(f).random(f) < 0.7).astype(np.uint8)
    run_and_compare(spv, M, A, S, semiring, xval, sorted_output=bool(f % 2))


def test_x_value_modes(spv, c1):
    A, M = c1
    S, _ = synth.sparse_x(A.n, 900, seed=77)
    run_and_compare(spv, M, A, S, spv.MIN_SELECT2ND_I32, None, flags=spv.X_VAL_IS_INDEX)
    run_and_compare(spv, M, A, S, spv.OR_AND_BOOL, None, flags=spv.X_ALL_TRUE, sorted_output=True)


@pytest.mark.parametrize("sched", [(8, 256, 4, 256), (9, 256, 16, 512), (10, 512, 4, 256), (11, 512, 8, 512),
                                   (12, 1024, 4, 256), (13, 256, 8, 256)])
def test_schedule_invariance(spv, c1, sched):
    """Int results and index sets do not depend on the schedule."""
    A, M = c1
    tl, sb, si, mb = sched
    s = spv.Schedule(0, tl, sb, si, mb, 0, LAUNCH["mode"])
    M.schedule = s
    try:
        assert M.schedule.as_dict() == s.as_dict()
        for f in (50, 3000, 16384):
            S, xv = synth.sparse_x(A.n, f, seed=500 + f)
            run_and_compare(spv, M, A, S, spv.MIN_SELECT2ND_I32, S.astype(np.int32), sorted_output=True)
            run_and_compare(spv, M, A, S, spv.PLUS_TIMES_F32, xv)
    finally:
        M.schedule = None
        set_launch(M)


@pytest.mark.parametrize("sb", [256, 512])
def test_more_buckets_than_scatter_threads(spv, sb):
    """512 buckets: with 256 scatter threads each thread reserves slots for
    two buckets (the looped reservation), with 512 for one (the reservation
    that overlaps the LDS sort)."""
    A = synth.rmat(17, seed=17, symmetrize=True)
    M = make(spv, A)
    M.schedule = spv.Schedule(0, 8, sb, 4, 256, 0, LAUNCH["mode"])
    assert (A.m + 255) // 256 == 512
    for f in (40, 2000, 60000):
        S, xv = synth.sparse_x(A.n, f, seed=900 + f)
        run_and_compare(spv, M, A, S, spv.PLUS_TIMES_F32, xv, sorted_output=True)
        run_and_compare(spv, M, A, S, spv.MIN_SELECT2ND_I32, S.astype(np.int32))


def test_empty_x_and_empty_columns(spv, c1):
    A, M = c1
    x = torch.empty(0, dtype=torch.int32, device="cuda")
    gi, gv, nnz = M.spmspv(x, torch.empty(0, dtype=torch.float32, device="cuda"))
    assert nnz == 0
    empty_cols = np.nonzero(A.degrees() == 0)[0][:500].astype(np.int32)
    assert empty_cols.size > 100
    gi, gv, nnz = M.spmspv(dev(empty_cols), dev(np.ones(empty_cols.size, np.float32)))
    assert nnz == 0 and M.last_stats()["W"] == 0


@pytest.mark.parametrize("shape", [(3000, 1000), (500, 5000), (1, 300), (300, 1)])
def test_rectangular(spv, shape):
    m, n = shape
    rng = np.random.default_rng(m * 7 + n)
    nt = 8 * max(m, n)
    rows = rng.integers(0, m, nt).astype(np.int32)
    cols = rng.integers(0, n, nt).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(m, n, rows, cols, drop_self=False)
    A = synth.CSC(m, n, colptr, rowids, synth.values(rowids.size, 3))
    M = make(spv, A)
    for f in sorted({1, max(1, n // 10), n}):
        S, xv = synth.sparse_x(n, f, seed=f)
        run_and_compare(spv, M, A, S, spv.PLUS_TIMES_F32, xv, sorted_output=True)
        run_and_compare(spv, M, A, S, spv.MIN_SELECT2ND_I32, rng.integers(0, 99, f).astype(np.int32))


def test_unit_vectors_bit_exact(spv, c1):
    A, M = c1
    for j in [0, 17, int(np.argmax(A.degrees()))]:
        gi, gv, nnz = M.spmspv(dev(np.array([j], np.int32)), dev(np.ones(1, np.float32)), sorted_output=True)
        col = A.rowids[A.colptr[j]:A.colptr[j + 1]]
        o = np.argsort(col)
        assert np.array_equal(to_np(gi), col[o])
        assert np.array_equal(to_np(gv), A.values[A.colptr[j]:A.colptr[j + 1]][o])


def test_permutation_matrix_bit_exact(spv):
    n = 100000
    perm = np.random.default_rng(3).permutation(n).astype(np.int32)
    A = synth.CSC(n, n, np.arange(n + 1, dtype=np.int32), perm, synth.values(n, 5))
    M = make(spv, A)
    S, xv = synth.sparse_x(n, 40000, seed=9)
    gi, gv, nnz = M.spmspv(dev(S), dev(xv), sorted_output=True)
    o = np.argsort(perm[S])
    assert np.array_equal(to_np(gi), perm[S][o])
    assert np.array_equal(to_np(gv), (A.values[S] * xv)[o].astype(np.float32))   # RN32(a * x)


def test_hub_row_and_large_buckets(spv):
    """One row present in every column (n hits on one accumulator cell), and
    buckets far beyond the register-resident entry count."""
    n = 20000
    rng = np.random.default_rng(1)
    rows = np.concatenate([np.full(n, 12345), rng.integers(0, n, 6 * n)]).astype(np.int32)
    cols = np.concatenate([np.arange(n), rng.integers(0, n, 6 * n)]).astype(np.int32)
    colptr, rowids = synth.coo_to_csc(n, n, rows, cols, drop_self=False)
    A = synth.CSC(n, n, colptr, rowids, synth.values(rowids.size, 8))
    M = make(spv, A)
    for tl in (8, 12):
        M.schedule = spv.Schedule(0, tl, 256, 8, 256, 0, LAUNCH["mode"])
        S, xv = synth.sparse_x(n, n, seed=2)
        run_and_compare(spv, M, A, S, spv.PLUS_TIMES_F32, xv)
        run_and_compare(spv, M, A, S, spv.MIN_SELECT2ND_I32, S.astype(np.int32), sorted_output=True)
        run_and_compare(spv, M, A, S, spv.OR_AND_BOOL, np.ones(n, np.uint8))


def test_unsorted_rowids_and_zero_values(spv):
    rng = np.random.default_rng(4)
    A = synth.rmat(12, seed=4)
    rowids = A.rowids.copy()
    for j in range(A.n):
        seg = rowids[A.colptr[j]:A.colptr[j + 1]]
        rng.shuffle(seg)
    vals = A.values.copy()
    vals[rng.random(vals.size) < 0.3] = 0.0
    B = synth.CSC(A.m, A.n, A.colptr, rowids, vals)
    M = make(spv, B)
    S, xv = synth.sparse_x(A.n, 1500, seed=6)
    run_and_compare(spv, M, B, S, spv.PLUS_TIMES_F32, xv)
    run_and_compare(spv, M, B, S, spv.OR_AND_BOOL, (rng.random(S.size) < 0.5).astype(np.uint8), sorted_output=True)
    run_and_compare(spv, M, B, S, spv.MIN_SELECT2ND_I32, S.astype(np.int32))


def test_pattern_matrix(spv):
    A = synth.rmat(13, seed=2, with_values=False)
    M = make(spv, A)
    S, xv = synth.sparse_x(A.n, 800, seed=3)
    run_and_compare(spv, M, A, S, spv.PLUS_TIMES_F32, xv)
    run_and_compare(spv, M, A, S, spv.OR_AND_BOOL, None, flags=spv.X_ALL_TRUE)


def test_capacity_reporting(spv, c1):
    A, M = c1
    S, xv = synth.sparse_x(A.n, 2000, seed=12)
    oi, _, _ = oracle.spmspv(A, S, xv)
    need = oi.size
    cap = need // 2
    y_idx = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    y_val = torch.empty(cap, dtype=torch.float32, device="cuda")
    with pytest.raises(spv.SpmspvError) as e:
        spv.spmspv_run(M.handle, 0, 0, S.size, dev(S), dev(xv), y_idx, y_val, cap)
    assert e.value.status == spv.ECAPACITY
    assert M.last_stats()["nnz_y"] == need
    assert int((y_idx == -7).sum()) == 0          # the first `cap` slots were written
    assert set(to_np(y_idx).tolist()) <= set(oi.tolist())
    # exact capacity succeeds
    y_idx = torch.empty(need, dtype=torch.int32, device="cuda")
    y_val = torch.empty(need, dtype=torch.float32, device="cuda")
    assert spv.spmspv_run(M.handle, 0, 0, S.size, dev(S), dev(xv), y_idx, y_val, need) == need


def test_invalid_inputs(spv, c1):
    A, M = c1
    y = torch.empty(A.m, dtype=torch.int32, device="cuda")
    yv = torch.empty(A.m, dtype=torch.float32, device="cuda")
    ones = dev(np.ones(3, np.float32))
    for bad in ([1, 1, 2], [0, A.n, 3], [-1, 2, 3]):
        with pytest.raises(spv.SpmspvError) as e:
            spv.spmspv_run(M.handle, 0, spv.VALIDATE, 3, dev(np.array(bad, np.int32)), ones, y, yv, A.m)
        assert e.value.status == spv.EINVAL
    # without validation an out-of-range index is caught on the device
    with pytest.raises(spv.SpmspvError) as e:
        spv.spmspv_run(M.handle, 0, 0, 3, dev(np.array([0, A.n + 5, 3], np.int32)), ones, y, yv, A.m)
    assert e.value.status == spv.EDEVICE
    # and the handle keeps working afterwards
    S, xv = synth.sparse_x(A.n, 164, seed=1000)
    run_and_compare(spv, M, A, S, spv.PLUS_TIMES_F32, xv)
    with pytest.raises(spv.SpmspvError):
        spv.spmspv_run(M.handle, 5, 0, 3, dev(np.array([0, 1, 2], np.int32)), ones, y, yv, A.m)


def test_duplicate_x_is_memory_safe(spv):
    """Duplicated x indices break the distinctness precondition.  The three
    launches' buckets may overflow, which the device reports while staying
    inside the workspace; the one launch has no per-bucket capacity and
    combines the repeated products like any others (as the oracle does),
    reporting an error only when the products outnumber A's stored entries."""
    n = 4096
    colptr = np.arange(n + 1, dtype=np.int32)
    A = synth.CSC(n, n, colptr, np.arange(n, dtype=np.int32), np.ones(n, np.float32))   # identity
    M = make(spv, A)
    S = np.full(3000, 7, np.int32)   # the same column 3000 times: row 7's bucket holds 2^tile_log2 slots
    y = torch.empty(n, dtype=torch.int32, device="cuda")
    yv = torch.empty(n, dtype=torch.float32, device="cuda")
    if LAUNCH["mode"] == 1:
        with pytest.raises(spv.SpmspvError) as e:
            spv.spmspv_run(M.handle, 0, 0, S.size, dev(S), dev(np.ones(S.size, np.float32)), y, yv, n)
        assert e.value.status == spv.EDEVICE
    else:
        nnz = spv.spmspv_run(M.handle, 0, 0, S.size, dev(S), dev(np.ones(S.size, np.float32)), y, yv, n)
        assert nnz == 1 and int(y[0]) == 7 and float(yv[0]) == 3000.0
        # column 0 with ten entries selected n times: more products than A stores
        cp = np.concatenate([[0], np.arange(10, n + 10)]).astype(np.int32)
        ri = np.concatenate([np.arange(10), np.arange(1, n)]).astype(np.int32)
        M5 = make(spv, synth.CSC(n, n, cp, ri, np.ones(ri.size, np.float32)))
        S5 = np.zeros(n, np.int32)
        with pytest.raises(spv.SpmspvError) as e:
            spv.spmspv_run(M5.handle, 0, 0, S5.size, dev(S5), dev(np.ones(S5.size, np.float32)), y, yv, n)
        assert e.value.status == spv.EDEVICE
    S2, xv = synth.sparse_x(n, 100, seed=1)
    run_and_compare(spv, M, A, S2, spv.PLUS_TIMES_F32, xv)


def test_invalid_csc_rejected(spv):
    colptr = np.array([0, 2, 1, 3], np.int32)        # not monotone
    rowids = np.array([0, 1, 2], np.int32)
    with pytest.raises(spv.SpmspvError) as e:
        spv.Matrix(3, 3, colptr, rowids, None, flags=spv.VALIDATE)
    assert e.value.status == spv.EINVAL
    with pytest.raises(spv.SpmspvError):
        spv.Matrix(3, 3, np.array([0, 1, 2, 3], np.int32), np.array([0, 3, 1], np.int32), None)


def test_profile_and_stats(spv, c1):
    A, M = c1
    S, xv = synth.sparse_x(A.n, 164, seed=1000)
    for _ in range(5):
        M.spmspv(dev(S), dev(xv), flags=spv.PROFILE)
    ms, calls = spv.spmspv_profile_read(M.handle)
    assert calls == 5 and ms[0] > 0
    if LAUNCH["mode"] == 1:
        assert all(t > 0 for t in ms)
    st = M.last_stats()
    assert st["W"] == int(A.degrees()[S].sum()) and st["maxlen"] == int(A.degrees()[S].max())
