"""The allocation-free multiply (spmspv_run_static: no handle, no workspace,
the library's own device scratch) against spmspv_run on a handle over the
same matrix, and against the oracle: two calls in a row, the second with a
smaller input (the scratch keeps the first call's contents), all three
semirings; then a smaller matrix after a larger one; capacity reporting
and the size limit.

Index sets and int / bool values bit-exact against the handle's output;
fp32 within the 1e-5 contract of the oracle's fp64 sums for both."""
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


VDT = {0: torch.float32, 1: torch.int32, 2: torch.uint8}


def x_for(semiring, S, xv):
    if semiring == 0:
        return xv
    if semiring == 1:
        return np.random.default_rng(S.size).integers(-(1 << 30), 1 << 30, S.size).astype(np.int32)
    return (np.random.default_rng(S.size).random(S.size) < 0.6).astype(np.uint8)


def run_static(spv, A, dA, S, xval, semiring, cap=None):
    cap = A.m if cap is None else cap
    y_idx = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    y_val = torch.empty(max(cap, 1), dtype=VDT[semiring], device="cuda")
    colptr, rowids, values = dA
    nnz = spv.spmspv_run_static(A.m, A.n, A.nnz, colptr, rowids, values, semiring, spv.SORTED_OUTPUT, S.size,
                                dev(S), dev(xval), y_idx, y_val, cap)
    return y_idx[:nnz], y_val[:nnz], nnz


def check_pair(spv, A, dA, M, S, xval, semiring):
    si, sv, snnz = run_static(spv, A, dA, S, xval, semiring)
    hi, hv, hnnz = M.spmspv(dev(S), dev(xval), semiring=semiring, sorted_output=True)
    assert snnz == hnnz
    assert np.array_equal(to_np(si), to_np(hi)), "index sets differ from spmspv_run"
    if semiring != 0:
        assert np.array_equal(to_np(sv), to_np(hv)), "values differ from spmspv_run"
    oi, ov, _ = oracle.spmspv(A, S, xval, semiring, sorted_output=True)
    compare(semiring, si, sv, oi, ov, sorted_output=True)
    compare(semiring, hi, hv, oi, ov, sorted_output=True)


@pytest.mark.parametrize("semiring", [0, 1, 2])
def test_static_matches_handle_on_two_calls(spv, semiring):
    A = synth.rmat(14, seed=1)   # R-MAT scale 14, edge factor 16, directed, fp32 values (0, 1]
    dA = (dev(A.colptr), dev(A.rowids), dev(A.values))
    M = spv.Matrix.from_csc(A)
    for f, seed in ((1638, 501), (164, 502)):   # the second call smaller
        S, xv = synth.sparse_x(A.n, f, seed=seed)
        check_pair(spv, A, dA, M, S, x_for(semiring, S, xv), semiring)
    M.close()


def test_static_smaller_matrix_after_larger(spv):
    big = synth.rmat(16, seed=5, symmetrize=True)
    small = synth.rmat(11, seed=6)
    for A, f in ((big, 6000), (small, 50)):
        dA = (dev(A.colptr), dev(A.rowids), dev(A.values))
        M = spv.Matrix.from_csc(A)
        S, xv = synth.sparse_x(A.n, f, seed=503 + f)
        check_pair(spv, A, dA, M, S, xv, 0)
        check_pair(spv, A, dA, M, S, x_for(1, S, xv), 1)
        M.close()


def test_static_capacity_and_limit(spv):
    A = synth.rmat(13, seed=7)
    dA = (dev(A.colptr), dev(A.rowids), dev(A.values))
    S, xv = synth.sparse_x(A.n, 2000, seed=504)
    oi, _, _ = oracle.spmspv(A, S, xv, sorted_output=True)
    cap = oi.size // 2
    with pytest.raises(spv.SpmspvError) as e:
        run_static(spv, A, dA, S, xv, 0, cap=cap)
    assert e.value.status == spv.ECAPACITY
    # still exact with room for y
    si, sv, nnz = run_static(spv, A, dA, S, xv, 0)
    assert nnz == oi.size and np.array_equal(to_np(si), oi)
    # a matrix whose workspace exceeds the 64 MiB scratch is refused before any device work
    m = n = 1 << 22
    assert spv.spmspv_static_scratch_need(m, n, 20_000_000) > (64 << 20)
    with pytest.raises(spv.SpmspvError) as e:
        spv.spmspv_run_static(m, n, 20_000_000, dA[0], dA[1], None, 0, 0, 0, None, None, None, None, 0)
    assert e.value.status == spv.EINVAL
