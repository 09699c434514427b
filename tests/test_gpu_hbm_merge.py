"""GPU parity of merge variant 1 (the sparse accumulator in HBM: dense cells
for every row updated with global atomics, then walked in row order)
against the oracle: every semiring over bucket widths from 2^8 rows to one
bucket for the whole matrix; semirings alternating on one handle (the cells
must be left empty for the next call, whatever its semiring); BFS, masks,
the GraphBLAS rules, left multiplication and bitvector calls through it; the
bucket counts of the selector's widest classes as explicit HBM schedules;
and the benchmark's scale-22 graph with 16 buckets.

Index sets and int32 / bool values bit-exact; fp32 within 1e-5 of the fp64
oracle (values positive)."""
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


def hbm(spv, M, tl):
    s = M.schedule
    s.direction = 0
    s.tile_log2 = tl
    s.merge_variant = 1
    M.schedule = s


def xfor(semiring, S, xv):
    if semiring == 0:
        return xv, 0
    if semiring == 1:
        return None, 4       # X_VAL_IS_INDEX
    return None, 8           # X_ALL_TRUE


def oracle_x(semiring, S, xv):
    if semiring == 0:
        return xv
    if semiring == 1:
        return S.astype(np.int32)
    return np.ones(S.size, np.uint8)


@pytest.fixture(scope="module")
def r16(spv):
    A = synth.rmat(16, 16, seed=91, symmetrize=True)
    M = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE)
    yield A, M
    M.close()


@pytest.mark.parametrize("tl", [8, 12, 15, 16, 30])
@pytest.mark.parametrize("semiring", [0, 1, 2])
def test_against_oracle(spv, r16, tl, semiring):
    A, M = r16
    hbm(spv, M, tl)
    rng = np.random.default_rng(tl * 3 + semiring)
    for f in (1, 60, A.n // 100, A.n // 5, A.n):
        S, xv = synth.sparse_x(A.n, f, seed=int(rng.integers(1 << 30)))
        v, fl = xfor(semiring, S, xv)
        gi, gv, nnz = M.spmspv(dev(S), None if v is None else dev(v), semiring=semiring, sorted_output=True,
                               flags=fl)
        oi, ov, _ = oracle.spmspv(A, S, oracle_x(semiring, S, xv), semiring, sorted_output=True)
        assert nnz == oi.size
        compare(semiring, gi, gv, oi, ov, sorted_output=True)
    assert M.last_stats()["err"] == 0
    M.schedule = None


def test_semirings_alternate_on_one_handle(spv, r16):
    """Each call leaves the HBM cells empty for the next one, whatever its
    semiring; LDS-merged calls in between do not touch them."""
    A, M = r16
    rng = np.random.default_rng(5)
    for k in range(12):
        semiring = int(rng.integers(0, 3))
        hbm(spv, M, int(rng.choice([9, 14, 17, 30])))
        if k % 4 == 3:
            M.schedule = None        # an LDS-merged call in between
        S, xv = synth.sparse_x(A.n, int(rng.integers(1, A.n // 4)), seed=100 + k)
        v, fl = xfor(semiring, S, xv)
        gi, gv, _ = M.spmspv(dev(S), None if v is None else dev(v), semiring=semiring, sorted_output=True,
                             flags=fl)
        oi, ov, _ = oracle.spmspv(A, S, oracle_x(semiring, S, xv), semiring, sorted_output=True)
        compare(semiring, gi, gv, oi, ov, sorted_output=True)
    M.schedule = None


@pytest.mark.parametrize("semiring", [1, 2])
def test_bfs(spv, semiring):
    A = synth.rmat(15, 8, seed=92, symmetrize=True)
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    for tl, flags in ((18, 0), (11, spv.USE_GRAPH), (16, spv.USE_GRAPH | spv.DIRECTION_OPT)):
        hbm(spv, M, tl)
        for root in synth.roots(A, 3, seed=tl):
            lev, par, nl = M.bfs(int(root), semiring=semiring, flags=flags)
            olev, opar, onl = oracle.bfs(A, int(root))
            assert nl == onl and np.array_equal(to_np(lev), olev)
            if semiring == 1:
                assert np.array_equal(to_np(par), opar)
    M.close()


def test_masked_graphblas_left_bitvector(spv, r16):
    A, M = r16
    hbm(spv, M, 13)
    rng = np.random.default_rng(6)
    S, xv = synth.sparse_x(A.n, 3000, seed=7)
    drop = rng.random(A.m) < 0.4
    words = np.zeros((A.m + 31) // 32, np.uint32)
    for i in np.nonzero(drop)[0]:
        words[i >> 5] |= np.uint32(1 << (i & 31))
    gi, gv, _ = M.spmspv(dev(S), dev(xv), sorted_output=True, mask=dev(words.view(np.int32)))
    oi, ov, _ = oracle.spmspv(A, S, xv, 0, mask=drop.astype(np.uint8), sorted_output=True)
    compare(0, gi, gv, oi, ov, sorted_output=True)
    # GraphBLAS: structural mask, accumulate with min
    mi = rng.permutation(A.m)[: A.m // 2].astype(np.int32)
    wi = np.sort(rng.permutation(A.m)[: A.m // 8]).astype(np.int32)
    wv = rng.integers(0, 1000, wi.size).astype(np.int32)
    y = torch.empty(A.m, dtype=torch.int32, device="cuda")
    yv = torch.empty(A.m, dtype=torch.int32, device="cuda")
    k = spv.spmspv_run_graphblas(M.handle, 1, spv.X_VAL_IS_INDEX, S.size, dev(S), None, dev(mi), None, mi.size, 0,
                                 spv.ACCUM_ADD, dev(wi), dev(wv), wi.size, y, yv, A.m)
    oi, ov = oracle.spmspv_graphblas(A, S, S.astype(np.int32), 1, mask_idx=mi, w_idx=wi, w_val=wv,
                                     accum=oracle.ACCUM_ADD)
    assert np.array_equal(to_np(y[:k]), oi) and np.array_equal(to_np(yv[:k]), ov)
    # left multiplication through the CSR copy
    gi, gv, _ = M.spmspv(dev(S), dev(xv), sorted_output=True, flags=spv.LEFT)
    oi, ov = oracle.spmspv_left(A, S, xv, 0)
    compare(0, gi, gv, oi, ov, sorted_output=True)
    # bitvector x / y
    Ss = np.sort(S)
    bits, _ = oracle.to_bitvector(Ss, None, A.n)
    yb, yv2, nnz = M.spmspv_bitvector(dev(bits.view(np.int32)), dev(xv[np.argsort(S)]))
    oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
    assert np.array_equal(oracle.from_bitvector(to_np(yb).view(np.uint32), A.m), oi)
    compare(0, torch.as_tensor(oi), yv2, oi, ov, sorted_output=True)
    M.schedule = None


def test_selector_classes_and_explicit_hbm_schedules(spv):
    """On a matrix with 2^22 rows the selector's classes are LDS tiles (2^15
    at most, 2^14 for plus-times); the same bucket counts as explicit HBM
    schedules (tiles 2^18 .. 2^16) give the same results."""
    rng = np.random.default_rng(8)
    m, n = 1 << 22, 4096
    colptr, rowids = synth.coo_to_csc(m, n, rng.integers(0, m, 400000).astype(np.int32),
                                      rng.integers(0, n, 400000).astype(np.int32), drop_self=False)
    A = synth.CSC(m, n, colptr, rowids, synth.values(rowids.size, 9))
    M = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE)
    S, xv = synth.sparse_x(n, 300, seed=10)
    oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
    for c in range(9):
        s = spv.spmspv_class_schedule(M.handle, 0, c)
        assert s.merge_variant == 0 and s.tile_log2 == min(18 - c, 14)
        s1 = spv.spmspv_class_schedule(M.handle, 1, c)
        assert s1.merge_variant == 0 and s1.tile_log2 == min(18 - c, 15)
        M.schedule = s
        gi, gv, _ = M.spmspv(dev(S), dev(xv), sorted_output=True)
        compare(0, gi, gv, oi, ov, sorted_output=True)
    for tl in (18, 17, 16):
        hbm(spv, M, tl)
        gi, gv, _ = M.spmspv(dev(S), dev(xv), sorted_output=True)
        compare(0, gi, gv, oi, ov, sorted_output=True)
    assert spv.spmspv_class_schedule(M.handle, 0, 9).direction == 1
    M.close()


def test_full_size_rmat22_sixteen_buckets(spv):
    A = synth.rmat(22, 16, seed=1, symmetrize=True)
    M = spv.Matrix.from_csc(A)
    hbm(spv, M, 18)
    for density, seed in ((1e-2, 2), (1e-1, 3)):
        S, xv = synth.sparse_x(A.n, synth.density_f(A.n, density), seed=seed)
        gi, gv, _ = M.spmspv(dev(S), dev(xv), sorted_output=True)
        oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
        compare(0, gi, gv, oi, ov, sorted_output=True)
    M.close()
