"""GPU parity of the masked multiply with accumulate and replace
(spmspv_run_graphblas: w<mask, replace> = w accum (A x)) against the oracle.

Every combination of mask kind (none, structural, value), complement,
accumulate operator (none, Add, first, second) and replace, in all three
semirings; masks and w of several densities; a scale-22 case at the
benchmark's size; and the error paths (unordered w, out-of-range mask rows,
small output capacity).

Index sets and int32 / bool values bit-exact; fp32 within 1e-5 of
|w| + sum|terms| (the product's contract, plus the one fp32 add of
accumulation)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VDT = {0: np.float32, 1: np.int32, 2: np.uint8}
TDT = {0: "float32", 1: "int32", 2: "uint8"}


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
def c1(spv):
    A = synth.rmat(14, seed=1)
    return A, spv.Matrix.from_csc(A)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def values_for(rng, semiring, k):
    if semiring == 0:
        return ((rng.integers(0, 1 << 24, k) + 1) / float(1 << 24)).astype(np.float32)
    if semiring == 1:
        return rng.integers(-(1 << 30), 1 << 30, k).astype(np.int32)
    return (rng.random(k) < 0.6).astype(np.uint8)


def run_gpu(spv, M, A, semiring, S, xv, mi, mv, mflags, accum, wi, wv, cap=None, flags=0):
    cap = A.m if cap is None else cap
    y_idx = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    y_val = torch.empty(max(cap, 1), dtype=getattr(torch, TDT[semiring]), device="cuda")
    nnz = spv.spmspv_run_graphblas(M.handle, semiring, flags, S.size, dev(S), dev(xv),
                                   None if mi is None else dev(mi), None if mv is None else dev(mv),
                                   0 if mi is None else mi.size, mflags, accum,
                                   dev(wi) if wi.size else None, dev(wv) if wi.size else None, wi.size,
                                   y_idx, y_val, cap)
    return to_np(y_idx[:nnz]), to_np(y_val[:nnz])


def check(spv, M, A, semiring, S, xv, mi, mv, comp, replace, accum, wi, wv):
    mflags = (spv.MASK_COMPLEMENT if comp else 0) | (spv.MASK_REPLACE if replace else 0)
    gi, gv = run_gpu(spv, M, A, semiring, S, xv, mi, mv, mflags, accum, wi, wv)
    ow = wv.astype(np.float64) if semiring == 0 else wv
    oi, ov = oracle.spmspv_graphblas(A, S, xv, semiring, mask_idx=mi, mask_val=mv, complement=comp, w_idx=wi,
                                     w_val=ow, accum=accum, replace=replace)
    assert np.all(np.diff(gi) > 0), "output not strictly ascending"
    assert np.array_equal(gi, oi), f"index sets differ ({gi.size} vs {oi.size})"
    if semiring == 0:
        ti, tv, _ = oracle.spmspv(A, S, xv, 0)
        t = np.zeros(A.m)
        t[ti] = np.abs(tv)
        w = np.zeros(A.m)
        w[wi] = np.abs(wv)
        bound = 1e-5 * (w[oi] + t[oi])
        err = np.abs(gv.astype(np.float64) - ov)
        assert np.all(err <= bound), f"worst {np.max(err - bound):.3e} over the bound"
    else:
        assert np.array_equal(gv.astype(np.int64), ov.astype(np.int64))
    return gi.size


CASES = [(sr, mk, comp, acc, rep) for sr in (0, 1, 2) for mk in ("none", "struct", "value")
         for comp in (False, True) for acc in (0, 1, 2, 3) for rep in (False, True)]


@pytest.mark.parametrize("semiring,mask,complement,accum,replace", CASES)
def test_every_combination(spv, c1, semiring, mask, complement, accum, replace):
    A, M = c1
    rng = np.random.default_rng(hash((semiring, mask, complement, accum, replace)) % (1 << 32))
    for f, wfrac, mfrac in ((164, 0.05, 0.3), (4000, 0.4, 0.7), (1, 0.0, 0.5)):
        S, xv0 = synth.sparse_x(A.n, f, seed=int(rng.integers(1 << 30)))
        xv = xv0 if semiring == 0 else values_for(rng, semiring, f)
        wi = np.sort(rng.permutation(A.m)[: int(wfrac * A.m)]).astype(np.int32)
        wv = values_for(rng, semiring, wi.size)
        mi = mv = None
        if mask != "none":
            mi = rng.permutation(A.m)[: int(mfrac * A.m)].astype(np.int32)
            if mask == "value":
                mv = (rng.random(mi.size) < 0.5).astype(np.uint8)
        check(spv, M, A, semiring, S, xv, mi, mv, complement, replace, accum, wi, wv)


def test_bfs_level_with_accumulated_parents_full_size(spv):
    """R-MAT scale 22 at 1 % density: the complement of a structural mask of
    visited rows (a BFS level) with min-select2nd, accumulating into w =
    earlier parents with Add (min) and replace off; and a value mask with
    plus-times accumulation."""
    A = synth.rmat(22, 16, seed=1, symmetrize=True)
    M = spv.Matrix.from_csc(A)
    rng = np.random.default_rng(2024)
    f = synth.density_f(A.n, 0.01)
    S, xv = synth.sparse_x(A.n, f, seed=2025)
    visited = rng.permutation(A.m)[: A.m // 4].astype(np.int32)
    wi = np.sort(visited[: visited.size // 2]).astype(np.int32)
    wv = rng.integers(0, A.n, wi.size).astype(np.int32)
    n1 = check(spv, M, A, 1, S, S.astype(np.int32), visited, None, True, False, 1, wi, wv)
    assert n1 > 100000
    mi = rng.permutation(A.m)[: A.m // 2].astype(np.int32)
    mv = (rng.random(mi.size) < 0.5).astype(np.uint8)
    wv2 = values_for(rng, 0, wi.size)
    check(spv, M, A, 0, S, xv, mi, mv, False, True, 1, wi, wv2)
    M.close()


def test_errors_and_capacity(spv, c1):
    A, M = c1
    S, xv = synth.sparse_x(A.n, 300, seed=77)
    wi = np.array([5, 3, 9], np.int32)                      # not ascending
    wv = np.ones(3, np.float32)
    with pytest.raises(spv.SpmspvError) as e:
        run_gpu(spv, M, A, 0, S, xv, None, None, 0, 1, wi, wv, flags=spv.VALIDATE)
    assert e.value.status == spv.EINVAL
    with pytest.raises(spv.SpmspvError) as e:                # caught on the device without VALIDATE
        run_gpu(spv, M, A, 0, S, xv, None, None, 0, 1, wi, wv)
    assert e.value.status == spv.EDEVICE
    with pytest.raises(spv.SpmspvError) as e:                # a mask row out of range
        run_gpu(spv, M, A, 0, S, xv, np.array([0, A.m + 3], np.int32), None, 0, 0, np.zeros(0, np.int32),
                np.zeros(0, np.float32))
    assert e.value.status == spv.EDEVICE
    # output capacity: the required size is reported, then an exact fit succeeds
    wi = np.arange(0, A.m, 3, dtype=np.int32)
    wv = np.ones(wi.size, np.float32)
    oi, _ = oracle.spmspv_graphblas(A, S, xv, 0, w_idx=wi, w_val=wv.astype(np.float64), accum=1)
    with pytest.raises(spv.SpmspvError) as e:
        run_gpu(spv, M, A, 0, S, xv, None, None, 0, 1, wi, wv, cap=oi.size - 1)
    assert e.value.status == spv.ECAPACITY
    gi, _ = run_gpu(spv, M, A, 0, S, xv, None, None, 0, 1, wi, wv, cap=oi.size)
    assert np.array_equal(gi, oi)
    # the handle keeps working for plain calls
    gi, gv, nnz = M.spmspv(dev(S), dev(xv), sorted_output=True)
    ti, tv, _ = oracle.spmspv(A, S, xv, sorted_output=True)
    assert np.array_equal(to_np(gi), ti)


@pytest.mark.parametrize("semiring", [0, 1])
def test_pairs_across_tile_boundaries(spv, semiring):
    """w holds every row of t plus others, so a w entry and its t partner
    sit next to each other all through the merged order and many pairs
    straddle a 2048-entry tile boundary; one case makes the merged length an
    exact multiple of the tile."""
    A = synth.rmat(16, 16, seed=5, symmetrize=True)
    M = spv.Matrix.from_csc(A)
    rng = np.random.default_rng(40 + semiring)
    for f, exact in ((3000, False), (40, True), (200, True)):
        S, xv0 = synth.sparse_x(A.n, f, seed=int(rng.integers(1 << 30)))
        xv = xv0 if semiring == 0 else values_for(rng, semiring, f)
        ti, _, _ = oracle.spmspv(A, S, xv, semiring, sorted_output=True)
        others = np.setdiff1d(np.arange(A.m, dtype=np.int32), ti)
        if exact:
            total = 2048 * ((2 * ti.size) // 2048 + 1)
            extra = total - 2 * ti.size
        else:
            extra = ti.size
        wi = np.sort(np.concatenate([ti, rng.choice(others, extra, replace=False)])).astype(np.int32)
        if exact:
            assert ti.size + wi.size == total
        wv = values_for(rng, semiring, wi.size)
        for accum in (0, 1, 2, 3):
            for replace in (False, True):
                mi = rng.permutation(A.m)[: A.m // 2].astype(np.int32)
                check(spv, M, A, semiring, S, xv, mi, None, False, replace, accum, wi, wv)
                check(spv, M, A, semiring, S, xv, None, None, False, replace, accum, wi, wv)
    M.close()
