"""GPU parity of the deterministic plus-times mode (SPMSPV_DETERMINISTIC)
against the oracle's sequential fp32 fold (oracle_spmspv_f32seq: products
rounded to fp32, each row's products added one at a time in product order),
bit for bit: R-MAT graphs at several densities with x in random order, under
every schedule (the bits must not move), a hub row of 300,000 products,
run lengths at the fold's and the radix tile's limits, a product count far
above the grids' estimate (several tiles per workgroup), masks, left
multiplication, a DCSC handle, and the benchmark's scale-22 graph."""
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


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def run(spv, M, S, xv, flags=0, mask=None):
    gi, gv, nnz = M.spmspv(dev(S), dev(xv), flags=flags | spv.DETERMINISTIC, mask=mask)
    return to_np(gi).astype(np.int64), to_np(gv)


def reference(A, S, xv, drop=None):
    oi, ov = oracle.spmspv_f32seq(A, S, xv)
    if drop is not None:
        keep = ~drop[oi]
        oi, ov = oi[keep], ov[keep]
    o = np.argsort(oi, kind="stable")
    return oi[o].astype(np.int64), ov[o]


def same_bits(gi, gv, oi, ov):
    assert np.array_equal(gi, oi), f"index sets differ ({gi.size} vs {oi.size})"
    bad = np.nonzero(gv.view(np.uint32) != ov.view(np.uint32))[0]
    assert bad.size == 0, f"{bad.size} values differ in their bits, e.g. rows {gi[bad[:4]]}: {gv[bad[:4]]} vs {ov[bad[:4]]}"


@pytest.fixture(scope="module")
def r16(spv):
    A = synth.rmat(16, 16, seed=71, symmetrize=True)
    M = spv.Matrix.from_csc(A, flags=spv.DETERMINISTIC)
    yield A, M
    M.close()


@pytest.mark.parametrize("density", [1e-4, 1e-3, 1e-2, 1e-1, 1.0])
def test_bits_equal_sequential_fold(spv, r16, density):
    A, M = r16
    S, xv = synth.sparse_x(A.n, max(1, synth.density_f(A.n, density)), seed=int(density * 1e6) + 3)
    gi, gv = run(spv, M, S, xv)
    same_bits(gi, gv, *reference(A, S, xv))
    assert M.last_stats()["err"] == 0


def test_bits_do_not_depend_on_the_schedule(spv, r16):
    A, M = r16
    S, xv = synth.sparse_x(A.n, A.n // 20, seed=5)
    oi, ov = reference(A, S, xv)
    for tl, sb, si, mb in ((8, 256, 4, 256), (12, 512, 8, 1024), (15, 1024, 8, 512), (10, 1024, 4, 1024)):
        M.schedule = spv.Schedule(0, tl, sb, si, mb, 0)
        gi, gv = run(spv, M, S, xv)
        same_bits(gi, gv, oi, ov)
    M.schedule = None
    # the fp64 default path agrees on the index set
    gi, _, _ = M.spmspv(dev(S), dev(xv), sorted_output=True)
    assert np.array_equal(to_np(gi).astype(np.int64), oi)


def test_hub_row_and_repeated_entries(spv):
    """Row 0 holds one entry of each of 300,000 columns (values spread over
    many binades), other rows are sparse; every column is selected, in a
    random order.  Repeated (i, j) entries inside a column keep their
    storage order."""
    rng = np.random.default_rng(9)
    n = 300000
    m = 5000
    rows = [np.zeros(n, np.int32)]
    cols = [np.arange(n, dtype=np.int32)]
    extra = 600000
    rows.append(rng.integers(1, m, extra).astype(np.int32))
    cols.append(rng.integers(0, n, extra).astype(np.int32))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    o = np.argsort(c, kind="stable")
    r, c = r[o], c[o]
    colptr = np.zeros(n + 1, np.int32)
    np.add.at(colptr, c + 1, 1)
    colptr = np.cumsum(colptr).astype(np.int32)
    vals = (rng.random(r.size) * 2.0 ** rng.integers(-10, 10, r.size)).astype(np.float32)
    A = synth.CSC(m, n, colptr, r, vals)
    M = spv.Matrix.from_csc(A, flags=spv.DETERMINISTIC)
    S = rng.permutation(n).astype(np.int32)
    xv = synth.values(n, 4, stream=77)
    gi, gv = run(spv, M, S, xv)
    same_bits(gi, gv, *reference(A, S, xv))
    M.close()


def test_mask_left_and_dcsc(spv):
    A = synth.rmat(14, 8, seed=72)                      # directed, no repeated entries
    M = spv.Matrix.from_csc(A, flags=spv.DETERMINISTIC | spv.WITH_TRANSPOSE)
    rng = np.random.default_rng(10)
    S, xv = synth.sparse_x(A.n, 1500, seed=11)
    # a mask bitmap (rows with a set bit are dropped)
    drop = rng.random(A.m) < 0.3
    words = np.zeros((A.m + 31) // 32, np.uint32)
    for i in np.nonzero(drop)[0]:
        words[i >> 5] |= np.uint32(1 << (i & 31))
    gi, gv = run(spv, M, S, xv, mask=dev(words.view(np.int32)))
    same_bits(gi, gv, *reference(A, S, xv, drop=drop))
    # left multiplication: the fold over A^T, which scipy builds
    T = A.to_scipy().T.tocsc()
    T.sort_indices()
    At = synth.CSC(A.n, A.m, T.indptr.astype(np.int32), T.indices.astype(np.int32), T.data.astype(np.float32))
    Sl, xl = synth.sparse_x(A.m, 2000, seed=12)
    gi, gv = run(spv, M, Sl, xl, flags=spv.LEFT)
    same_bits(gi, gv, *reference(At, Sl, xl))
    M.close()
    # a DCSC handle with the mode
    H = synth.column_subset(A, rng.random(A.n) < 0.2)
    D = synth.csc_to_dcsc(H)
    Md = spv.Matrix.from_dcsc(D, flags=spv.DETERMINISTIC)
    gi, gv = run(spv, Md, S, xv)
    same_bits(gi, gv, *reference(H, S, xv))
    Md.close()


def test_flag_on_other_semirings_and_without_storage(spv, r16):
    A, M = r16
    S, _ = synth.sparse_x(A.n, 700, seed=13)
    gi, gv, _ = M.spmspv(dev(S), None, semiring=spv.MIN_SELECT2ND_I32, sorted_output=True,
                         flags=spv.X_VAL_IS_INDEX | spv.DETERMINISTIC)
    oi, ov, _ = oracle.spmspv(A, S, S.astype(np.int32), 1, sorted_output=True)
    assert np.array_equal(to_np(gi), oi) and np.array_equal(to_np(gv), ov)
    P = spv.Matrix.from_csc(A)                           # created without the mode's storage
    with pytest.raises(spv.SpmspvError) as e:
        P.spmspv(dev(S), dev(np.ones(S.size, np.float32)), flags=spv.DETERMINISTIC)
    assert e.value.status == spv.EUNSUPPORTED
    P.close()
    # empty x, x of empty columns only (no products: one empty radix tile),
    # and a short output capacity
    gi, gv = run(spv, M, np.zeros(0, np.int32), np.zeros(0, np.float32))
    assert gi.size == 0
    iso = np.nonzero(A.degrees() == 0)[0].astype(np.int32)
    assert iso.size > 0
    gi, gv = run(spv, M, iso[:50], np.ones(min(50, iso.size), np.float32))
    assert gi.size == 0 and M.last_stats()["W"] == 0
    S, xv = synth.sparse_x(A.n, 300, seed=14)
    oi, ov = reference(A, S, xv)
    y = torch.empty(A.m, dtype=torch.int32, device="cuda")
    yv = torch.empty(A.m, dtype=torch.float32, device="cuda")
    with pytest.raises(spv.SpmspvError) as e:
        spv.spmspv_run(M.handle, 0, spv.DETERMINISTIC, S.size, dev(S), dev(xv), y, yv, oi.size - 1)
    assert e.value.status == spv.ECAPACITY
    assert np.array_equal(to_np(y[:oi.size - 1]).astype(np.int64), oi[:-1])


def test_full_size_rmat22(spv):
    """The benchmark's graph at 1 % and 10 % density, twice each: identical
    bits, equal to the sequential fold."""
    A = synth.rmat(22, 16, seed=1, symmetrize=True)
    M = spv.Matrix.from_csc(A, flags=spv.DETERMINISTIC)
    for density, seed in ((1e-2, 2), (1e-1, 3)):
        S, xv = synth.sparse_x(A.n, synth.density_f(A.n, density), seed=seed)
        g1 = run(spv, M, S, xv)
        g2 = run(spv, M, S, xv)
        assert np.array_equal(g1[1].view(np.uint32), g2[1].view(np.uint32))
        same_bits(*g1, *reference(A, S, xv))
    M.close()


def test_calls_of_changing_length_in_a_row(spv):
    """The deterministic path clears the scan's look-back words for the next
    call itself (no bucket scatter runs): calls whose x spans more scan tiles
    than the call before stay exact, in any order of lengths."""
    A = synth.rmat(15, 16, seed=73, symmetrize=True)
    M = spv.Matrix.from_csc(A, flags=spv.DETERMINISTIC)
    for k, f in enumerate((100, 20000, A.n, 300, A.n, 5000)):
        S, xv = synth.sparse_x(A.n, f, seed=80 + k)
        gi, gv = run(spv, M, S, xv)
        same_bits(gi, gv, *reference(A, S, xv))
        st = M.last_stats()
        assert st["err"] == 0 and st["W"] == int(A.degrees()[S].sum())
    # and the default path afterwards on the same handle
    gi, gv, _ = M.spmspv(dev(S), dev(xv), sorted_output=True)
    assert np.array_equal(to_np(gi).astype(np.int64), reference(A, S, xv)[0])
    M.close()


def test_run_lengths_around_the_fold_and_tile_limits(spv):
    """Rows with product counts at and around the short fold's limit (129
    entries), a radix tile (4096 entries) and a single entry, shuffled so that
    runs start and end at every offset of the tiles: one product per column,
    values of both signs over many binades; x in column order and permuted;
    and under a mask whose dropped rows sort after every real one (their tail
    starts inside a tile or in the entries staged after it)."""
    rng = np.random.default_rng(21)
    lengths = np.array([1, 2, 3, 127, 128, 129, 130, 131, 257, 4095, 4096, 4097])
    m = 1200
    rows = np.repeat(np.arange(m, dtype=np.int32), rng.choice(lengths, m))
    rng.shuffle(rows)
    n = rows.size
    colptr = np.arange(n + 1, dtype=np.int32)
    vals = (rng.random(n) * 2.0 ** rng.integers(-12, 12, n) * rng.choice([-1.0, 1.0], n)).astype(np.float32)
    A = synth.CSC(m, n, colptr, rows, vals)
    M = spv.Matrix.from_csc(A, flags=spv.DETERMINISTIC)
    xv = synth.values(n, 4, stream=78)
    for S in (np.arange(n, dtype=np.int32), rng.permutation(n).astype(np.int32)):
        gi, gv = run(spv, M, S, xv)
        same_bits(gi, gv, *reference(A, S, xv))
    drop = rng.random(m) < 0.4
    words = np.zeros((m + 31) // 32, np.uint32)
    for i in np.nonzero(drop)[0]:
        words[i >> 5] |= np.uint32(1 << (i & 31))
    gi, gv = run(spv, M, S, xv, mask=dev(words.view(np.int32)))
    same_bits(gi, gv, *reference(A, S, xv, drop=drop))
    M.close()


def test_product_count_far_above_the_grid_estimate(spv):
    """The kernels take their chunk and tile counts from the product count on
    the device and loop over them; the grids come from the expected count
    f * nnz / n.  Here x selects the only long columns of a mostly empty
    matrix (3M products where the estimate is ~300), so each workgroup takes
    several radix tiles and gather chunks in turn."""
    rng = np.random.default_rng(23)
    n, m, k, deg = 1_000_000, 200_000, 100, 30_000
    long_cols = np.sort(rng.choice(n, k, replace=False)).astype(np.int32)
    colptr = np.zeros(n + 1, np.int64)
    colptr[long_cols + 1] = deg
    colptr = np.cumsum(colptr).astype(np.int32)
    rows = rng.integers(0, m, k * deg).astype(np.int32)
    vals = (rng.random(k * deg) * 2.0 ** rng.integers(-8, 8, k * deg)).astype(np.float32)
    A = synth.CSC(m, n, colptr, rows, vals)
    M = spv.Matrix.from_csc(A, flags=spv.DETERMINISTIC)
    S = rng.permutation(long_cols).astype(np.int32)
    xv = synth.values(S.size, 4, stream=79)
    gi, gv = run(spv, M, S, xv)
    same_bits(gi, gv, *reference(A, S, xv))
    assert M.last_stats()["W"] == k * deg
    M.close()
