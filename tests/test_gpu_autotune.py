"""GPU tests of the autotuner: tuned schedules never change results, the
table is consistent, and the batched tuner keeps a feasible schedule."""
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
def rmat15():
    return synth.rmat(15, 16, seed=41, symmetrize=True)


@pytest.mark.parametrize("semiring", [0, 1])
def test_autotune_table_and_parity(spv, rmat15, semiring):
    A = rmat15
    M = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE)
    with pytest.raises(spv.SpmspvError):
        spv.spmspv_tuned_schedule(M.handle, 100)          # not tuned yet
    dens = (1e-3, 1e-2, 1e-1)
    table = M.autotune(semiring, dens, reps=3)
    assert [e["density"] for e in table] == list(dens)
    for e in table:
        # the draw is Bernoulli(density) per column: within 6 sigma of n * density
        mu = A.n * e["density"]
        assert abs(e["f"] - mu) <= 6 * np.sqrt(mu) + 2
        assert e["us"] <= e["default_us"] + 1e-9
        sc = e["sched"]
        assert 8 <= sc["tile_log2"] <= 15 and sc["direction"] in (0, 1)
    for k, d in enumerate(dens):
        f = synth.density_f(A.n, d)
        got = spv.spmspv_tuned_schedule(M.handle, f)
        assert got.as_dict() == table[k]["sched"]
        S, xv = synth.sparse_x(A.n, f, seed=60 + k)
        if semiring == 0:
            gi, gv, _ = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True, flags=spv.AUTO_SCHEDULE)
            oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
        else:
            gi, gv, _ = M.spmspv(dev(S), None, semiring=1, sorted_output=True,
                                 flags=spv.AUTO_SCHEDULE | spv.X_VAL_IS_INDEX)
            oi, ov, _ = oracle.spmspv(A, S, S.astype(np.int32), 1, sorted_output=True)
        compare(semiring, gi, gv, oi, ov, sorted_output=True)
    # the handle's own schedule is untouched by tuning and by auto calls
    assert M.schedule.direction == 0


def test_autotune_bad_arguments(spv, rmat15):
    M = spv.Matrix.from_csc(rmat15)
    with pytest.raises(spv.SpmspvError):
        M.autotune(0, (0.0,), reps=1)
    with pytest.raises(spv.SpmspvError):
        M.autotune(0, (1.5,), reps=1)


def test_autotune_batch(spv, rmat15):
    A = rmat15
    M = spv.Matrix.from_csc(A)
    sizes = synth.log_uniform_sizes(16, A.n / 4, seed=3)
    xs = [synth.sparse_x(A.n, int(f), seed=90 + k) for k, f in enumerate(sizes)]
    off = np.zeros(17, np.int64)
    off[1:] = np.cumsum(sizes)
    idx = np.concatenate([x[0] for x in xs])
    val = np.concatenate([x[1] for x in xs])
    W = int(sum(A.degrees()[x[0]].sum() for x in xs))
    M.attach_batch(16, max_f=int(off[-1]), max_products=W)
    cap = 16 * A.m
    y_off = torch.empty(17, dtype=torch.int64, device="cuda")
    y_idx = torch.empty(cap, dtype=torch.int32, device="cuda")
    y_val = torch.empty(cap, dtype=torch.float32, device="cuda")
    best, us = spv.spmspv_autotune_batch(M.handle, 0, 0, 16, dev(off), dev(idx), dev(val), y_off, y_idx, y_val, cap,
                                         reps=2)
    assert us > 0
    eff = spv.spmspv_get_batch_schedule(M.handle, 16)
    assert eff.as_dict() == best.as_dict()
    total = spv.spmspv_run_batch(M.handle, 0, 0, 16, dev(off), dev(idx), dev(val), y_off, y_idx, y_val, cap)
    yo = to_np(y_off)
    assert yo[-1] == total
    for b in range(16):
        oi, ov, _ = oracle.spmspv(A, xs[b][0], xs[b][1], 0, sorted_output=True)
        compare(0, y_idx[yo[b]:yo[b + 1]], y_val[yo[b]:yo[b + 1]], oi, ov, sorted_output=True)


def test_default_schedule_sizes_the_scatter_chunk(spv, rmat15):
    """With no schedule set, each call takes the largest scatter chunk (up to
    4096 products) that the expected product count f * nnz / n spreads over
    every compute unit;
    an explicit schedule is used as given.  Results match the oracle either
    way."""
    A = rmat15
    M = spv.Matrix.from_csc(A)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    chunks = [(512, 8), (256, 8), (256, 4)]
    for f in (10, 300, 3000, A.n):
        eff = spv.spmspv_effective_schedule(M.handle, f)
        w_est = f * A.nnz / A.n
        fits = [c for c in chunks if w_est >= c[0] * c[1] * cus]
        want = fits[0] if fits else chunks[-1]
        assert (eff.scatter_block, eff.scatter_items) == want, (f, eff.as_dict())
        assert eff.tile_log2 == M.schedule.tile_log2
        S, xv = synth.sparse_x(A.n, f, seed=70 + f)
        gi, gv, _ = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True)
        oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
        compare(0, gi, gv, oi, ov, sorted_output=True)
    s = M.schedule
    s.scatter_block, s.scatter_items = 1024, 4
    M.schedule = s
    eff = spv.spmspv_effective_schedule(M.handle, 10)
    assert (eff.scatter_block, eff.scatter_items) == (1024, 4)
    M.schedule = None
    eff = spv.spmspv_effective_schedule(M.handle, 10)
    assert (eff.scatter_block, eff.scatter_items) == (256, 4)


def test_tuning_table_persists_and_reloads(spv, rmat15, tmp_path):
    """A saved table reloads onto a new handle over the same matrix (same
    schedules, AUTO_SCHEDULE calls still match the oracle) and is refused,
    leaving the handle untouched, for another matrix, other kernels, another
    device, another format version or a damaged file."""
    A = rmat15
    M = spv.Matrix.from_csc(A)
    path = str(tmp_path / "tuning.txt")
    with pytest.raises(spv.SpmspvError) as e:
        M.save_tuning(path)                                  # nothing tuned yet
    assert e.value.status == spv.EINVAL
    dens = (1e-3, 1e-1)
    M.autotune(0, dens, reps=2)
    M.save_tuning(path)
    text = open(path).read().splitlines()
    assert text[0] == "spmspv-tuning 1" and text[2] == "library " + spv.spmspv_source_digest()
    N = spv.Matrix.from_csc(A)
    N.load_tuning(path)
    for d in dens:
        f = synth.density_f(A.n, d)
        assert spv.spmspv_tuned_schedule(N.handle, f).as_dict() == spv.spmspv_tuned_schedule(M.handle, f).as_dict()
        S, xv = synth.sparse_x(A.n, f, seed=70)
        gi, gv, _ = N.spmspv(dev(S), dev(xv), sorted_output=True, flags=spv.AUTO_SCHEDULE)
        oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
        compare(0, gi, gv, oi, ov, sorted_output=True)
    # another matrix of the same shape and size
    B = synth.rmat(15, 16, seed=42, symmetrize=True)
    O = spv.Matrix.from_csc(B)
    with pytest.raises(spv.SpmspvError) as e:
        O.load_tuning(path)
    assert e.value.status == spv.EUNSUPPORTED
    with pytest.raises(spv.SpmspvError):
        spv.spmspv_tuned_schedule(O.handle, 100)            # still untuned
    # edited keys, another version, a damaged file, a missing one
    for k, line, status in ((2, "library 0000000000000000", spv.EUNSUPPORTED),
                            (1, "device some other GPU|gfx000|1", spv.EUNSUPPORTED),
                            (0, "spmspv-tuning 2", spv.EINVAL),
                            (5, "0.5 0 12", spv.EINVAL)):
        bad = list(text)
        bad[k] = line
        p2 = str(tmp_path / f"bad{k}.txt")
        open(p2, "w").write("\n".join(bad) + "\n")
        with pytest.raises(spv.SpmspvError) as e:
            N.load_tuning(p2)
        assert e.value.status == status, (k, e.value)
    with pytest.raises(spv.SpmspvError) as e:
        N.load_tuning(str(tmp_path / "missing.txt"))
    assert e.value.status == spv.EINVAL
    # the good table is still installed on N
    f = synth.density_f(A.n, 1e-1)
    assert spv.spmspv_tuned_schedule(N.handle, f).as_dict() == spv.spmspv_tuned_schedule(M.handle, f).as_dict()
