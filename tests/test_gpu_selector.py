"""GPU tests of the schedule selector: the MLP forward / backward / Adam
kernels against the fp64 oracle, masked SpMSpV, and selector-driven
SpMSpV and BFS (every class must give the oracle's result)."""
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


def init_params(rng, scale=1.0):
    i, h1, h2, o = oracle.MLP_SHAPE
    parts = [rng.normal(0, scale / np.sqrt(i), h1 * i), rng.normal(0, 0.1, h1),
             rng.normal(0, scale / np.sqrt(h1), h2 * h1), rng.normal(0, 0.1, h2),
             rng.normal(0, scale / np.sqrt(h2), o * h2), rng.normal(0, 0.1, o)]
    return np.concatenate(parts).astype(np.float32)


def test_param_count(spv):
    assert spv.spmspv_mlp_param_count() == oracle.mlp_param_count() == spv.MLP_PARAMS


@pytest.mark.parametrize("batch", [1, 7, 128, 1000])
def test_mlp_forward_matches_oracle(spv, batch):
    rng = np.random.default_rng(batch)
    p = init_params(rng)
    X = rng.normal(0, 1.5, (batch, 6)).astype(np.float32)
    logits = torch.empty((batch, 10), dtype=torch.float32, device="cuda")
    spv.spmspv_mlp_forward(dev(p), dev(X), logits)
    torch.cuda.synchronize()
    ref = oracle.mlp_forward(p.astype(np.float64), X.astype(np.float64))
    err = np.abs(to_np(logits).astype(np.float64) - ref)
    # fp32 dot products of length <= 64 on O(1) values
    assert np.max(err / (1.0 + np.abs(ref))) < 1e-4


@pytest.mark.parametrize("batch", [1, 33, 128])
def test_mlp_gradient_matches_oracle(spv, batch):
    rng = np.random.default_rng(100 + batch)
    p = init_params(rng)
    X = rng.normal(0, 1.0, (batch, 6)).astype(np.float32)
    y = rng.integers(0, 10, batch).astype(np.int32)
    pd = dev(p)
    grad = torch.empty(p.size, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    spv.spmspv_mlp_train_step(pd, None, None, 1, 0.0, dev(X), dev(y), grad=grad, loss=loss)
    torch.cuda.synchronize()
    ref_loss, ref_g = oracle.mlp_loss_grad(p.astype(np.float64), X.astype(np.float64), y)
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * max(1.0, abs(ref_loss))
    g = to_np(grad).astype(np.float64)
    scale = np.max(np.abs(ref_g))
    assert np.max(np.abs(g - ref_g)) <= 1e-4 * scale, "gradient differs from the fp64 oracle"
    # lr = 0 leaves the parameters untouched
    assert np.array_equal(to_np(pd), p)


def test_mlp_adam_update(spv):
    rng = np.random.default_rng(7)
    p = init_params(rng)
    X = rng.normal(0, 1.0, (64, 6)).astype(np.float32)
    y = rng.integers(0, 10, 64).astype(np.int32)
    m0 = rng.normal(0, 1e-2, p.size).astype(np.float32)
    v0 = rng.uniform(0, 1e-3, p.size).astype(np.float32)
    pd, md, vd = dev(p), dev(m0), dev(v0)
    grad = torch.empty(p.size, dtype=torch.float32, device="cuda")
    step, lr = 5, 1e-2
    spv.spmspv_mlp_train_step(pd, md, vd, step, lr, dev(X), dev(y), grad=grad)
    torch.cuda.synchronize()
    g = to_np(grad).astype(np.float64)
    m1 = 0.9 * m0 + 0.1 * g
    v1 = 0.999 * v0 + 0.001 * g * g
    p1 = p - lr * (m1 / (1 - 0.9 ** step)) / (np.sqrt(v1 / (1 - 0.999 ** step)) + 1e-8)
    assert np.allclose(to_np(md), m1, rtol=1e-5, atol=1e-9)
    assert np.allclose(to_np(vd), v1, rtol=1e-5, atol=1e-12)
    assert np.max(np.abs(to_np(pd) - p1)) <= 1e-4 * lr + 1e-6


def test_mlp_training_reduces_loss(spv):
    """A separable synthetic task: the class is a function of two features."""
    rng = np.random.default_rng(3)
    N = 2048
    X = rng.normal(0, 1, (N, 6)).astype(np.float32)
    y = (np.clip(np.floor((X[:, 0] + 2.5) * 2), 0, 9)).astype(np.int32)
    p = dev(init_params(rng))
    m = torch.zeros(p.numel(), dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    Xd, yd = dev(X), dev(y)
    losses = []
    for step in range(1, 601):
        b = (step * 128) % N
        spv.spmspv_mlp_train_step(p, m, v, step, 3e-3, Xd[b:b + 128], yd[b:b + 128], loss=loss)
        if step % 100 == 1:
            losses.append(float(loss.item()))
    logits = torch.empty((N, 10), dtype=torch.float32, device="cuda")
    spv.spmspv_mlp_forward(p, Xd, logits)
    acc = float((logits.argmax(1).cpu().numpy() == y).mean())
    assert losses[-1] < 0.5 * losses[0], losses
    assert acc > 0.8, acc


def test_mlp_bad_arguments(spv):
    p = torch.zeros(spv.MLP_PARAMS, dtype=torch.float32, device="cuda")
    X = torch.zeros((129, 6), dtype=torch.float32, device="cuda")
    y = torch.zeros(129, dtype=torch.int32, device="cuda")
    with pytest.raises(spv.SpmspvError):
        spv.spmspv_mlp_train_step(p, None, None, 1, 0.0, X, y)          # batch > 128
    with pytest.raises(spv.SpmspvError):
        spv.spmspv_mlp_train_step(p, None, None, 1, 0.1, X[:4], y[:4])  # lr > 0 without moments
    with pytest.raises(spv.SpmspvError):
        spv.spmspv_mlp_train_step(p, None, None, 0, 0.0, X[:4], y[:4])  # step 0


# ------------------------------------------------------------ masked SpMSpV
def mask_words(bits):
    m = bits.size
    w = np.zeros((m + 31) // 32, np.uint32)
    idx = np.nonzero(bits)[0]
    np.bitwise_or.at(w, idx >> 5, (np.uint32(1) << (idx & 31).astype(np.uint32)))
    return w.view(np.int32)


@pytest.fixture(scope="module")
def rmat14():
    return synth.rmat(14, 16, seed=11, symmetrize=True)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("semiring", [0, 1, 2])
def test_masked_run_matches_oracle(spv, rmat14, direction, semiring):
    A = rmat14
    M = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE)
    if direction:
        s = M.schedule
        s.direction = 1
        M.schedule = s
    rng = np.random.default_rng(semiring + 10 * direction)
    bits = (rng.random(A.m) < 0.4).astype(np.uint8)
    S, xv = synth.sparse_x(A.n, synth.density_f(A.n, 0.05), seed=3, tag=semiring)
    if semiring == 0:
        gi, gv, _ = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True, mask=dev(mask_words(bits)))
    elif semiring == 1:
        xv = S.astype(np.int32)
        gi, gv, _ = M.spmspv(dev(S), None, semiring=1, sorted_output=True, flags=spv.X_VAL_IS_INDEX,
                             mask=dev(mask_words(bits)))
    else:
        xv = np.ones(S.size, np.uint8)
        gi, gv, _ = M.spmspv(dev(S), None, semiring=2, sorted_output=True, flags=spv.X_ALL_TRUE,
                             mask=dev(mask_words(bits)))
    oi, ov, _ = oracle.spmspv(A, S, xv, semiring, mask=bits, sorted_output=True)
    compare(semiring, gi, gv, oi, ov, sorted_output=True)
    assert M.last_stats()["err"] == 0


# --------------------------------------------------------- selector classes
def constant_selector(cls):
    """Weights whose output is class `cls` for every input."""
    p = np.zeros(oracle.mlp_param_count(), np.float32)
    p[-10 + cls] = 5.0
    return p, np.zeros(6, np.float32), np.ones(6, np.float32)


@pytest.mark.parametrize("cls", list(range(10)))
def test_selector_every_class_matches_oracle(spv, rmat14, cls):
    A = rmat14
    M = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE)
    M.load_selector(*constant_selector(cls))
    for k, f in enumerate([0.0005, 0.02, 0.3]):
        for semiring in (0, 1):
            S, xv = synth.sparse_x(A.n, synth.density_f(A.n, f), seed=5 + k, tag=cls)
            if semiring == 0:
                gi, gv, _ = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True, flags=spv.USE_SELECTOR)
            else:
                xv = S.astype(np.int32)
                gi, gv, _ = M.spmspv(dev(S), None, semiring=1, sorted_output=True,
                                     flags=spv.USE_SELECTOR | spv.X_VAL_IS_INDEX)
            st = M.last_stats()
            assert st["cls"] == cls and st["err"] == 0
            oi, ov, W = oracle.spmspv(A, S, xv, semiring, sorted_output=True)
            compare(semiring, gi, gv, oi, ov, sorted_output=True)
            assert st["W"] == W and st["nnz_y"] == oi.size
    # a plain call after selector calls still agrees (counters left clean)
    S, xv = synth.sparse_x(A.n, synth.density_f(A.n, 0.01), seed=99, tag=1)
    gi, gv, _ = M.spmspv(dev(S), dev(xv), semiring=0, sorted_output=True)
    oi, ov, _ = oracle.spmspv(A, S, xv, 0, sorted_output=True)
    compare(0, gi, gv, oi, ov, sorted_output=True)


def test_selector_class_tiles(spv, rmat14):
    M = spv.Matrix.from_csc(rmat14, flags=spv.WITH_TRANSPOSE)
    tiles = [M.class_tile(c) for c in range(9)]
    assert all(8 <= t <= 15 for t in tiles)
    assert tiles == sorted(tiles, reverse=True)
    assert M.class_tile(9) == -1


@pytest.mark.parametrize("cls", [0, 4, 8, 9])
@pytest.mark.parametrize("semiring", [1, 2])
def test_selector_bfs_matches_oracle(spv, rmat14, cls, semiring):
    A = rmat14
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    M.load_selector(*constant_selector(cls))
    deg = A.degrees()
    root = int(np.argmax(deg))
    lev, par, nl = M.bfs(root, semiring=semiring, flags=spv.USE_SELECTOR)
    olev, opar, onl = oracle.bfs(A, root)
    assert nl == onl
    assert np.array_equal(to_np(lev), olev)
    if semiring == 1:
        assert np.array_equal(to_np(par), opar)
    assert M.selector_classes() == [cls] * (onl)


def test_selector_bfs_mixed_classes(spv, rmat14):
    """Random weights give a mix of classes over the levels; results unchanged."""
    A = rmat14
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    rng = np.random.default_rng(5)
    p = init_params(rng, scale=3.0)
    M.load_selector(p, np.full(6, 8.0, np.float32), np.full(6, 4.0, np.float32))
    for root in synth.roots(A, 4, seed=2):
        lev, par, nl = M.bfs(int(root), semiring=1, flags=spv.USE_SELECTOR)
        olev, opar, onl = oracle.bfs(A, int(root))
        assert nl == onl
        assert np.array_equal(to_np(lev), olev) and np.array_equal(to_np(par), opar)
        assert len(M.selector_classes()) == onl


def test_selector_load_rejects_bad_weights(spv, rmat14):
    M = spv.Matrix.from_csc(rmat14)
    p, mu, sd = constant_selector(0)
    bad = p.copy()
    bad[3] = np.nan
    with pytest.raises(spv.SpmspvError):
        M.load_selector(bad, mu, sd)
    with pytest.raises(spv.SpmspvError):
        M.load_selector(p, mu, np.zeros(6, np.float32))
    S = dev(np.arange(10, dtype=np.int32))
    with pytest.raises(spv.SpmspvError):
        M.spmspv(S, dev(np.ones(10, np.float32)), flags=spv.USE_SELECTOR)   # selector disabled


def test_device_features_match_host(spv, rmat14):
    """The features the device computes for its decision equal the host's
    computation from the same call's statistics (what training uses)."""
    from paper_1610_07902_amd import selector
    A = rmat14
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    rng = np.random.default_rng(8)
    mean = rng.normal(5, 2, 6).astype(np.float32)
    std = rng.uniform(0.5, 3, 6).astype(np.float32)
    p = np.zeros(spv.MLP_PARAMS, np.float32)
    p[-10 + 4] = 1.0
    M.load_selector(p, mean, std)
    for f in (1, 37, 2000):
        S, _ = synth.sparse_x(A.n, f, seed=f)
        M.spmspv(dev(S), None, semiring=1, flags=spv.USE_SELECTOR | spv.X_VAL_IS_INDEX)
        st = M.last_stats()
        dev_feat = np.array(spv.spmspv_selector_features(M.handle))
        raw = selector.raw_features(f, st["W"], st["maxlen"], A.n, A.nnz, A.n)
        host = (selector.encode(raw) - mean) / std
        assert np.allclose(dev_feat, host, rtol=1e-5, atol=1e-5), (dev_feat, host)
    # inside a BFS the last feature counts the vertices not yet reached
    root = int(np.argmax(A.degrees()))
    lev, _, nl = M.bfs(root, semiring=1, flags=spv.USE_SELECTOR)
    dev_feat = np.array(spv.spmspv_selector_features(M.handle))
    reached = int((to_np(lev) >= 0).sum())
    assert np.isclose(dev_feat[5] * std[5] + mean[5], np.log2(1 + A.n - reached), atol=1e-4)


@pytest.mark.parametrize("cls", [4, 9, -1])
@pytest.mark.parametrize("semiring", [1, 2])
def test_selector_bfs_device_gated(spv, rmat14, cls, semiring):
    """Selector inside the captured level graph: the decision stays on the
    device (direction only); results equal the oracle's for every class."""
    A = rmat14
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    if cls >= 0:
        M.load_selector(*constant_selector(cls))
    else:
        rng = np.random.default_rng(5)
        M.load_selector(init_params(rng, scale=3.0), np.full(6, 8.0, np.float32), np.full(6, 4.0, np.float32))
    for root in synth.roots(A, 3, seed=9):
        lev, par, nl = M.bfs(int(root), semiring=semiring, flags=spv.USE_SELECTOR | spv.USE_GRAPH)
        olev, opar, onl = oracle.bfs(A, int(root))
        assert nl == onl
        assert np.array_equal(to_np(lev), olev)
        if semiring == 1:
            assert np.array_equal(to_np(par), opar)


def test_forced_class_sequence_replay(spv, rmat14):
    """A given class sequence replaces the network step by step; results stay
    the oracle's and the recorded classes are the forced ones."""
    A = rmat14
    M = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    root = int(np.argmax(A.degrees()))
    olev, opar, onl = oracle.bfs(A, root)
    seq = [9, 3, 9, 0, 8, 9, 2, 9, 5, 1][:onl]
    spv.spmspv_force_classes(M.handle, seq)
    lev, par, nl = M.bfs(root, semiring=1, flags=spv.USE_SELECTOR)   # no weights needed while forced
    assert nl == onl and np.array_equal(to_np(lev), olev) and np.array_equal(to_np(par), opar)
    assert M.selector_classes() == seq
    spv.spmspv_force_classes(M.handle, [])
    with pytest.raises(spv.SpmspvError):
        M.bfs(root, semiring=1, flags=spv.USE_SELECTOR)                # no weights, nothing forced
    with pytest.raises(spv.SpmspvError):
        spv.spmspv_force_classes(M.handle, [10])
