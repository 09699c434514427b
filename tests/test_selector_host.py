"""CPU tests of the selector's host-side logic (no GPU): feature encoding,
tie-tolerant labels, regret, sample persistence and the weights file."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def selector():
    # the module imports the binding's constants only; nothing used here
    # loads the library
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1610_07902_amd import selector as sel
    return sel


def test_encode_and_features():
    sel = selector()
    raw = sel.raw_features(41943, 1267850, 163196, 1 << 22, 128304750, 1 << 22)
    assert raw.shape == (6,)
    assert raw[4] == 128304750 / (1 << 22)
    enc = sel.encode(raw)
    assert np.allclose(enc, np.log2(1 + raw))
    assert sel.encode(np.zeros(6)).tolist() == [0.0] * 6


def test_labels_break_near_ties_by_prior():
    sel = selector()
    T = np.array([[10.0, 10.2, 50, 50, 50, 50, 50, 50, 50, 50],   # 0 and 1 tied (within 3%)
                  [20.0, 10.0, 50, 50, 50, 50, 50, 50, 50, 50],   # 1 clearly best
                  [30.0, 10.0, 50, 50, 50, 50, 50, 50, 50, 50],   # 1 clearly best
                  [10.0, 50.0, 50, 50, 50, 50, 50, 50, 50, 9.0]])  # 9 best, 0 not within 3%
    y = sel.labels(T, tie=0.03)
    # class 1 is fastest most often, so the tie in row 0 goes to 1
    assert y.tolist() == [1, 1, 1, 9]
    assert sel.labels(T, tie=0.0).tolist() == [0, 1, 1, 9]


def test_regret():
    sel = selector()
    T = np.array([[1.0, 2.0], [4.0, 3.0]])
    assert sel.regret(T, np.array([0, 1])) == 1.0
    assert abs(sel.regret(T, np.array([1, 0])) - 6.0 / 4.0) < 1e-12


def test_samples_roundtrip(tmp_path):
    sel = selector()
    s = sel.Samples()
    rng = np.random.default_rng(0)
    for k in range(5):
        s.add(rng.random(6), rng.random(10), f"g/r{k}/L{k}")
    p = tmp_path / "s.npz"
    s.save(str(p))
    t = sel.Samples.load(str(p))
    assert np.array_equal(t.X, s.X) and np.array_equal(t.T, s.T) and t.tags == s.tags


def test_committed_weights_file_is_well_formed():
    sel = selector()
    params, mean, std, meta = sel.load_weights()
    assert params.shape == (5258,) and mean.shape == (6,) and std.shape == (6,)
    assert np.all(np.isfinite(params)) and np.all(std > 0)
    assert meta.get("samples", 0) > 0 and not meta.get("quick", True)
    with open(sel.WEIGHTS_PATH) as fh:
        d = json.load(fh)
    assert set(d) == {"params", "mean", "std", "meta", "multiply"}
    mp, mm, ms, _ = sel.load_weights(kind="multiply")
    assert mp.shape == (5258,) and mm.shape == (6,) and ms.shape == (6,)
    assert np.all(np.isfinite(mp)) and np.all(ms > 0)
    assert meta.get("bfs_samples", 0) > 0 and meta.get("multiply_samples", 0) > 0


def test_init_params_layout():
    sel = selector()
    p = sel.init_params(np.random.default_rng(1))
    assert p.dtype == np.float32 and p.size == 5258
    # biases start at zero: b1 after W1 (64*6), b2 after W2, b3 last
    assert np.all(p[384:448] == 0) and np.all(p[448 + 4096:448 + 4096 + 64] == 0) and np.all(p[-10:] == 0)


def test_weights_are_tied_to_the_kernel_sources(tmp_path):
    """The committed weights carry the digest of the device sources they were
    trained on and it matches the sources in the tree (retrain after any
    kernel change); a weights file from other kernels is recognised as
    stale."""
    sel = selector()
    _, _, _, meta = sel.load_weights()
    assert meta.get("kernel_digest") == sel.kernel_digest(), "selector weights trained on other kernels: retrain"
    assert sel.weights_current(meta)
    stale = dict(meta, kernel_digest="0" * 16)
    assert not sel.weights_current(stale)
    p, m, s, _ = sel.load_weights()
    out = tmp_path / "w.json"
    sel.save_weights(p, m, s, {"samples": 1}, str(out))
    assert sel.load_weights(str(out))[3]["kernel_digest"] == sel.kernel_digest()


def test_scale_augmentation_copies():
    """Training copies of BFS steps (unvisited < n): size features scaled,
    nnz/n kept, timings repeated; standalone multiplies are not copied."""
    from paper_1610_07902_amd import selector
    raw = np.array([[10.0, 300.0, 40.0, 1000.0, 8.0, 900.0],     # a BFS step
                    [1.0, 2.0, 2.0, 50.0, 3.0, 50.0],            # a standalone multiply
                    [5.0, 90.0, 30.0, 400.0, 6.0, 399.0]])       # a BFS step
    times = np.arange(30, dtype=np.float64).reshape(3, 10)
    X, T = selector.augmented(raw, times, scales=(2.0, 4.0))
    assert X.shape == (7, 6) and T.shape == (7, 10)
    assert np.array_equal(X[:3], raw) and np.array_equal(T[:3], times)
    b = raw[[0, 2]]
    assert np.array_equal(X[3:5, [0, 1, 2, 3, 5]], 2.0 * b[:, [0, 1, 2, 3, 5]])
    assert np.array_equal(X[5:7, [0, 1, 2, 3, 5]], 4.0 * b[:, [0, 1, 2, 3, 5]])
    assert np.array_equal(X[3:, 4], np.tile(b[:, 4], 2))
    assert np.array_equal(T[3:], np.tile(times[[0, 2]], (2, 1)))
