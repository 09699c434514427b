"""What the trained selector gains over the method without it.

The network is trained on the GPU (the library's own forward / backward /
Adam kernels) from timings of the library's own calls on small training
graphs, then judged on held-out graphs it never saw, two ways:

* per step: on each held-out input every class is timed and the selector's
  choice is scored against the fastest class (regret = summed time of the
  choices / summed best time); without the selector the library runs its
  default schedule (push with 256 buckets, class 4) everywhere;
* end to end: whole BFS runs from several roots of a held-out scale-20
  R-MAT graph, host-timed, with the selector consuming its decisions inside
  the captured level graph, against the default schedule (the method
  without the selector) and the frontier-edge direction heuristic.  (On
  graphs of 2^17 vertices and below a direction-switching level's extra
  decision and gated kernels cost more than pull saves, for the heuristic
  as for the selector.)

The test requires the learned choices to cost less than the default per
step and the learned BFS to beat the default BFS end to end; it reports the
heuristic and the best single class in hindsight beside them."""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def spv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_07902_amd as spv
    spv.load_library()
    synth.build(force=False)
    return spv


DEFAULT_CLASS = 4


def collect(spv, A, name, roots, seed):
    from paper_1610_07902_amd import selector
    P = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    s = selector.bfs_samples(P, A.nnz, synth.roots(A, roots, seed=seed), reps=2, tag=name)
    s.extend(selector.random_samples(P, A.nnz, (1e-4, 1e-3, 1e-2, 1e-1, 3e-1), spv.MIN_SELECT2ND_I32, reps=2,
                                     seed=seed, tag=name))
    P.close()
    return s


def test_trained_selector_beats_default_schedule_on_held_out_graph(spv, capsys):
    from paper_1610_07902_amd import selector
    train = selector.Samples()
    for name, A in (("rmat13", synth.rmat(13, 16, seed=201, symmetrize=True)),
                    ("rmat15", synth.rmat(15, 16, seed=202, symmetrize=True)),
                    ("rmat17", synth.rmat(17, 16, seed=204, symmetrize=True)),
                    ("rmat18", synth.rmat(18, 16, seed=206, symmetrize=True)),
                    ("rmat19", synth.rmat(19, 16, seed=207, symmetrize=True)),
                    ("grid2d-128", synth.grid(128, 128, 1)),
                    ("grid2d-512", synth.grid(512, 512, 1)),
                    ("grid3d-24", synth.grid(24, 24, 24)),
                    ("grid3d-64", synth.grid(64, 64, 64))):
        train.extend(collect(spv, A, name, 3, 11))
    params, mean, std, hist = selector.train(train, epochs=200, lr=2e-3)
    assert hist[-1] < hist[0]
    held = selector.Samples()
    held.extend(collect(spv, synth.rmat(16, 16, seed=203, symmetrize=True), "rmat16", 3, 12))
    held.extend(collect(spv, synth.grid(40, 40, 20), "grid3d-40", 2, 13))
    T = held.T
    pred = selector.predict(params, mean, std, held.X)
    learned = selector.regret(T, pred)
    default = selector.regret(T, np.full(len(pred), DEFAULT_CLASS))
    single = min(selector.regret(T, np.full(len(pred), c)) for c in range(10) if np.isfinite(T[:, c]).all())
    with capsys.disabled():
        print(f"\n[selector gain] held-out samples {len(pred)}: regret learned {learned:.3f}, "
              f"default class {default:.3f}, best single class in hindsight {single:.3f}")
        print("[selector gain] best classes", np.bincount(T.argmin(1), minlength=10).tolist(),
              "chosen", np.bincount(pred, minlength=10).tolist())
        worst = np.argsort(-(T[np.arange(len(pred)), pred] - T.min(1)))[:5]
        for k in worst:
            print("  ", held.tags[k], "chose", pred[k], "best", T[k].argmin(), "us", np.round(T[k], 1).tolist())
    assert learned < default, (learned, default)
    assert learned < 1.5
    # end to end on a held-out R-MAT graph large enough that a level's
    # decision kernels (a few microseconds) do not dominate, with the weights
    # just trained
    A = synth.rmat(20, 16, seed=205, symmetrize=True)
    P = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
    P.load_selector(params, mean, std)
    roots = [int(r) for r in synth.roots(A, 8, seed=14)]

    def bfs_ms(flags):
        P.bfs(roots[0], spv.MIN_SELECT2ND_I32, flags=flags)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(3):
            t = time.perf_counter()
            for r in roots:
                P.bfs(r, spv.MIN_SELECT2ND_I32, flags=flags)
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t) * 1e3)
        return best

    t_default = bfs_ms(spv.USE_GRAPH)
    t_heur = bfs_ms(spv.USE_GRAPH | spv.DIRECTION_OPT)
    t_learned = bfs_ms(spv.USE_GRAPH | spv.USE_SELECTOR)
    P.close()
    with capsys.disabled():
        print(f"[selector gain] held-out rmat20 BFS, 8 roots: default {t_default:.2f} ms, heuristic "
              f"{t_heur:.2f} ms, learned in-graph {t_learned:.2f} ms")
    assert t_learned < t_default, (t_learned, t_default)
