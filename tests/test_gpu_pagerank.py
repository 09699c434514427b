"""GPU data-driven PageRank (fp32) against the fp64 oracle running the same
rule.  Which vertices stay active is decided in each side's own precision,
so vertices near the threshold may differ; the bound allows the mass such a
difference can move (at most tol * rank per vertex per step)."""
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


def check(A, r_gpu, it_gpu, tol, max_iter, d=0.85):
    ref, it_ref, _ = oracle.pagerank(A, d, tol, max_iter)
    g = to_np(r_gpu).astype(np.float64)
    scale = np.max(ref)
    bound = (2 * max(it_ref, 1) * tol + 2e-5) * scale
    err = np.max(np.abs(g - ref))
    assert err <= bound, f"max |rank - oracle| {err:.3e} > {bound:.3e} (iters gpu {it_gpu} oracle {it_ref})"
    assert abs(it_gpu - it_ref) <= max(2, it_ref // 10)
    return ref, it_ref


@pytest.mark.parametrize("sym", [True, False])
def test_pagerank_rmat(spv, sym):
    A = synth.rmat(14, 16, seed=71, symmetrize=sym)
    M = spv.Matrix.from_csc(A, pattern=True)
    r, it = M.pagerank(0.85, 1e-6, 100)
    check(A, r, it, 1e-6, 100)


def test_pagerank_fixed_steps_match_closely(spv):
    """tol = 0: every reached vertex stays active, both sides run exactly
    max_iter multiplies and differ only by fp32 rounding."""
    A = synth.rmat(12, 8, seed=72, symmetrize=False)
    M = spv.Matrix.from_csc(A, pattern=True)
    r, it = M.pagerank(0.85, 0.0, 30)
    ref, it_ref, _ = oracle.pagerank(A, 0.85, 0.0, 30)
    assert it == it_ref == 30
    g = to_np(r).astype(np.float64)
    assert np.max(np.abs(g - ref) / ref) < 2e-5


def test_pagerank_grid_and_residual(spv):
    A = synth.grid(16, 16, 8)
    M = spv.Matrix.from_csc(A, pattern=True)
    tol = 1e-5
    r, it = M.pagerank(0.85, tol, 200)
    ref, it_ref = check(A, r, it, tol, 200)
    g = to_np(r).astype(np.float64)
    # residual of the fixed-point equation, p - (1-d)/n - d A_n p
    deg = np.diff(A.colptr).astype(np.float64)
    push = np.zeros(A.n)
    cols = np.repeat(np.arange(A.n), np.diff(A.colptr))
    np.add.at(push, A.rowids, 0.85 * g[cols] / deg[cols])
    res = g - 0.15 / A.n - push
    assert np.max(np.abs(res)) <= 4 * it * tol * np.max(g)
    assert abs(g.sum() - 1.0) < 1e-3                   # no dangling vertices: mass ~ 1


@pytest.mark.parametrize("cls", [2, 9])
def test_pagerank_with_selector(spv, cls):
    A = synth.rmat(13, 16, seed=73, symmetrize=True)
    M = spv.Matrix.from_csc(A, pattern=True, flags=spv.SYMMETRIC)
    p = np.zeros(spv.MLP_PARAMS, np.float32)
    p[-10 + cls] = 5.0
    M.load_selector(p, np.zeros(6, np.float32), np.ones(6, np.float32))
    r, it = M.pagerank(0.85, 1e-6, 100, flags=spv.USE_SELECTOR)
    check(A, r, it, 1e-6, 100)
    assert M.selector_classes() == [cls] * it


@pytest.mark.parametrize("cls", [2, 9])
def test_pagerank_with_selector_on_device(spv, cls):
    """Direction consumed on the device (no host read per multiply): same
    ranks as the oracle whichever direction the network picks."""
    A = synth.rmat(13, 16, seed=75, symmetrize=True)
    M = spv.Matrix.from_csc(A, pattern=True, flags=spv.SYMMETRIC)
    p = np.zeros(spv.MLP_PARAMS, np.float32)
    p[-10 + cls] = 5.0
    M.load_selector(p, np.zeros(6, np.float32), np.ones(6, np.float32))
    r, it = M.pagerank(0.85, 1e-6, 100, flags=spv.USE_SELECTOR | spv.USE_GRAPH)
    check(A, r, it, 1e-6, 100)


def test_pagerank_bad_arguments(spv):
    A = synth.rmat(10, 8, seed=74, symmetrize=True)
    Mv = spv.Matrix.from_csc(A)                        # has values
    with pytest.raises(spv.SpmspvError):
        Mv.pagerank()
    M = spv.Matrix.from_csc(A, pattern=True)
    with pytest.raises(spv.SpmspvError):
        M.pagerank(damping=1.5)
    with pytest.raises(spv.SpmspvError):
        M.pagerank(tol=-1.0)
    r, it = M.pagerank(max_iter=0)                     # no multiply: rank = (1-d)/n
    assert it == 0 and np.allclose(to_np(r), 0.15 / A.n)
