"""GPU connected components (cc_run: data-driven label propagation by
min-select2nd SpMSpV) against the oracle, label for label: symmetric and
directed R-MAT graphs, a 3-D grid, the benchmark's scale-22 graph, and a
persistent BFS on the same handle afterwards (cc_run borrows its scratch)."""
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


@pytest.mark.parametrize("scale,ef,sym,seed", [(14, 16, True, 1), (16, 4, True, 2), (12, 2, False, 3),
                                               (13, 1, True, 4), (10, 8, False, 5)])
def test_rmat_against_oracle(spv, scale, ef, sym, seed):
    A = synth.rmat(scale, ef, seed=seed, symmetrize=sym, with_values=False)
    M = spv.Matrix.from_csc(A, pattern=True)
    lab, it = M.connected_components()
    ref, k = oracle.cc(A)
    assert np.array_equal(to_np(lab), ref)
    assert it >= 1
    M.close()


def test_matrix_with_values_and_repeat(spv):
    """Values are ignored (min-select2nd); a second run on the same handle
    gives the same labels."""
    A = synth.rmat(13, 8, seed=6, symmetrize=True)
    M = spv.Matrix.from_csc(A)
    ref, _ = oracle.cc(A)
    for _ in range(2):
        lab, _ = M.connected_components()
        assert np.array_equal(to_np(lab), ref)
    M.close()


def test_grid_then_persistent_bfs(spv):
    """A connected 3-D grid: every label 0, reached after its eccentricity
    from vertex 0 (nx + ny + nz - 3 steps, plus the last one that changes
    nothing); then the persistent BFS on the same handle still matches."""
    nx, ny, nz = 24, 20, 12
    A = synth.grid(nx, ny, nz)
    M = spv.Matrix.from_csc(A, pattern=True)
    lab, it = M.connected_components()
    assert not to_np(lab).any()
    assert it == nx + ny + nz - 3 + 1
    lev, _, nl = M.bfs(0, spv.OR_AND_BOOL, parents=False, flags=spv.PERSISTENT)
    olev, _, onl = oracle.bfs(A, 0)
    assert nl == onl and np.array_equal(to_np(lev), olev)
    M.close()


def test_rectangular_refused(spv):
    rows = np.array([0, 1, 2], np.int32)
    cols = np.array([0, 0, 1], np.int32)
    colptr, rowids = synth.coo_to_csc(3, 2, rows, cols, drop_self=False)
    M = spv.Matrix(3, 2, colptr, rowids, None)
    with pytest.raises(spv.SpmspvError) as e:
        M.connected_components()
    assert e.value.status == spv.EINVAL
    M.close()


def test_full_size_rmat22(spv):
    """The benchmark's graph (R-MAT scale 22, symmetrised; 43 % isolated
    vertices, each its own component)."""
    A = synth.rmat(22, 16, seed=1, symmetrize=True, with_values=False)
    M = spv.Matrix.from_csc(A, pattern=True)
    lab, it = M.connected_components()
    ref, k = oracle.cc(A)
    assert np.array_equal(to_np(lab), ref)
    assert k > A.n // 3
    M.close()
