"""GPU BFS (repeated masked SpMSpV on the frontier) against the oracle's
queue BFS: levels exactly, parents by the minimum-parent rule exactly."""
import numpy as np
import pytest

import oracle
import synth

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


@pytest.fixture(scope="module")
def rmat16(spv):
    A = synth.rmat(16, seed=1, symmetrize=True, with_values=False)
    return A, spv.Matrix.from_csc(A)


@pytest.mark.parametrize("graph", [False, True])
def test_rmat_bfs_min_select2nd(spv, rmat16, graph):
    A, M = rmat16
    for root in synth.roots(A, 3, seed=2000):
        lev, par, nl = M.bfs(int(root), spv.MIN_SELECT2ND_I32, flags=spv.USE_GRAPH if graph else 0)
        olev, opar, onl = oracle.bfs(A, int(root))
        assert nl == onl
        assert np.array_equal(lev.cpu().numpy(), olev)
        assert np.array_equal(par.cpu().numpy(), opar)


def test_rmat_bfs_or_and(spv, rmat16):
    A, M = rmat16
    root = int(synth.roots(A, 1, seed=2001)[0])
    lev, par, nl = M.bfs(root, spv.OR_AND_BOOL, flags=spv.USE_GRAPH)
    olev, _, onl = oracle.bfs(A, root)
    assert par is None and nl == onl
    assert np.array_equal(lev.cpu().numpy(), olev)


@pytest.mark.parametrize("dims", [(40, 40, 40), (128, 96, 1)])
def test_grid_bfs_closed_form(spv, dims):
    nx, ny, nz = dims
    G = synth.grid(nx, ny, nz, diag=True)
    M = spv.Matrix.from_csc(G)
    lev, par, nl = M.bfs(0, spv.MIN_SELECT2ND_I32, flags=spv.USE_GRAPH)
    v = np.arange(G.n)
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    assert np.array_equal(lev.cpu().numpy(), x + y + z)
    assert nl == (nx - 1) + (ny - 1) + (nz - 1) + 1
    ep = np.where(z > 0, v - nx * ny, np.where(y > 0, v - nx, v - 1))
    ep[0] = 0
    assert np.array_equal(par.cpu().numpy(), ep)
    lev2, _, nl2 = M.bfs(0, spv.OR_AND_BOOL)
    assert nl2 == nl and np.array_equal(lev2.cpu().numpy(), x + y + z)


def test_isolated_root_and_directed(spv):
    A = synth.rmat(12, seed=9)    # directed: edges j -> i for stored A(i, j)
    M = spv.Matrix.from_csc(A)
    iso = int(np.nonzero((A.degrees() == 0))[0][0])
    lev, par, nl = M.bfs(iso, spv.MIN_SELECT2ND_I32)
    olev, opar, onl = oracle.bfs(A, iso)
    assert nl == onl and np.array_equal(lev.cpu().numpy(), olev) and np.array_equal(par.cpu().numpy(), opar)
    for root in synth.roots(A, 2, seed=5):
        lev, par, nl = M.bfs(int(root), spv.MIN_SELECT2ND_I32)
        olev, opar, onl = oracle.bfs(A, int(root))
        assert nl == onl and np.array_equal(lev.cpu().numpy(), olev) and np.array_equal(par.cpu().numpy(), opar)


def test_bfs_rejects_bad_arguments(spv, rmat16):
    A, M = rmat16
    lev = torch.empty(A.n, dtype=torch.int32, device="cuda")
    par = torch.empty(A.n, dtype=torch.int32, device="cuda")
    with pytest.raises(spv.SpmspvError):
        spv.bfs_run(M.handle, spv.PLUS_TIMES_F32, 0, 0, lev, par)
    with pytest.raises(spv.SpmspvError):
        spv.bfs_run(M.handle, spv.OR_AND_BOOL, 0, 0, lev, par)
    with pytest.raises(spv.SpmspvError):
        spv.bfs_run(M.handle, spv.MIN_SELECT2ND_I32, A.n, 0, lev, par)
