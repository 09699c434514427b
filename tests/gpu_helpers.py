"""Shared helpers of the GPU parity tests (compare the HIP path with the oracle)."""
import functools

import numpy as np

# fp32 plus-times contract: |y - y64| <= REL_TOL * sum_k |term_k|; every input
# value is positive here, so sum_k |term_k| = y64.
REL_TOL = 1e-5


def to_np(t):
    return t.detach().cpu().numpy()


def sort_pair(idx, val):
    o = np.argsort(idx, kind="stable")
    return idx[o], val[o]


def compare(semiring, g_idx, g_val, o_idx, o_val, sorted_output=False, terms_abs=None):
    """Element-by-element comparison of one GPU output with the oracle's."""
    gi = to_np(g_idx).astype(np.int64)
    gv = to_np(g_val)
    if sorted_output:
        assert np.all(np.diff(gi) > 0), "sorted output is not strictly ascending"
    gi, gv = sort_pair(gi, gv)
    oi, ov = sort_pair(np.asarray(o_idx, np.int64), np.asarray(o_val))
    assert gi.size == oi.size, f"nnz(y) {gi.size} != oracle {oi.size}"
    assert np.array_equal(gi, oi), "index sets differ"
    if semiring == 0:
        ref = ov.astype(np.float64)
        bound = REL_TOL * (np.abs(ref) if terms_abs is None else terms_abs)
        err = np.abs(gv.astype(np.float64) - ref)
        bad = np.nonzero(~(err <= bound))[0]   # written so that a NaN counts as outside
        assert bad.size == 0, f"{bad.size} values outside tolerance, worst rel {np.max(err / np.maximum(np.abs(ref), 1e-300))}"
    elif semiring == 1:
        bad = np.nonzero(gv.astype(np.int64) != ov.astype(np.int64))[0]
        assert bad.size == 0, f"{bad.size} int32 values differ, e.g. rows {gi[bad[:5]]} gpu {gv[bad[:5]]} oracle {ov[bad[:5]]}"
    else:
        bad = np.nonzero(gv.astype(np.uint8) != ov.astype(np.uint8))[0]
        assert bad.size == 0, f"{bad.size} bool values differ, e.g. rows {gi[bad[:5]]} gpu {gv[bad[:5]]} oracle {ov[bad[:5]]}"


@functools.lru_cache(maxsize=1)
def rmat24_pattern():
    """The held-out evaluation graph (R-MAT scale 24, edge factor 16,
    symmetrised, pattern only: 16,777,216 vertices, 520,757,406 stored
    entries), generated once per test session."""
    import synth
    A = synth.rmat(24, 16, seed=24, symmetrize=True, with_values=False)
    assert (A.n, A.nnz) == (16777216, 520757406)
    return A
