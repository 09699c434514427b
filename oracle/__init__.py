"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations (``oracle.c``,
plain C built with gcc) of what the GPU library computes.  Only the test
suite, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg
may import this package.  It shares no code with the GPU library.

Each function names the passage of the paper (Azad and Buluç, "A
work-efficient parallel sparse matrix-sparse vector multiplication
algorithm") it follows; see ``oracle.c`` for the C side.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

PLUS_TIMES, MIN_SELECT2ND, OR_AND = 0, 1, 2


def build(force: bool = True, src: Optional[str] = None, out: Optional[str] = None) -> str:
    """Compile the oracle (gcc -O2, no fast-math: fp64 semantics kept exact)."""
    global _lib
    src = src or _SRC
    out = out or _LIB_PATH
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", src, "-o", tmp,
                        "-lm"], check=True)
        os.replace(tmp, out)
        if out == _LIB_PATH:
            _lib = None
    return out


def _bind(lib):
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_validate.argtypes = [i64, i64, vp, vp, i64, vp]
    lib.oracle_spmspv.argtypes = [ctypes.c_int, i64, i64, vp, vp, vp, i64, vp, vp, vp, ctypes.c_int, vp, vp,
                                  vp, vp]
    lib.oracle_spmspv_f32seq.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, vp, vp]
    if hasattr(lib, "oracle_spmspv_graphblas"):
        ci = ctypes.c_int
        lib.oracle_spmspv_graphblas.argtypes = [ci, i64, i64, vp, vp, vp, i64, vp, vp, ci, vp, vp, i64, ci, ci, vp,
                                                vp, i64, ci, vp, vp, vp]
    if hasattr(lib, "oracle_spmspv_left"):
        lib.oracle_spmspv_left.argtypes = [ctypes.c_int, i64, i64, vp, vp, vp, i64, vp, vp, vp, vp, vp]
        lib.oracle_spmspv_left.restype = ctypes.c_int
    if hasattr(lib, "oracle_spmspv_dcsc"):
        lib.oracle_spmspv_dcsc.argtypes = [ctypes.c_int, i64, i64, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp,
                                           vp]
        lib.oracle_spmspv_dcsc.restype = ctypes.c_int
    if hasattr(lib, "oracle_cc"):
        lib.oracle_cc.argtypes = [i64, vp, vp, vp]
        lib.oracle_cc.restype = i64
    lib.oracle_bfs.argtypes = [i64, vp, vp, ctypes.c_int32, vp, vp]
    lib.oracle_bfs.restype = ctypes.c_int
    if hasattr(lib, "oracle_pagerank"):
        lib.oracle_pagerank.argtypes = [i64, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp, vp]
        lib.oracle_pagerank.restype = ctypes.c_int
    if hasattr(lib, "oracle_mlp_forward"):
        ci = ctypes.c_int
        lib.oracle_mlp_forward.argtypes = [ci, ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_mlp_loss_grad.argtypes = [ci, ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_mlp_loss_grad.restype = ctypes.c_double
    return lib


def load(path: Optional[str] = None):
    """Load (building if needed) the oracle library; `path` loads a variant build."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def validate(m, n, colptr, rowids, x_idx, lib=None) -> int:
    lib = lib or load()
    x_idx = np.ascontiguousarray(x_idx, np.int32)
    return int(lib.oracle_validate(m, n, _p(colptr), _p(rowids), x_idx.size, _p(x_idx)))


def spmspv(A, x_idx: np.ndarray, x_val: np.ndarray, semiring: int = PLUS_TIMES,
           mask: Optional[np.ndarray] = None, sorted_output: bool = False, lib=None):
    """y <- A x (Algorithm 1's result) with a dense accumulator.

    Returns (y_idx int32, y_val, W) with y_val float64 (plus-times),
    int32 (min-select2nd) or uint8 (or-and).  `A` is a ``synth.CSC``.
    """
    lib = lib or load()
    x_idx = np.ascontiguousarray(x_idx, np.int32)
    f = x_idx.size
    if semiring == PLUS_TIMES:
        xv = np.ascontiguousarray(x_val, np.float32)
        yv = np.empty(max(A.m, 1), np.float64)
    elif semiring == MIN_SELECT2ND:
        xv = np.ascontiguousarray(x_val, np.int32)
        yv = np.empty(max(A.m, 1), np.int32)
    elif semiring == OR_AND:
        xv = np.ascontiguousarray(x_val, np.uint8)
        yv = np.empty(max(A.m, 1), np.uint8)
    else:
        raise ValueError("semiring")
    yi = np.empty(max(A.m, 1), np.int32)
    mk = None if mask is None else np.ascontiguousarray(mask, np.uint8)
    nnz = ctypes.c_int64(0)
    W = ctypes.c_int64(0)
    vals = None if A.values is None else np.ascontiguousarray(A.values, np.float32)
    rc = lib.oracle_spmspv(semiring, A.m, A.n, _p(A.colptr), _p(A.rowids), _p(vals), f, _p(x_idx), _p(xv),
                           _p(mk), int(bool(sorted_output)), _p(yi), _p(yv), ctypes.byref(nnz), ctypes.byref(W))
    if rc != 0:
        raise ValueError(f"oracle_spmspv rc={rc}")
    k = nnz.value
    return yi[:k].copy(), yv[:k].copy(), W.value


def _xv(semiring, x_val):
    dt = {PLUS_TIMES: np.float32, MIN_SELECT2ND: np.int32, OR_AND: np.uint8}[semiring]
    return np.ascontiguousarray(x_val, dt)


def _yv(semiring, size):
    dt = {PLUS_TIMES: np.float64, MIN_SELECT2ND: np.int32, OR_AND: np.uint8}[semiring]
    return np.empty(max(size, 1), dt)


def spmspv_left(A, x_idx: np.ndarray, x_val: np.ndarray, semiring: int = PLUS_TIMES, lib=None):
    """Left multiplication y' <- x' A (Background, Notation: the row-vector
    case): x' over A's rows, y' over its columns, y'(j) = Add over stored
    A(i,j) with i in x' of Mult(A(i,j), x'(i)).  Column-driven with a dense
    x'.  Returns (y_idx ascending, y_val) with y_val typed as in spmspv."""
    lib = lib or load()
    x_idx = np.ascontiguousarray(x_idx, np.int32)
    xv = _xv(semiring, x_val)
    yi = np.empty(max(A.n, 1), np.int32)
    yv = _yv(semiring, A.n)
    nnz = ctypes.c_int64(0)
    vals = None if A.values is None else np.ascontiguousarray(A.values, np.float32)
    rc = lib.oracle_spmspv_left(semiring, A.m, A.n, _p(A.colptr), _p(A.rowids), _p(vals), x_idx.size, _p(x_idx),
                                _p(xv), _p(yi), _p(yv), ctypes.byref(nnz))
    if rc != 0:
        raise ValueError(f"oracle_spmspv_left rc={rc}")
    k = nnz.value
    return yi[:k].copy(), yv[:k].copy()


def spmspv_dcsc(D, x_idx: np.ndarray, x_val: np.ndarray, semiring: int = PLUS_TIMES, lib=None):
    """y <- A x with A in DCSC (``synth.DCSC``; Background, Sparse matrix and
    vector data structures): columns looked up by binary search over the
    non-empty column ids.  Returns (y_idx ascending, y_val, W)."""
    lib = lib or load()
    x_idx = np.ascontiguousarray(x_idx, np.int32)
    xv = _xv(semiring, x_val)
    yi = np.empty(max(D.m, 1), np.int32)
    yv = _yv(semiring, D.m)
    nnz = ctypes.c_int64(0)
    W = ctypes.c_int64(0)
    vals = None if D.values is None else np.ascontiguousarray(D.values, np.float32)
    rc = lib.oracle_spmspv_dcsc(semiring, D.m, D.n, D.nzc, _p(np.ascontiguousarray(D.jc, np.int32)),
                                _p(np.ascontiguousarray(D.cp, np.int32)), _p(np.ascontiguousarray(D.rowids, np.int32)),
                                _p(vals), x_idx.size, _p(x_idx), _p(xv), _p(yi), _p(yv), ctypes.byref(nnz),
                                ctypes.byref(W))
    if rc != 0:
        raise ValueError(f"oracle_spmspv_dcsc rc={rc}")
    k = nnz.value
    return yi[:k].copy(), yv[:k].copy(), W.value


def to_bitvector(idx: np.ndarray, val: Optional[np.ndarray], length: int):
    """Bitvector form of a sparse vector (Background, Sparse matrix and
    vector data structures): a bitmap of `length` bits in uint32 words, bit
    (i mod 32) of word i div 32 set for every present index i, and the
    values listed in ascending index order.  Returns (bits, values)."""
    idx = np.asarray(idx, np.int64)
    bits = np.zeros((length + 31) // 32, np.uint32)
    for i in idx.tolist():
        bits[i >> 5] |= np.uint32(1 << (i & 31))
    order = np.argsort(idx, kind="stable")
    return bits, (None if val is None else np.asarray(val)[order])


def from_bitvector(bits: np.ndarray, length: int) -> np.ndarray:
    """Present indices of a bitmap, ascending (bits at or past `length`
    must be clear)."""
    b = np.unpackbits(np.ascontiguousarray(bits, "<u4").view(np.uint8), bitorder="little")
    if b[length:].any():
        raise ValueError("bit set past the vector length")
    return np.nonzero(b[:length])[0].astype(np.int32)


ACCUM_NONE, ACCUM_ADD, ACCUM_FIRST, ACCUM_SECOND = 0, 1, 2, 3


def spmspv_graphblas(A, x_idx: np.ndarray, x_val: np.ndarray, semiring: int = PLUS_TIMES,
                     mask_idx: Optional[np.ndarray] = None, mask_val: Optional[np.ndarray] = None,
                     complement: bool = False, w_idx: Optional[np.ndarray] = None,
                     w_val: Optional[np.ndarray] = None, accum: int = ACCUM_NONE, replace: bool = False,
                     lib=None):
    """w<mask, replace> = w accum (A x), the GraphBLAS rules on top of
    Algorithm 1's product (the masked SpMSpV of the paper's conclusions).

    mask_idx None: every row is in the mask (complement: none is);
    mask_val None: structural mask, else a row counts only if its value is
    nonzero.  w_val: plus-times float64, min-select2nd int32, or-and uint8.
    Returns (y_idx int32 ascending, y_val).
    """
    lib = lib or load()
    x_idx = np.ascontiguousarray(x_idx, np.int32)
    dt = {PLUS_TIMES: np.float64, MIN_SELECT2ND: np.int32, OR_AND: np.uint8}[semiring]
    xdt = {PLUS_TIMES: np.float32, MIN_SELECT2ND: np.int32, OR_AND: np.uint8}[semiring]
    xv = np.ascontiguousarray(x_val, xdt)
    has_mask = mask_idx is not None
    mi = np.ascontiguousarray(mask_idx if has_mask else np.zeros(0), np.int32)
    mv = None if mask_val is None else np.ascontiguousarray(mask_val, np.uint8)
    wi = np.ascontiguousarray(np.zeros(0) if w_idx is None else w_idx, np.int32)
    wv = np.ascontiguousarray(np.zeros(wi.size) if w_val is None else w_val, dt)
    yi = np.empty(max(A.m, 1), np.int32)
    yv = np.empty(max(A.m, 1), dt)
    nnz = ctypes.c_int64(0)
    vals = None if A.values is None else np.ascontiguousarray(A.values, np.float32)
    rc = lib.oracle_spmspv_graphblas(semiring, A.m, A.n, _p(A.colptr), _p(A.rowids), _p(vals), x_idx.size,
                                     _p(x_idx), _p(xv), int(has_mask), _p(mi), _p(mv), mi.size, int(bool(complement)),
                                     int(accum), _p(wi), _p(wv), wi.size, int(bool(replace)), _p(yi), _p(yv),
                                     ctypes.byref(nnz))
    if rc != 0:
        raise ValueError(f"oracle_spmspv_graphblas rc={rc}")
    k = nnz.value
    return yi[:k].copy(), yv[:k].copy()


def cc(A, lib=None):
    """Connected components (a data-driven SpMSpV use named in the paper's
    introduction): label(v) = the smallest vertex that reaches v along edges
    j -> i of the stored A(i, j); for a symmetric A, the smallest vertex of
    v's component.  Returns (labels int32 [n], number of components)."""
    lib = lib or load()
    lab = np.empty(max(A.n, 1), np.int32)
    k = lib.oracle_cc(A.n, _p(A.colptr), _p(A.rowids), _p(lab))
    return lab[: A.n].copy(), int(k)


def spmspv_f32seq(A, x_idx: np.ndarray, x_val: np.ndarray, lib=None):
    """Plus-times accumulated in fp32 in x order; returns (y_idx, y_val float32)."""
    lib = lib or load()
    x_idx = np.ascontiguousarray(x_idx, np.int32)
    xv = np.ascontiguousarray(x_val, np.float32)
    yi = np.empty(max(A.m, 1), np.int32)
    yv = np.empty(max(A.m, 1), np.float32)
    nnz = ctypes.c_int64(0)
    vals = None if A.values is None else np.ascontiguousarray(A.values, np.float32)
    lib.oracle_spmspv_f32seq(A.m, _p(A.colptr), _p(A.rowids), _p(vals), x_idx.size, _p(x_idx), _p(xv), _p(yi),
                             _p(yv), ctypes.byref(nnz))
    k = nnz.value
    return yi[:k].copy(), yv[:k].copy()


def bfs(A, root: int, lib=None):
    """Queue BFS: (levels int32[n], parents int32[n] by the minimum-parent rule, num_levels)."""
    lib = lib or load()
    lev = np.empty(A.n, np.int32)
    par = np.empty(A.n, np.int32)
    nl = lib.oracle_bfs(A.n, _p(A.colptr), _p(A.rowids), int(root), _p(lev), _p(par))
    return lev, par, int(nl)


def pagerank(A, damping: float = 0.85, tol: float = 1e-6, max_iter: int = 100, lib=None):
    """Data-driven (delta) PageRank in fp64: (rank float64[n], multiplies, active counts per step)."""
    lib = lib or load()
    rank = np.empty(A.n, np.float64)
    act = np.zeros(max_iter + 1, np.int32)
    it = lib.oracle_pagerank(A.n, _p(A.colptr), _p(A.rowids), float(damping), float(tol), int(max_iter), _p(rank),
                             _p(act))
    return rank, int(it), act[:it + 1].copy()


# ------------------------------------------------------------ selector MLP
MLP_SHAPE = (6, 64, 64, 10)


def mlp_param_count(shape=MLP_SHAPE) -> int:
    i, h1, h2, o = shape
    return h1 * i + h1 + h2 * h1 + h2 + o * h2 + o


def mlp_forward(params, X, shape=MLP_SHAPE, lib=None):
    """fp64 logits [B][out] of the selector MLP (6 -> 64 ReLU -> 64 ReLU -> 10)."""
    lib = lib or load()
    i, h1, h2, o = shape
    p = np.ascontiguousarray(params, np.float64)
    X = np.ascontiguousarray(X, np.float64)
    B = X.shape[0]
    out = np.empty((B, o), np.float64)
    lib.oracle_mlp_forward(i, h1, h2, o, B, _p(p), _p(X), _p(out), None, None, None, None)
    return out


def mlp_loss_grad(params, X, labels, shape=MLP_SHAPE, lib=None):
    """(mean softmax cross-entropy, gradient in the parameter layout), fp64."""
    lib = lib or load()
    i, h1, h2, o = shape
    p = np.ascontiguousarray(params, np.float64)
    X = np.ascontiguousarray(X, np.float64)
    y = np.ascontiguousarray(labels, np.int32)
    g = np.empty(mlp_param_count(shape), np.float64)
    loss = lib.oracle_mlp_loss_grad(i, h1, h2, o, X.shape[0], _p(p), _p(X), _p(y), _p(g), None, None, None, None)
    return float(loss), g
