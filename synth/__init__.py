"""Seeded synthetic inputs (R-MAT and grid graphs in CSC, sparse vectors).

This module only builds inputs.  It holds none of the sparse
matrix-sparse vector arithmetic, so the GPU library and the CPU oracle can
both consume its outputs without sharing any of the method's code.

The C core (``csrc/synth.c``) is compiled with gcc into ``_synth.so`` next
to this file by :func:`build` and loaded through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "synth.c")
_LIB_PATH = os.path.join(_HERE, "_synth.so")
_lib = None

# Value streams: matrix values use stream 7; x vector r uses 64 + r.
_STREAM_A_VALUES = 7
_STREAM_X_VALUES = 64


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (-O3, OpenMP)."""
    global _lib
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
        _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, u64, i32p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        lib.synth_rmat_tuples.argtypes = [ctypes.c_int, i64, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, u64, i32p, i32p]
        lib.synth_permutation.argtypes = [i64, u64, i32p]
        lib.synth_coo_to_csc.argtypes = [i64, i64, i64, i32p, i32p, i32p, ctypes.c_int, ctypes.c_int,
                                         i32p, i32p]
        lib.synth_coo_to_csc.restype = i64
        lib.synth_values.argtypes = [i64, u64, u64, i32p]
        lib.synth_distinct.argtypes = [i64, i64, u64, u64, i32p]
        lib.synth_distinct.restype = ctypes.c_int
        lib.synth_grid_csc.argtypes = [i64, i64, i64, ctypes.c_int, i32p, i32p]
        lib.synth_grid_csc.restype = i64
        lib.synth_roots.argtypes = [i64, i32p, ctypes.c_int, u64, i32p]
        lib.synth_roots.restype = ctypes.c_int
        lib.synth_log_uniform.argtypes = [ctypes.c_int, ctypes.c_double, u64, i32p]
        lib.synth_draw.argtypes = [u64, u64, u64]
        lib.synth_draw.restype = u64
        _lib = lib
    return _lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class CSC:
    """A sparse matrix in compressed sparse column form (int32 indices)."""
    m: int
    n: int
    colptr: np.ndarray          # int32[n+1]
    rowids: np.ndarray          # int32[nnz]
    values: Optional[np.ndarray]  # float32[nnz] or None (pattern matrix)
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.colptr.astype(np.int64))

    def to_scipy(self):
        import scipy.sparse as sp
        vals = self.values if self.values is not None else np.ones(self.nnz, np.float32)
        return sp.csc_matrix((vals.astype(np.float64), self.rowids, self.colptr), shape=(self.m, self.n))


@dataclass
class DCSC:
    """A sparse matrix in doubly compressed sparse column form: only the nzc
    non-empty columns are stored, their ids ascending in jc and their
    entries at [cp[k], cp[k+1]) of rowids / values (int32 indices)."""
    m: int
    n: int
    jc: np.ndarray              # int32[nzc]
    cp: np.ndarray              # int32[nzc+1]
    rowids: np.ndarray          # int32[nnz]
    values: Optional[np.ndarray]  # float32[nnz] or None (pattern matrix)
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.cp[-1])

    @property
    def nzc(self) -> int:
        return int(self.jc.size)


def csc_to_dcsc(A: CSC) -> DCSC:
    """The same matrix with its empty columns dropped (a format change only)."""
    jc = np.nonzero(np.diff(A.colptr.astype(np.int64)) > 0)[0].astype(np.int32)
    cp = np.empty(jc.size + 1, np.int32)
    cp[:-1] = A.colptr[jc]
    cp[-1] = A.colptr[-1]
    return DCSC(A.m, A.n, jc, cp, A.rowids, A.values, A.name + "-dcsc")


def column_subset(A: CSC, keep: np.ndarray) -> CSC:
    """A with every column outside `keep` (a boolean mask over columns)
    emptied: a way to make hypersparse inputs from the generators' graphs."""
    keep = np.asarray(keep, bool)
    lens = np.where(keep, np.diff(A.colptr.astype(np.int64)), 0)
    colptr = np.zeros(A.n + 1, np.int64)
    colptr[1:] = np.cumsum(lens)
    sel = np.repeat(keep, np.diff(A.colptr.astype(np.int64)))
    vals = None if A.values is None else A.values[sel].copy()
    return CSC(A.m, A.n, colptr.astype(np.int32), A.rowids[sel].copy(), vals, A.name + "-cols")


def values(count: int, seed: int, stream: int = _STREAM_A_VALUES) -> np.ndarray:
    out = np.empty(count, np.float32)
    if count:
        _load().synth_values(count, seed, stream, _p(out))
    return out


def coo_to_csc(m: int, n: int, rows: np.ndarray, cols: np.ndarray, perm: Optional[np.ndarray] = None,
               symmetrize: bool = False, drop_self: bool = True) -> tuple[np.ndarray, np.ndarray]:
    rows = np.ascontiguousarray(rows, np.int32)
    cols = np.ascontiguousarray(cols, np.int32)
    nt = rows.size
    colptr = np.empty(n + 1, np.int32)
    rowids = np.empty(max(1, (2 if symmetrize else 1) * nt), np.int32)
    pp = _p(np.ascontiguousarray(perm, np.int32)) if perm is not None else None
    if perm is not None:
        perm = np.ascontiguousarray(perm, np.int32)
        pp = _p(perm)
    nnz = _load().synth_coo_to_csc(m, n, nt, _p(rows), _p(cols), pp, int(symmetrize), int(drop_self),
                                   _p(colptr), _p(rowids))
    return colptr, rowids[:nnz].copy()


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, symmetrize: bool = False, relabel: bool = True, with_values: bool = True) -> CSC:
    """R-MAT graph (Chakrabarti, Zhan, Faloutsos 2004) as an n x n CSC matrix.

    edge_factor * 2^scale tuples, optional seeded vertex relabelling, optional
    symmetrisation; self loops and duplicate entries removed.  Values, when
    requested, are uniform on (0, 1] on the 2^-24 grid.
    """
    n = 1 << scale
    nt = edge_factor * n
    lib = _load()
    rows = np.empty(nt, np.int32)
    cols = np.empty(nt, np.int32)
    lib.synth_rmat_tuples(scale, nt, a, b, c, seed, _p(rows), _p(cols))
    perm = None
    if relabel:
        perm = np.empty(n, np.int32)
        lib.synth_permutation(n, seed, _p(perm))
    colptr, rowids = coo_to_csc(n, n, rows, cols, perm, symmetrize, True)
    del rows, cols
    vals = values(int(colptr[-1]), seed) if with_values else None
    name = f"rmat-s{scale}-ef{edge_factor}{'-sym' if symmetrize else ''}{'' if relabel else '-raw'}"
    return CSC(n, n, colptr, rowids, vals, name)


def grid(nx: int, ny: int, nz: int = 1, diag: bool = True, with_values: bool = False, seed: int = 1) -> CSC:
    """2-D 5-point (nz == 1) or 3-D 7-point grid adjacency, v = x + nx*y + nx*ny*z."""
    n = nx * ny * nz
    per = 1 + (2 if nx > 1 else 0) + (2 if ny > 1 else 0) + (2 if nz > 1 else 0)
    colptr = np.empty(n + 1, np.int32)
    rowids = np.empty(n * per, np.int32)
    nnz = _load().synth_grid_csc(nx, ny, nz, int(diag), _p(colptr), _p(rowids))
    rowids = rowids[:nnz]
    vals = values(nnz, seed) if with_values else None
    return CSC(n, n, colptr, rowids, vals, f"grid-{nx}x{ny}x{nz}")


def distinct_indices(n: int, f: int, seed: int, tag: int = 0, sort: bool = False) -> np.ndarray:
    """f distinct uniform indices of [0, n) in random order (or ascending)."""
    out = np.empty(max(f, 1), np.int32)
    if f:
        rc = _load().synth_distinct(n, f, seed, tag, _p(out))
        if rc != 0:
            raise ValueError("f must be in [0, n]")
    out = out[:f]
    if sort:
        out.sort()
    return out


def sparse_x(n: int, f: int, seed: int, tag: int = 0, sort: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """Sparse vector x: f distinct uniform indices, values uniform on (0, 1] (2^-24 grid)."""
    idx = distinct_indices(n, f, seed, tag, sort)
    val = values(f, seed, _STREAM_X_VALUES + tag)
    return idx, val


def density_f(n: int, density: float) -> int:
    """Number of x entries for a frontier density: round(density * n)."""
    return int(np.floor(density * n + 0.5))


def roots(A: CSC, count: int, seed: int) -> np.ndarray:
    out = np.empty(count, np.int32)
    rc = _load().synth_roots(A.n, _p(A.colptr), count, seed, _p(out))
    if rc != 0:
        raise ValueError("graph has no non-empty column")
    return out


def log_uniform_sizes(count: int, hi: float, seed: int) -> np.ndarray:
    out = np.empty(count, np.int64)
    _load().synth_log_uniform(count, float(hi), seed, _p(out))
    return out


def draw(seed: int, stream: int, i: int) -> int:
    return int(_load().synth_draw(seed, stream, i))
