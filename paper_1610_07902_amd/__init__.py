"""SpMSpV-bucket on MI355X: Python binding of libspmspv.so.

The functions below have the names of the C ABI in ``include/spmspv.h`` and
only marshal arguments: every step of the computation runs in the library's
HIP kernels.  PyTorch provides device memory and the HIP stream.  Importing
the binding fails loudly when the library has not been built; there is no
CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmspv.so")

PLUS_TIMES_F32 = 0
MIN_SELECT2ND_I32 = 1
OR_AND_BOOL = 2

SORTED_OUTPUT = 1
VALIDATE = 2
X_VAL_IS_INDEX = 4
X_ALL_TRUE = 8
USE_GRAPH = 16
PROFILE = 32
WITH_TRANSPOSE = 64
SYMMETRIC = 128
DIRECTION_OPT = 256
USE_SELECTOR = 512
MSBFS = 1024
AUTO_SCHEDULE = 2048
PULL_ROWWISE = 4096
PERSISTENT = 8192
LEFT = 16384
DETERMINISTIC = 32768

MLP_PARAMS = 5258
NUM_CLASSES = 10

OK, EINVAL, ENOMEM, ECAPACITY, EHIP, EUNSUPPORTED, EDEVICE = 0, -1, -2, -3, -4, -5, -6

EXPORTED = (
    "spmspv_workspace_size", "spmspv_create", "spmspv_run", "bfs_run", "spmspv_get_schedule",
    "spmspv_set_schedule", "spmspv_last_stats", "spmspv_profile_read", "spmspv_destroy",
    "spmspv_status_string", "spmspv_last_error", "spmspv_run_masked", "spmspv_selector_load",
    "spmspv_selector_classes", "spmspv_class_tile", "spmspv_mlp_param_count", "spmspv_mlp_forward",
    "spmspv_mlp_train_step", "spmspv_batch_workspace_size", "spmspv_batch_attach", "spmspv_run_batch",
    "spmspv_set_batch_schedule", "spmspv_get_batch_schedule", "msbfs_run", "spmspv_autotune",
    "spmspv_tuned_schedule", "spmspv_autotune_batch", "pagerank_scratch_size", "pagerank_run",
    "spmspv_selector_features", "spmspv_force_classes", "spmspv_effective_schedule", "spmspv_run_static", "spmspv_run_graphblas", "cc_run",
    "spmspv_dcsc_workspace_size", "spmspv_create_dcsc", "spmspv_run_bitvector", "spmspv_class_schedule",
    "spmspv_tuning_save", "spmspv_tuning_load", "spmspv_source_digest",
)


class SpmspvError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"status {status}: {message}")
        self.status = status


class Schedule(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int), ("tile_log2", ctypes.c_int), ("scatter_block", ctypes.c_int),
                ("scatter_items", ctypes.c_int), ("merge_block", ctypes.c_int), ("merge_variant", ctypes.c_int),
                ("launch", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [("density", ctypes.c_double), ("f", ctypes.c_int64), ("sched", Schedule), ("us", ctypes.c_double),
                ("default_us", ctypes.c_double)]

    def as_dict(self):
        return {"density": self.density, "f": self.f, "sched": self.sched.as_dict(), "us": self.us,
                "default_us": self.default_us}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libspmspv.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    # PyTorch provides the device memory and streams: load its HIP runtime
    # first so the library binds to the same runtime instance.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    i64, vp, ci, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    lib.spmspv_workspace_size.argtypes = [i64, i64, i64, ci, ctypes.POINTER(sz)]
    lib.spmspv_create.argtypes = [ctypes.POINTER(vp), i64, i64, i64, vp, vp, vp, vp, sz, ci, vp]
    lib.spmspv_run.argtypes = [vp, ci, ci, i64, vp, vp, vp, vp, i64, vp, ctypes.POINTER(i64), vp]
    lib.bfs_run.argtypes = [vp, ci, ctypes.c_int32, ci, vp, vp, ctypes.POINTER(ctypes.c_int32), vp]
    lib.spmspv_get_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
    lib.spmspv_set_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
    lib.spmspv_effective_schedule.argtypes = [vp, ci, i64, ci, ctypes.POINTER(Schedule)]
    lib.spmspv_last_stats.argtypes = [vp, ctypes.POINTER(i64), vp]
    lib.spmspv_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.spmspv_destroy.argtypes = [vp]
    lib.spmspv_status_string.argtypes = [ci]
    lib.spmspv_status_string.restype = ctypes.c_char_p
    lib.spmspv_run_masked.argtypes = [vp, ci, ci, i64, vp, vp, vp, vp, vp, i64, vp, ctypes.POINTER(i64), vp]
    lib.spmspv_run_static.argtypes = [i64, i64, i64, vp, vp, vp, ci, ci, i64, vp, vp, vp, vp, i64, vp,
                                      ctypes.POINTER(i64), ctypes.POINTER(sz), vp]
    lib.cc_run.argtypes = [vp, ci, vp, ctypes.POINTER(ctypes.c_int32), vp]
    lib.spmspv_dcsc_workspace_size.argtypes = [i64, i64, i64, i64, ci, ctypes.POINTER(sz)]
    lib.spmspv_create_dcsc.argtypes = [ctypes.POINTER(vp), i64, i64, i64, i64, vp, vp, vp, vp, vp, sz, ci, vp]
    lib.spmspv_run_bitvector.argtypes = [vp, ci, ci, vp, vp, vp, vp, i64, vp, ctypes.POINTER(i64), vp]
    lib.spmspv_run_graphblas.argtypes = [vp, ci, ci, i64, vp, vp, vp, vp, i64, ci, ci, vp, vp, i64, vp, vp, i64,
                                         vp, ctypes.POINTER(i64), vp]
    lib.spmspv_selector_load.argtypes = [vp, vp, vp, vp, vp]
    lib.spmspv_selector_classes.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.spmspv_class_tile.argtypes = [vp, ci, ctypes.POINTER(ctypes.c_int32)]
    lib.spmspv_class_schedule.argtypes = [vp, ci, ci, ctypes.POINTER(Schedule)]
    lib.spmspv_tuning_save.argtypes = [vp, ctypes.c_char_p, vp]
    lib.spmspv_tuning_load.argtypes = [vp, ctypes.c_char_p, vp]
    lib.spmspv_source_digest.argtypes = []
    lib.spmspv_source_digest.restype = ctypes.c_char_p
    lib.spmspv_mlp_param_count.argtypes = []
    lib.spmspv_mlp_forward.argtypes = [vp, vp, ci, vp, vp]
    lib.spmspv_mlp_train_step.argtypes = [vp, vp, vp, ci, ctypes.c_float, vp, vp, ci, vp, vp, vp]
    lib.spmspv_batch_workspace_size.argtypes = [vp, ci, i64, i64, ci, ctypes.POINTER(sz)]
    lib.spmspv_batch_attach.argtypes = [vp, ci, i64, i64, ci, vp, sz, vp]
    lib.spmspv_run_batch.argtypes = [vp, ci, ci, ci, vp, vp, vp, vp, vp, vp, i64, ctypes.POINTER(i64), vp]
    lib.spmspv_set_batch_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
    lib.spmspv_get_batch_schedule.argtypes = [vp, ci, ci, ctypes.POINTER(Schedule)]
    lib.msbfs_run.argtypes = [vp, ci, ci, vp, ci, vp, vp, ctypes.POINTER(ctypes.c_int32), vp]
    lib.spmspv_autotune.argtypes = [vp, ci, ctypes.POINTER(ctypes.c_double), ci, ci, vp, vp, vp, vp,
                                    ctypes.POINTER(TuneEntry), vp]
    lib.spmspv_tuned_schedule.argtypes = [vp, i64, ctypes.POINTER(Schedule)]
    lib.spmspv_autotune_batch.argtypes = [vp, ci, ci, ci, vp, vp, vp, vp, vp, vp, i64, ci, ctypes.POINTER(Schedule),
                                          ctypes.POINTER(ctypes.c_double), vp]
    lib.spmspv_selector_features.argtypes = [vp, ctypes.POINTER(ctypes.c_float), vp]
    lib.spmspv_force_classes.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    lib.pagerank_scratch_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.pagerank_run.argtypes = [vp, ctypes.c_float, ctypes.c_float, ci, ci, vp, vp, sz,
                                 ctypes.POINTER(ctypes.c_int32), vp]
    lib.spmspv_last_error.argtypes = []
    lib.spmspv_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        lib = load_library()
        msg = lib.spmspv_status_string(rc).decode() + ": " + lib.spmspv_last_error().decode()
        raise SpmspvError(rc, msg)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------- C-ABI mirrors
def spmspv_workspace_size(m: int, n: int, nnz: int, flags: int = 0) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().spmspv_workspace_size(m, n, nnz, flags, ctypes.byref(out)))
    return out.value


def spmspv_create(m, n, nnz, colptr, rowids, values, workspace, ws_bytes, flags=0, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p(None)
    _check(load_library().spmspv_create(ctypes.byref(h), m, n, nnz, _ptr(colptr), _ptr(rowids), _ptr(values),
                                        _ptr(workspace), ws_bytes, flags, _stream(stream)))
    return h


def spmspv_dcsc_workspace_size(m: int, n: int, nzc: int, nnz: int, flags: int = 0) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().spmspv_dcsc_workspace_size(m, n, nzc, nnz, flags, ctypes.byref(out)))
    return out.value


def spmspv_create_dcsc(m, n, nzc, nnz, jc, cp, rowids, values, workspace, ws_bytes, flags=0,
                       stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p(None)
    _check(load_library().spmspv_create_dcsc(ctypes.byref(h), m, n, nzc, nnz, _ptr(jc), _ptr(cp), _ptr(rowids),
                                             _ptr(values), _ptr(workspace), ws_bytes, flags, _stream(stream)))
    return h


def spmspv_run_bitvector(handle, semiring, flags, x_bits, x_val, y_bits, y_val, y_capacity, d_nnz_y=None,
                         sync=True, stream=None) -> Optional[int]:
    """Bitvector x -> bitvector y (bitmaps as int32/uint32 words); with sync=True returns nnz(y)."""
    h = ctypes.c_int64(0)
    _check(load_library().spmspv_run_bitvector(handle, semiring, flags, _ptr(x_bits), _ptr(x_val), _ptr(y_bits),
                                               _ptr(y_val), y_capacity, _ptr(d_nnz_y),
                                               ctypes.byref(h) if sync else None, _stream(stream)))
    return h.value if sync else None


def spmspv_run(handle, semiring, flags, f, x_idx, x_val, y_idx, y_val, y_capacity, d_nnz_y=None, sync=True,
               stream=None) -> Optional[int]:
    """Enqueue y <- A x; with sync=True waits and returns nnz(y)."""
    h = ctypes.c_int64(0)
    _check(load_library().spmspv_run(handle, semiring, flags, f, _ptr(x_idx), _ptr(x_val), _ptr(y_idx),
                                     _ptr(y_val), y_capacity, _ptr(d_nnz_y), ctypes.byref(h) if sync else None,
                                     _stream(stream)))
    return h.value if sync else None


def spmspv_run_masked(handle, semiring, flags, f, x_idx, x_val, mask, y_idx, y_val, y_capacity, d_nnz_y=None,
                      sync=True, stream=None) -> Optional[int]:
    """y <- A x with rows whose mask bit is set excluded (mask: int32/uint32 words)."""
    h = ctypes.c_int64(0)
    _check(load_library().spmspv_run_masked(handle, semiring, flags, f, _ptr(x_idx), _ptr(x_val), _ptr(mask),
                                            _ptr(y_idx), _ptr(y_val), y_capacity, _ptr(d_nnz_y),
                                            ctypes.byref(h) if sync else None, _stream(stream)))
    return h.value if sync else None


def spmspv_run_static(m, n, nnz, colptr, rowids, values, semiring, flags, f, x_idx, x_val, y_idx, y_val,
                      y_capacity, d_nnz_y=None, sync=True, stream=None) -> Optional[int]:
    """Allocation-free y <- A x (no handle, no workspace: the library's own
    device scratch).  Returns nnz(y) when sync."""
    h = ctypes.c_int64(0)
    _check(load_library().spmspv_run_static(m, n, nnz, _ptr(colptr), _ptr(rowids), _ptr(values), semiring, flags,
                                            f, _ptr(x_idx), _ptr(x_val), _ptr(y_idx), _ptr(y_val), y_capacity,
                                            _ptr(d_nnz_y), ctypes.byref(h) if sync else None, None,
                                            _stream(stream)))
    return h.value if sync else None


def cc_run(handle, labels, flags=0, stream=None) -> int:
    """Connected components into `labels` (int32 [n] device); returns the multiplies run."""
    it = ctypes.c_int32(0)
    _check(load_library().cc_run(handle, flags, _ptr(labels), ctypes.byref(it), _stream(stream)))
    return it.value


MASK_COMPLEMENT, MASK_REPLACE = 1, 2
ACCUM_NONE, ACCUM_ADD, ACCUM_FIRST, ACCUM_SECOND = 0, 1, 2, 3


def spmspv_run_graphblas(handle, semiring, flags, f, x_idx, x_val, mask_idx, mask_val, mask_count, mask_flags,
                         accum, w_idx, w_val, w_count, y_idx, y_val, y_capacity, d_nnz_y=None, sync=True,
                         stream=None) -> Optional[int]:
    """w<mask, replace> = w accum (A x); returns nnz(y) when sync."""
    h = ctypes.c_int64(0)
    _check(load_library().spmspv_run_graphblas(handle, semiring, flags, f, _ptr(x_idx), _ptr(x_val),
                                               _ptr(mask_idx), _ptr(mask_val), mask_count, mask_flags, accum,
                                               _ptr(w_idx), _ptr(w_val), w_count, _ptr(y_idx), _ptr(y_val),
                                               y_capacity, _ptr(d_nnz_y), ctypes.byref(h) if sync else None,
                                               _stream(stream)))
    return h.value if sync else None


def spmspv_static_scratch_need(m, n, nnz) -> int:
    """Scratch bytes spmspv_run_static needs for an m x n matrix with nnz entries."""
    return spmspv_workspace_size(m, n, nnz, 0)


def spmspv_selector_load(handle, params, mean, std, stream=None):
    """params / mean / std: host float32 numpy arrays (5258, 6, 6)."""
    import numpy as np
    p = np.ascontiguousarray(params, np.float32)
    mu = np.ascontiguousarray(mean, np.float32)
    sd = np.ascontiguousarray(std, np.float32)
    if p.size != MLP_PARAMS or mu.size != 6 or sd.size != 6:
        raise ValueError("selector weights must be 5258 + 6 + 6 floats")
    _check(load_library().spmspv_selector_load(handle, p.ctypes.data, mu.ctypes.data, sd.ctypes.data,
                                               _stream(stream)))


def spmspv_selector_classes(handle) -> list:
    cnt = ctypes.c_int32(0)
    _check(load_library().spmspv_selector_classes(handle, None, 0, ctypes.byref(cnt)))
    buf = (ctypes.c_int32 * max(cnt.value, 1))()
    _check(load_library().spmspv_selector_classes(handle, buf, cnt.value, ctypes.byref(cnt)))
    return list(buf[:cnt.value])


def spmspv_selector_features(handle, stream=None) -> list:
    out = (ctypes.c_float * 6)()
    _check(load_library().spmspv_selector_features(handle, out, _stream(stream)))
    return list(out)


def spmspv_force_classes(handle, classes=()):
    arr = (ctypes.c_int32 * max(len(classes), 1))(*[int(c) for c in classes])
    _check(load_library().spmspv_force_classes(handle, arr, len(classes)))


def spmspv_tuning_save(handle, path: str, stream=None):
    _check(load_library().spmspv_tuning_save(handle, os.fsencode(path), _stream(stream)))


def spmspv_tuning_load(handle, path: str, stream=None):
    _check(load_library().spmspv_tuning_load(handle, os.fsencode(path), _stream(stream)))


def spmspv_source_digest() -> str:
    return load_library().spmspv_source_digest().decode()


def spmspv_class_schedule(handle, semiring: int, cls: int) -> Schedule:
    out = Schedule()
    _check(load_library().spmspv_class_schedule(handle, int(semiring), int(cls), ctypes.byref(out)))
    return out


def spmspv_class_tile(handle, cls: int) -> int:
    t = ctypes.c_int32(0)
    _check(load_library().spmspv_class_tile(handle, int(cls), ctypes.byref(t)))
    return t.value


def spmspv_mlp_param_count() -> int:
    return int(load_library().spmspv_mlp_param_count())


def spmspv_mlp_forward(params, X, logits, stream=None):
    """logits[B][10] <- MLP(params, X[B][6]); device float32 tensors."""
    _check(load_library().spmspv_mlp_forward(_ptr(params), _ptr(X), int(X.shape[0]), _ptr(logits),
                                             _stream(stream)))


def spmspv_mlp_train_step(params, adam_m, adam_v, step, lr, X, labels, grad=None, loss=None, stream=None):
    _check(load_library().spmspv_mlp_train_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), int(step), float(lr),
                                                _ptr(X), _ptr(labels), int(X.shape[0]), _ptr(grad), _ptr(loss),
                                                _stream(stream)))


def spmspv_batch_workspace_size(handle, max_batch, max_f=0, max_products=0, flags=0) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().spmspv_batch_workspace_size(handle, int(max_batch), int(max_f), int(max_products),
                                                      int(flags), ctypes.byref(out)))
    return out.value


def spmspv_batch_attach(handle, max_batch, max_f, max_products, flags, workspace, ws_bytes, stream=None):
    _check(load_library().spmspv_batch_attach(handle, int(max_batch), int(max_f), int(max_products), int(flags),
                                              _ptr(workspace), int(ws_bytes), _stream(stream)))


def spmspv_run_batch(handle, semiring, flags, nbatch, x_off, x_idx, x_val, y_off, y_idx, y_val, y_capacity,
                     sync=True, stream=None) -> Optional[int]:
    """Batched y_b <- A x_b; with sync=True waits and returns the total nnz."""
    h = ctypes.c_int64(0)
    _check(load_library().spmspv_run_batch(handle, semiring, flags, int(nbatch), _ptr(x_off), _ptr(x_idx),
                                           _ptr(x_val), _ptr(y_off), _ptr(y_idx), _ptr(y_val), int(y_capacity),
                                           ctypes.byref(h) if sync else None, _stream(stream)))
    return h.value if sync else None


def spmspv_set_batch_schedule(handle, sched: Optional[Schedule] = None):
    _check(load_library().spmspv_set_batch_schedule(handle, ctypes.byref(sched) if sched is not None else None))


def spmspv_get_batch_schedule(handle, nbatch, semiring=0) -> Schedule:
    sc = Schedule()
    _check(load_library().spmspv_get_batch_schedule(handle, int(semiring), int(nbatch), ctypes.byref(sc)))
    return sc


def msbfs_run(handle, semiring, roots, flags, level, parent=None, stream=None) -> int:
    import numpy as np
    r = np.ascontiguousarray(roots, np.int32)
    nl = ctypes.c_int32(0)
    _check(load_library().msbfs_run(handle, semiring, int(r.size), r.ctypes.data, flags, _ptr(level), _ptr(parent),
                                    ctypes.byref(nl), _stream(stream)))
    return nl.value


def spmspv_autotune(handle, semiring, densities, reps, x_idx, x_val, y_idx, y_val, stream=None) -> list:
    d = (ctypes.c_double * len(densities))(*[float(v) for v in densities])
    out = (TuneEntry * len(densities))()
    _check(load_library().spmspv_autotune(handle, semiring, d, len(densities), int(reps), _ptr(x_idx), _ptr(x_val),
                                          _ptr(y_idx), _ptr(y_val), out, _stream(stream)))
    return [e.as_dict() for e in out]


def spmspv_effective_schedule(handle, f, flags=0, semiring=0) -> Schedule:
    sc = Schedule()
    _check(load_library().spmspv_effective_schedule(handle, int(semiring), int(f), int(flags), ctypes.byref(sc)))
    return sc


def spmspv_tuned_schedule(handle, f) -> Schedule:
    sc = Schedule()
    _check(load_library().spmspv_tuned_schedule(handle, int(f), ctypes.byref(sc)))
    return sc


def spmspv_autotune_batch(handle, semiring, flags, nbatch, x_off, x_idx, x_val, y_off, y_idx, y_val, y_capacity,
                          reps=5, stream=None):
    sc = Schedule()
    us = ctypes.c_double(0)
    _check(load_library().spmspv_autotune_batch(handle, semiring, flags, int(nbatch), _ptr(x_off), _ptr(x_idx),
                                                _ptr(x_val), _ptr(y_off), _ptr(y_idx), _ptr(y_val), int(y_capacity),
                                                int(reps), ctypes.byref(sc), ctypes.byref(us), _stream(stream)))
    return sc, us.value


def pagerank_scratch_size(handle) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().pagerank_scratch_size(handle, ctypes.byref(out)))
    return out.value


def pagerank_run(handle, damping, tol, max_iter, flags, rank, scratch, scratch_bytes, stream=None) -> int:
    it = ctypes.c_int32(0)
    _check(load_library().pagerank_run(handle, float(damping), float(tol), int(max_iter), int(flags), _ptr(rank),
                                       _ptr(scratch), int(scratch_bytes), ctypes.byref(it), _stream(stream)))
    return it.value


def bfs_run(handle, semiring, root, flags, level, parent=None, stream=None) -> int:
    nl = ctypes.c_int32(0)
    _check(load_library().bfs_run(handle, semiring, int(root), flags, _ptr(level), _ptr(parent), ctypes.byref(nl),
                                  _stream(stream)))
    return nl.value


def spmspv_get_schedule(handle) -> Schedule:
    s = Schedule()
    _check(load_library().spmspv_get_schedule(handle, ctypes.byref(s)))
    return s


def spmspv_set_schedule(handle, sched: Optional[Schedule] = None):
    _check(load_library().spmspv_set_schedule(handle, ctypes.byref(sched) if sched is not None else None))


def spmspv_last_stats(handle, stream=None) -> dict:
    out = (ctypes.c_int64 * 6)()
    _check(load_library().spmspv_last_stats(handle, out, _stream(stream)))
    return {"W": out[0], "nnz_y": out[1], "fnz": out[2], "maxlen": out[3], "err": out[4], "cls": out[5]}


def spmspv_profile_read(handle) -> Tuple[list, int]:
    ms = (ctypes.c_double * 3)()
    calls = ctypes.c_int64(0)
    _check(load_library().spmspv_profile_read(handle, ms, ctypes.byref(calls)))
    return [ms[0], ms[1], ms[2]], calls.value


def spmspv_destroy(handle):
    _check(load_library().spmspv_destroy(handle))


# ------------------------------------------------------------ convenience
# Handles still open when the interpreter exits are released by an exit
# handler, which runs while the HIP runtime is fully up (before the C-level
# exit handlers and library destructors that tear it down), after the
# device has finished its work; a handle's own __del__ may otherwise run at
# an arbitrary point of interpreter shutdown.
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    if not _live:
        return
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except Exception:
        pass
    for M in list(_live):
        try:
            M.close()
        except Exception:
            pass


class Matrix:
    """A CSC matrix resident on the GPU with its library handle and workspace.

    Holds torch tensors for colptr / rowids / values / workspace (the library
    borrows them) and exposes spmspv() and bfs().
    """

    def __init__(self, m: int, n: int, colptr, rowids, values=None, flags: int = 0, device="cuda"):
        import torch
        self.m, self.n = int(m), int(n)
        self.colptr = torch.as_tensor(colptr, dtype=torch.int32).to(device).contiguous()
        self.rowids = torch.as_tensor(rowids, dtype=torch.int32).to(device).contiguous()
        self.values = None if values is None else torch.as_tensor(values, dtype=torch.float32).to(device).contiguous()
        self.nnz = int(self.rowids.numel())
        self.ws_bytes = spmspv_workspace_size(self.m, self.n, self.nnz, flags)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.handle = spmspv_create(self.m, self.n, self.nnz, self.colptr, self.rowids, self.values, self.workspace,
                                    self.ws_bytes, flags)
        _live.add(self)
        self._d_nnz = torch.zeros(1, dtype=torch.int64, device=device)

    @classmethod
    def from_csc(cls, A, flags: int = 0, device="cuda", pattern: bool = False):
        return cls(A.m, A.n, A.colptr, A.rowids, None if pattern else A.values, flags, device)

    @classmethod
    def from_dcsc(cls, D, flags: int = 0, device="cuda", pattern: bool = False):
        """A DCSC matrix (non-empty columns only: ids D.jc, starts D.cp)."""
        import torch
        self = cls.__new__(cls)
        self.m, self.n = int(D.m), int(D.n)
        self.jc = torch.as_tensor(D.jc, dtype=torch.int32).to(device).contiguous()
        self.colptr = torch.as_tensor(D.cp, dtype=torch.int32).to(device).contiguous()
        self.rowids = torch.as_tensor(D.rowids, dtype=torch.int32).to(device).contiguous()
        vals = None if (pattern or D.values is None) else D.values
        self.values = None if vals is None else torch.as_tensor(vals, dtype=torch.float32).to(device).contiguous()
        self.nnz = int(self.rowids.numel())
        self.nzc = int(self.jc.numel())
        self.ws_bytes = spmspv_dcsc_workspace_size(self.m, self.n, self.nzc, self.nnz, flags)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.handle = spmspv_create_dcsc(self.m, self.n, self.nzc, self.nnz, self.jc, self.colptr, self.rowids,
                                         self.values, self.workspace, self.ws_bytes, flags)
        _live.add(self)
        self._d_nnz = torch.zeros(1, dtype=torch.int64, device=device)
        return self

    def close(self):
        if getattr(self, "handle", None) is not None:
            spmspv_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def schedule(self) -> Schedule:
        return spmspv_get_schedule(self.handle)

    @schedule.setter
    def schedule(self, s: Optional[Schedule]):
        spmspv_set_schedule(self.handle, s)

    def spmspv(self, x_idx, x_val=None, semiring: int = PLUS_TIMES_F32, sorted_output: bool = False,
               flags: int = 0, y_capacity: Optional[int] = None, out=None, sync: bool = True, mask=None):
        """y <- A x (rows with a set `mask` bit excluded).  Returns (y_idx, y_val, nnz), trimmed when sync."""
        import torch
        dev = self.colptr.device
        cap = (self.n if flags & LEFT else self.m) if y_capacity is None else int(y_capacity)
        if out is None:
            y_idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            vdt = {PLUS_TIMES_F32: torch.float32, MIN_SELECT2ND_I32: torch.int32, OR_AND_BOOL: torch.uint8}[semiring]
            y_val = torch.empty(max(cap, 1), dtype=vdt, device=dev)
        else:
            y_idx, y_val = out
        fl = flags | (SORTED_OUTPUT if sorted_output else 0)
        f = int(x_idx.numel())
        nnz = spmspv_run_masked(self.handle, semiring, fl, f, x_idx, x_val, mask, y_idx, y_val, cap, self._d_nnz,
                                sync=sync)
        if not sync:
            return y_idx, y_val, self._d_nnz
        k = min(nnz, cap)
        return y_idx[:k], y_val[:k], nnz

    def spmspv_bitvector(self, x_bits, x_val=None, semiring: int = PLUS_TIMES_F32, flags: int = 0,
                         y_capacity: Optional[int] = None):
        """Bitvector x (uint32-word bitmap + values ascending by index) -> (y_bits, y_val, nnz)."""
        import torch
        dev = self.colptr.device
        ylen = self.n if flags & LEFT else self.m
        cap = ylen if y_capacity is None else int(y_capacity)
        y_bits = torch.empty(max((ylen + 31) // 32, 1), dtype=torch.int32, device=dev)
        vdt = {PLUS_TIMES_F32: torch.float32, MIN_SELECT2ND_I32: torch.int32, OR_AND_BOOL: torch.uint8}[semiring]
        y_val = torch.empty(max(cap, 1), dtype=vdt, device=dev)
        nnz = spmspv_run_bitvector(self.handle, semiring, flags, x_bits, x_val, y_bits, y_val, cap, self._d_nnz)
        return y_bits, y_val[:min(nnz, cap)], nnz

    def bfs(self, root: int, semiring: int = MIN_SELECT2ND_I32, parents: bool = True, flags: int = 0):
        import torch
        dev = self.colptr.device
        level = torch.empty(self.n, dtype=torch.int32, device=dev)
        parent = torch.empty(self.n, dtype=torch.int32, device=dev) if (parents and semiring == MIN_SELECT2ND_I32) \
            else None
        nl = bfs_run(self.handle, semiring, root, flags, level, parent)
        return level, parent, nl

    def last_stats(self) -> dict:
        return spmspv_last_stats(self.handle)

    def attach_batch(self, max_batch: int, max_f: int = 0, max_products: int = 0, msbfs: bool = False):
        """Allocate and bind the batch workspace (torch uint8 tensor held here)."""
        import torch
        fl = MSBFS if msbfs else 0
        nbytes = spmspv_batch_workspace_size(self.handle, max_batch, max_f, max_products, fl)
        self.batch_ws = torch.empty(nbytes, dtype=torch.uint8, device=self.colptr.device)
        spmspv_batch_attach(self.handle, max_batch, max_f, max_products, fl, self.batch_ws, nbytes)
        return nbytes

    def spmspv_batch(self, x_off, x_idx, x_val=None, semiring: int = PLUS_TIMES_F32, flags: int = 0,
                     y_capacity: Optional[int] = None, out=None, sync: bool = True):
        """Batched multiply; x_off int64 [B+1], x_idx / x_val concatenated (device tensors).
        Returns (y_off, y_idx, y_val, total)."""
        import torch
        dev = self.colptr.device
        nb = int(x_off.numel()) - 1
        cap = int(y_capacity) if y_capacity is not None else nb * self.m
        if out is None:
            vdt = {PLUS_TIMES_F32: torch.float32, MIN_SELECT2ND_I32: torch.int32, OR_AND_BOOL: torch.uint8}[semiring]
            y_off = torch.empty(nb + 1, dtype=torch.int64, device=dev)
            y_idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            y_val = torch.empty(max(cap, 1), dtype=vdt, device=dev)
        else:
            y_off, y_idx, y_val = out
        total = spmspv_run_batch(self.handle, semiring, flags, nb, x_off, x_idx, x_val, y_off, y_idx, y_val, cap,
                                 sync=sync)
        return y_off, y_idx, y_val, total

    def msbfs(self, roots, semiring: int = MIN_SELECT2ND_I32, parents: bool = True, flags: int = 0):
        import torch
        dev = self.colptr.device
        k = len(roots)
        level = torch.empty((k, self.n), dtype=torch.int32, device=dev)
        parent = torch.empty((k, self.n), dtype=torch.int32, device=dev) \
            if (parents and semiring == MIN_SELECT2ND_I32) else None
        nl = msbfs_run(self.handle, semiring, roots, flags, level, parent)
        return level, parent, nl

    def autotune(self, semiring: int = PLUS_TIMES_F32, densities=(1e-4, 1e-3, 1e-2, 1e-1), reps: int = 8):
        """Run the autotuner (device scratch allocated here); returns the per-band table."""
        import torch
        dev = self.colptr.device
        xi = torch.empty(max(self.n, 1), dtype=torch.int32, device=dev)
        xv = torch.empty(max(self.n, 1), dtype=torch.float32, device=dev) if semiring == PLUS_TIMES_F32 else None
        yi = torch.empty(max(self.m, 1), dtype=torch.int32, device=dev)
        yv = torch.empty(max(self.m, 1), dtype=torch.int32, device=dev)
        return spmspv_autotune(self.handle, semiring, densities, reps, xi, xv, yi, yv)

    def save_tuning(self, path: str):
        spmspv_tuning_save(self.handle, path)

    def load_tuning(self, path: str):
        spmspv_tuning_load(self.handle, path)

    def pagerank(self, damping: float = 0.85, tol: float = 1e-6, max_iter: int = 100, flags: int = 0):
        """Data-driven PageRank on a pattern handle; returns (rank float32 tensor, multiplies)."""
        import torch
        dev = self.colptr.device
        nbytes = pagerank_scratch_size(self.handle)
        if getattr(self, "_pr_scratch", None) is None or self._pr_scratch.numel() < nbytes:
            self._pr_scratch = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        rank = torch.empty(self.n, dtype=torch.float32, device=dev)
        it = pagerank_run(self.handle, damping, tol, max_iter, flags, rank, self._pr_scratch, nbytes)
        return rank, it

    def connected_components(self):
        """labels[v] = the smallest vertex reaching v (the component's smallest
        vertex for a symmetric matrix); returns (labels, multiplies)."""
        import torch
        labels = torch.empty(self.n, dtype=torch.int32, device=self.colptr.device)
        it = cc_run(self.handle, labels)
        return labels, it

    def load_selector(self, params, mean, std):
        spmspv_selector_load(self.handle, params, mean, std)

    def selector_classes(self) -> list:
        return spmspv_selector_classes(self.handle)

    def class_tile(self, cls: int) -> int:
        return spmspv_class_tile(self.handle, cls)
