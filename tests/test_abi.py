"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spmspv.h")


def _lib():
    import paper_1610_07902_amd as spv
    if not os.path.exists(spv.LIB_PATH):
        pytest.skip("libspmspv.so not built")
    return spv, spv.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|const char\*)\s+(\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("spmspv_create", "spmspv_run", "bfs_run", "spmspv_workspace_size", "spmspv_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    spv, lib = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", spv.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    assert set(spv.EXPORTED) <= exported


def test_workspace_size_host_only():
    spv, lib = _lib()
    b1 = spv.spmspv_workspace_size(1000, 1000, 5000)
    b2 = spv.spmspv_workspace_size(1000, 1000, 50000)
    assert b2 - b1 >= 8 * 45000          # buckets hold nnz (row, value) pairs
    with pytest.raises(spv.SpmspvError) as e:
        spv.spmspv_workspace_size(0, 10, 10)
    assert e.value.status == spv.EINVAL
    with pytest.raises(spv.SpmspvError):
        spv.spmspv_workspace_size(10, 10, 1 << 31)


def test_null_arguments_rejected_without_gpu():
    spv, lib = _lib()
    h = ctypes.c_void_p(None)
    rc = lib.spmspv_create(ctypes.byref(h), 10, 10, 5, None, None, None, None, 0, 0, None)
    assert rc == spv.EINVAL and h.value is None
    assert lib.spmspv_run(None, 0, 0, 0, None, None, None, None, 0, None, None, None) == spv.EINVAL
    assert lib.bfs_run(None, 1, 0, 0, None, None, None, None) == spv.EINVAL
    assert lib.spmspv_destroy(None) == spv.OK
    assert lib.spmspv_status_string(spv.ECAPACITY).decode() == "output capacity too small"
    assert lib.spmspv_last_error().decode() != ""


def test_static_multiply_refuses_oversized_matrix_without_gpu():
    """The allocation-free multiply checks its scratch limit on the host,
    before any device call: a matrix whose workspace exceeds the 64 MiB
    scratch is refused with EINVAL and the size it would need."""
    spv, lib = _lib()
    need = ctypes.c_size_t(0)
    m = n = 1 << 22
    rc = lib.spmspv_run_static(m, n, 20_000_000, None, None, None, 0, 0, 0, None, None, None, None, 0, None, None,
                               ctypes.byref(need), None)
    assert rc == spv.EINVAL
    assert need.value == spv.spmspv_workspace_size(m, n, 20_000_000, 0) > (64 << 20)
    assert "static scratch" in lib.spmspv_last_error().decode()


def test_format_variants_host_checks():
    """DCSC sizing and argument checks, and the bitvector / left calls'
    refusals, all before any device work."""
    spv, lib = _lib()
    csc = spv.spmspv_workspace_size(5000, 100000, 20000)
    dcsc = spv.spmspv_dcsc_workspace_size(5000, 100000, 3000, 20000)
    assert dcsc > csc                                  # plus the column index over jc
    for args in ((5000, 100000, 100001, 200000),       # nzc > n
                 (5000, 100000, 0, 10),                # no stored column but entries
                 (5000, 100000, 30, 20)):              # more columns than entries
        with pytest.raises(spv.SpmspvError) as e:
            spv.spmspv_dcsc_workspace_size(*args)
        assert e.value.status == spv.EINVAL
    with pytest.raises(spv.SpmspvError) as e:          # no transpose for a DCSC handle
        spv.spmspv_dcsc_workspace_size(50, 50, 10, 20, spv.WITH_TRANSPOSE)
    assert e.value.status == spv.EINVAL
    h = ctypes.c_void_p(None)
    rc = lib.spmspv_create_dcsc(ctypes.byref(h), 10, 10, 2, 5, None, None, None, None, None, 0, 0, None)
    assert rc == spv.EINVAL and h.value is None
    assert lib.spmspv_run_bitvector(None, 0, 0, None, None, None, None, 0, None, None, None) == spv.EINVAL
    # the transpose-sized regions grow the workspace of a wide matrix only with a transpose
    assert spv.spmspv_workspace_size(100, 200000, 1000, spv.WITH_TRANSPOSE) > \
        spv.spmspv_workspace_size(100, 200000, 1000) + 200000 * 4


def test_library_records_its_source_digest():
    spv, lib = _lib()
    from paper_1610_07902_amd import build
    assert spv.spmspv_source_digest() == build.source_digest(), "library built from other sources: rebuild"
