"""The C ABI library loads on a machine without a GPU, exports every symbol
that include/mlspgemm.h declares, and its host-only logic behaves (status
strings, options, host CSR validation, workspace sizing). No compute calls."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1804_00695_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mlspgemm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spgemm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_abi.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for each of them
    assert set(names) <= set(_abi.SIGNATURES), set(names) - set(_abi.SIGNATURES)


def test_status_strings_and_version():
    lib = _abi.load()
    assert lib.spgemm_status_string(0) == b"ok"
    assert b"CSR" in lib.spgemm_status_string(2)
    assert lib.spgemm_version() >= 10000


def test_options():
    lib = _abi.load()
    assert lib.spgemm_set_option(_abi.OPT_GROUP_SIZE, 12) == 1
    assert lib.spgemm_set_option(_abi.OPT_GROUP_SIZE, 16) == 0
    assert lib.spgemm_get_option(_abi.OPT_GROUP_SIZE) == 16
    assert lib.spgemm_set_option(_abi.OPT_GROUP_SIZE, 0) == 0
    assert lib.spgemm_get_option(_abi.OPT_VALIDATE) == 1


def host_handle(rp, ci, nrows, ncols):
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    h = _abi.CsrT(nrows, ncols, len(ci), rp.ctypes.data, ci.ctypes.data if len(ci) else None, None)
    return h, (rp, ci)


@pytest.mark.parametrize("case,expect", [
    (([0, 2, 3], [0, 2, 1], 2, 3), 0),
    (([1, 2, 3], [0, 2, 1], 2, 3), 2),      # row_ptr[0] != 0
    (([0, 2, 1], [0, 2], 2, 3), 2),         # decreasing
    (([0, 2, 3], [0, 3, 1], 2, 3), 2),      # column out of range
    (([0, 2, 3], [2, 0, 1], 2, 3), 2),      # unsorted
    (([0, 2, 3], [1, 1, 1], 2, 3), 2),      # duplicate
])
def test_validate_host(case, expect):
    lib = _abi.load()
    h, keep = host_handle(*case)
    assert lib.spgemm_validate_host(ctypes.byref(h)) == expect


def test_workspace_size_monotone():
    lib = _abi.load()
    sizes = []
    for n in (10, 1000, 100000):
        h = _abi.CsrT(n, n, 27 * n, None, None, None)
        out = ctypes.c_size_t(0)
        assert lib.spgemm_workspace_size(ctypes.byref(h), ctypes.byref(h), ctypes.byref(out)) == 0
        sizes.append(out.value)
    assert sizes[0] < sizes[1] < sizes[2]
    assert sizes[2] >= 27 * 100000 * 8        # compressed words of B
