"""CPU oracle for the SpGEMM hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark
may import this package. It shares no code with the HIP library under
``paper_1804_00695_amd/`` and never imports it.

``oracle.c`` (plain C, fp64, compiled with -ffp-contract=off) holds the
products; ``plan.py`` holds the chunking heuristic; the small helpers here
(compression, row work) are written directly from their definitions.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from synth import Csr

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no GPU code)."""
    import subprocess
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class using_library:
    """Context manager: run the oracle functions against another build of
    oracle.c (used by the tests that plant mistakes in a copy of it)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib, _LIB_PATH
        self._saved = (_lib, _LIB_PATH)
        _lib, _LIB_PATH = None, self.path
        return self

    def __exit__(self, *exc):
        global _lib, _LIB_PATH
        _lib, _LIB_PATH = self._saved
        return False


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        _lib.oracle_csr_check.argtypes = [i32, i32, P, P]
        _lib.oracle_csr_check.restype = ctypes.c_int
        _lib.oracle_spgemm_count.argtypes = [i32, P, P, i32, P, P, P, i32, P, ctypes.c_int]
        _lib.oracle_spgemm_count.restype = i64
        _lib.oracle_spgemm_fill.argtypes = [i32, P, P, P, i32, P, P, P, P, i32, P, P, P, P, ctypes.c_int]
        _lib.oracle_spgemm_fill.restype = None
        _lib.oracle_tc_lower.argtypes = [i32, P, P, P, P, P]
        _lib.oracle_tc_lower.restype = i64
        _lib.oracle_tc_count.argtypes = [i32, P, P, P, i32, P, ctypes.c_int]
        _lib.oracle_tc_count.restype = i64
        _lib.oracle_spgemm_backward.argtypes = [i32, P, P, P, i32, i32, P, P, P, P, P, P, P, P, P, P]
        _lib.oracle_spgemm_backward.restype = ctypes.c_int
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def csr_check(M: Csr) -> int:
    """0 if M is valid CSR with strictly increasing in-range columns."""
    return _load().oracle_csr_check(M.nrows, M.ncols, _p(_i32(M.row_ptr)), _p(_i32(M.col_idx)))


def _rows_arg(m, rows):
    if rows is None:
        return None, m
    r = _i32(rows)
    if r.size and (r.min() < 0 or r.max() >= m):
        raise ValueError("row index out of range")
    return r, int(r.size)


def spgemm_count(A: Csr, B: Csr, rows=None, nthreads: int = 1) -> np.ndarray:
    """Symbolic phase: int64 prefix of the distinct-column counts of the selected rows of A*B."""
    if A.ncols != B.nrows:
        raise ValueError("dimension mismatch")
    r, nr = _rows_arg(A.nrows, rows)
    crp = np.zeros(nr + 1, dtype=np.int64)
    arp, aci, brp, bci = _i32(A.row_ptr), _i32(A.col_idx), _i32(B.row_ptr), _i32(B.col_idx)
    _load().oracle_spgemm_count(A.nrows, _p(arp), _p(aci), B.ncols, _p(brp), _p(bci),
                                _p(r), nr, _p(crp), nthreads)
    return crp


def spgemm(A: Csr, B: Csr, rows=None, nthreads: int = 1, with_abs: bool = True):
    """C = A*B (selected rows). Returns (C, cabs) where cabs[e] = sum |a||b| over
    the terms of entry e (None for pattern-only inputs or with_abs=False).

    For a row subset, C has one row per selected row, in the given order.
    """
    crp = spgemm_count(A, B, rows, nthreads)
    r, nr = _rows_arg(A.nrows, rows)
    nnz = int(crp[-1])
    if nnz >= 2**31:
        raise ValueError("nnz(C) does not fit int32 indices")
    cci = np.empty(nnz, dtype=np.int32)
    vals = A.values is not None and B.values is not None
    cval = np.empty(nnz) if vals else None
    cabs = np.empty(nnz) if (vals and with_abs) else None
    arp, aci, brp, bci = _i32(A.row_ptr), _i32(A.col_idx), _i32(B.row_ptr), _i32(B.col_idx)
    av, bv = (_f64(A.values), _f64(B.values)) if vals else (None, None)
    _load().oracle_spgemm_fill(A.nrows, _p(arp), _p(aci), _p(av), B.ncols, _p(brp), _p(bci), _p(bv),
                               _p(r), nr, _p(crp), _p(cci), _p(cval), _p(cabs), nthreads)
    C = Csr(nr, B.ncols, crp.astype(np.int32), cci, cval)
    return C, cabs


def tc_lower(G: Csr):
    """(perm, L): perm[new] = old vertex id; L = strict lower triangle after the
    descending-degree relabelling (ties by ascending id)."""
    nv = G.nrows
    perm = np.empty(nv, dtype=np.int32)
    lrp = np.empty(nv + 1, dtype=np.int32)
    lci = np.empty(G.nnz // 2 + 1, dtype=np.int32)
    nnz = _load().oracle_tc_lower(nv, _p(_i32(G.row_ptr)), _p(_i32(G.col_idx)), _p(perm), _p(lrp), _p(lci))
    return perm, Csr(nv, nv, lrp, lci[:nnz].copy(), None)


def tc_count(L: Csr, rows=None, nthreads: int = 1):
    """(counts int64 per selected row, total) for the masked product (L*L) o L."""
    r, nr = _rows_arg(L.nrows, rows)
    counts = np.zeros(nr, dtype=np.int64)
    total = _load().oracle_tc_count(L.nrows, _p(_i32(L.row_ptr)), _p(_i32(L.col_idx)), _p(r), nr,
                                    _p(counts), nthreads)
    return counts, int(total)


def triangle_count(G: Csr, nthreads: int = 1):
    perm, L = tc_lower(G)
    counts, total = tc_count(L, nthreads=nthreads)
    return total, counts, perm, L


def backward(A: Csr, B: Csr, W: Csr):
    """(dA, dB, dA_abs, dB_abs) for loss = sum_ij W_ij (A*B)_ij, W on pat(A*B)."""
    dA = np.empty(A.nnz)
    dB = np.empty(B.nnz)
    dAa = np.empty(A.nnz)
    dBa = np.empty(B.nnz)
    arp, aci, brp, bci = _i32(A.row_ptr), _i32(A.col_idx), _i32(B.row_ptr), _i32(B.col_idx)
    wrp, wci = _i32(W.row_ptr), _i32(W.col_idx)
    av, bv, wv = _f64(A.values), _f64(B.values), _f64(W.values)
    err = _load().oracle_spgemm_backward(A.nrows, _p(arp), _p(aci), _p(av), B.nrows, B.ncols,
                                         _p(brp), _p(bci), _p(bv), _p(wrp), _p(wci), _p(wv),
                                         _p(dA), _p(dB), _p(dAa), _p(dBa))
    if err:
        raise ValueError("W does not cover the pattern of A*B")
    return dA, dB, dAa, dBa


def compress(B: Csr, rows=None):
    """Compressed rows of B's pattern: 32 columns per word, (set, mask) pairs.

    The paper encodes several columns of a row of B in fewer integers so that
    unions become bitwise ORs (Sec. 2.1) but does not fix the encoding. Here
    column j lives in set j >> 5 at bit j & 31; each row lists its distinct
    sets in ascending order with the OR of the bits of its columns.
    ``rows`` selects a subset of rows (default all), in the given order.
    Returns (comp_row_ptr int32, set int32, mask uint32).
    """
    sel = range(B.nrows) if rows is None else [int(r) for r in rows]
    sets_all, masks_all, counts = [], [], []
    for i in sel:
        cols, _ = B.row(i)
        words = {}
        for j in cols.tolist():
            s = j >> 5
            words[s] = words.get(s, 0) | (1 << (j & 31))
        keys = sorted(words)
        counts.append(len(keys))
        sets_all.extend(keys)
        masks_all.extend(words[k] for k in keys)
    rp = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(np.array(counts, dtype=np.int64), out=rp[1:])
    return rp.astype(np.int32), np.array(sets_all, dtype=np.int32), np.array(masks_all, dtype=np.uint32)


def row_work(A: Csr, B: Csr) -> np.ndarray:
    """Multiply-adds of each row of A*B: sum over k in row i of A of nnz(row k of B)."""
    blen = np.diff(B.row_ptr.astype(np.int64))
    arow = np.repeat(np.arange(A.nrows), np.diff(A.row_ptr.astype(np.int64)))
    w = np.zeros(A.nrows, dtype=np.int64)
    np.add.at(w, arow, blen[A.col_idx])
    return w
