"""The symbolic phase under an HBM budget (spgemm_symbolic_chunked): B's
compressed pattern resident, row parts of A streamed. Row pointers and
columns of C must equal the oracle's bit for bit at budgets from "everything
fits" down to many parts, on stencil, random, rectangular, empty-row and
power-law products (rows of C past the LDS classes). The host-side refusals
(a budget below B's compressed pattern, inconsistent row pointers) happen
before any HIP call and are checked without a GPU."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from paper_1804_00695_amd import _abi

BUDGET, BAD_CSR = 6, 2


def compressed_bytes(B):
    return 8 * B.nnz + 8 * B.nrows


def host_handle(M, keep):
    rp = np.ascontiguousarray(M.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(M.col_idx, dtype=np.int32)
    keep.append((rp, ci))
    return _abi.CsrT(M.nrows, M.ncols, int(rp[-1]), rp.ctypes.data, ci.ctypes.data if ci.size else None, None)


def test_refusals_before_any_hip_call():
    lib = _abi.load()
    A = synth.poisson_csr(300, 200, 5.0, 1)
    B = synth.poisson_csr(200, 250, 6.0, 2)
    keep = []
    ha, hb = host_handle(A, keep), host_handle(B, keep)
    crp = np.zeros(A.nrows + 1, dtype=np.int32)
    nnz = ctypes.c_int64(0)
    fake_ws = 1 << 20   # never dereferenced: the calls fail first
    # budget smaller than B's compressed pattern
    st = lib.spgemm_symbolic_chunked(ctypes.byref(ha), ctypes.byref(hb), crp.ctypes.data, None, ctypes.byref(nnz),
                                     fake_ws, compressed_bytes(B) // 2, None)
    assert st == BUDGET
    # decreasing row pointers of A
    bad = synth.Csr(A.nrows, A.ncols, A.row_ptr.copy(), A.col_idx, None)
    bad.row_ptr[3], bad.row_ptr[4] = bad.row_ptr[4], bad.row_ptr[3] - 1
    hbad = host_handle(bad, keep)
    st = lib.spgemm_symbolic_chunked(ctypes.byref(hbad), ctypes.byref(hb), crp.ctypes.data, None, ctypes.byref(nnz),
                                     fake_ws, 1 << 30, None)
    assert st == BAD_CSR


def cases():
    st = synth.stencil27_3d(14, amp=0.1)
    G = synth.rmat_graph(11, 8, seed=5)
    rm = synth.Csr(G.nrows, G.ncols, G.row_ptr, G.col_idx, None)
    empty = synth.random_csr(300, 200, 0.05, 3, empty_rows=0.5)
    empty_b = synth.random_csr(200, 150, 0.05, 4, empty_rows=0.5)
    return {
        "stencil": (st, st),
        "poisson_rect": (synth.poisson_csr(3000, 2000, 6.0, 41), synth.poisson_csr(2000, 4100, 8.0, 42)),
        "rmat_spill": (rm, rm),
        "empty_rows": (empty, empty_b),
    }


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["stencil", "poisson_rect", "rmat_spill", "empty_rows"])
@pytest.mark.parametrize("extra", [1 << 30, 4 << 20, 600_000, 150_000])
def test_matches_oracle_at_any_budget(name, extra):
    import paper_1804_00695_amd as mls
    A, B = cases()[name]
    print(f"symbolic_chunked {name} budget = compressed B + {extra}", flush=True)
    R, _ = oracle.spgemm(A, B)
    budget = compressed_bytes(B) + 4 * (B.nrows + 1) + 8192 + extra
    try:
        rp, ci = mls.symbolic_chunked(A, B, budget)
    except mls.SpgemmError as e:
        assert "BUDGET" in str(e)
        pytest.skip("budget below one row of A")
    assert np.array_equal(rp, R.row_ptr)
    assert np.array_equal(ci, R.col_idx)
