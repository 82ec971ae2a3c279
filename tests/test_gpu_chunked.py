"""GPU parity of the chunked numeric phase (pinned host A, B, C; HBM budget).

For budgets from "everything fits" down to dozens of parts, with single,
double, triple and quadruple buffering: C's values must equal the oracle's
bit for bit (and the in-HBM GPU result), and the bytes the executor queued
must equal the plan's schedule (which equals the oracle planner's, see
test_plan_parity). Alg. "chunkknl" (only B's parts are copied; the kernels
use A and C in place, in pinned host memory or in HBM) is held to the same
bar."""
import numpy as np
import pytest
import torch

import oracle
import oracle.plan as op
import synth

pytestmark = pytest.mark.gpu
mls = pytest.importorskip("paper_1804_00695_amd")


def run_chunked(A, B, R, budget, nbuf, min_parts):
    Ah, Bh = mls.HostCsr.from_host(A), mls.HostCsr.from_host(B)
    C = synth.Csr(R.nrows, R.ncols, R.row_ptr, R.col_idx, np.full(R.nnz, np.nan))
    Ch = mls.HostCsr.from_host(C)
    plan = mls.chunked_plan(A.row_ptr, B.row_ptr, B.ncols, R.row_ptr, budget, nbuf=nbuf, min_parts=min_parts)
    mls.numeric_chunked(Ah, Bh, Ch, plan)
    torch.cuda.synchronize()
    return Ch.values.numpy().copy(), plan


CASES = [
    ("stencil", 12, 4.0), ("stencil", 12, 0.5), ("stencil", 12, 0.15), ("stencil", 12, 0.05),
    ("poisson", 0, 3.0), ("poisson", 0, 0.3), ("poisson", 0, 0.08),
    ("rmat", 12, 0.3),   # rows of C past the LDS classes: spill windows on B's row parts
    ("wide", 0, 0.2),    # B has more rows than A (the shape of R x A)
]


def case_inputs(kind, n):
    if kind == "stencil":
        A = synth.stencil27_3d(n, amp=0.1)
        B = A
    elif kind == "rmat":
        G = synth.rmat_graph(n, 8, seed=5)
        A = synth.Csr(G.nrows, G.ncols, G.row_ptr, G.col_idx, synth.normal_values(len(G.col_idx), 8))
        B = A
    elif kind == "wide":
        A = synth.poisson_csr(600, 5000, 12.0, 43)
        B = synth.poisson_csr(5000, 900, 6.0, 44)
    else:
        A = synth.poisson_csr(3000, 2500, 6.0, 41)
        B = synth.poisson_csr(2500, 2800, 9.0, 42)
    return A, B


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("nbuf,min_parts", [(1, 1), (2, 1), (2, 4), (3, 1), (4, 5)])
def test_chunked_bitwise(case, nbuf, min_parts):
    kind, n, frac = case
    print(f"chunked {case} nbuf={nbuf} min_parts={min_parts}", flush=True)
    A, B = case_inputs(kind, n)
    R, cabs = oracle.spgemm(A, B)
    total = op.range_bytes(A.row_ptr, 0, A.nrows) + op.range_bytes(B.row_ptr, 0, B.nrows) + \
        op.range_bytes(R.row_ptr, 0, R.nrows)
    budget = plan_base(A, B, R) + int(total * frac)
    try:
        vals, plan = run_chunked(A, B, R, budget, nbuf, min_parts)
    except mls.SpgemmError as e:
        assert "BUDGET" in str(e)
        pytest.skip("budget below a single row")
    assert np.array_equal(vals, R.values)
    info = plan.info
    assert info["issued_h2d"] == info["h2d_bytes"] and info["issued_d2h"] == info["d2h_bytes"]
    assert info["ws_bytes"] <= budget


def test_chunked_matches_in_hbm_gpu():
    A = synth.stencil27_3d(14, amp=0.1, seed=5)
    dA = mls.DeviceCsr.from_host(A)
    C = mls.spgemm(dA, dA)
    torch.cuda.synchronize()
    rp, ci, v = C.numpy()
    R = synth.Csr(A.nrows, A.ncols, rp, ci, v)
    vals, plan = run_chunked(A, A, R, 3_000_000 + plan_base(A, A, R), 2, 3)
    assert plan.info["n_ac_parts"] * plan.info["n_b_parts"] > 2
    assert np.array_equal(vals, v)


def plan_base(A, B, R):
    """Workspace the plan reserves beside the part buffers (budget-independent)."""
    p = mls.chunked_plan(A.row_ptr, B.row_ptr, B.ncols, R.row_ptr, 10**10)
    return p.info["ws_bytes"] - p.info["chunk_bytes"]


def test_chunked_after_unsynchronised_product_on_same_workspace():
    # the chunked call's copy streams must wait for the work still queued on
    # the compute stream that uses the same workspace
    A = synth.stencil27_3d(16, amp=0.1, seed=6)
    ws = mls.Workspace()
    dA = mls.DeviceCsr.from_host(A)
    R, _ = oracle.spgemm(A, A)
    for _ in range(2):
        C = mls.spgemm(dA, dA, ws)   # numeric phase still running when the next call starts
        Ah = mls.HostCsr.from_host(A)
        Ch = mls.HostCsr.from_host(synth.Csr(R.nrows, R.ncols, R.row_ptr, R.col_idx, np.full(R.nnz, np.nan)))
        plan = mls.chunked_plan(A.row_ptr, A.row_ptr, A.ncols, R.row_ptr, plan_base(A, A, R) + 400_000,
                                nbuf=2, min_parts=2)
        assert plan.info["ws_bytes"] <= ws.nbytes
        mls.numeric_chunked(Ah, Ah, Ch, plan, ws)
        torch.cuda.synchronize()
        assert np.array_equal(Ch.values.numpy(), R.values)
        assert np.array_equal(C.values.cpu().numpy(), R.values)


@pytest.mark.parametrize("case", [("stencil", 12, 2.0), ("stencil", 12, 0.3), ("stencil", 12, 0.06),
                                  ("poisson", 0, 0.25), ("rmat", 12, 0.2), ("wide", 0, 0.2)])
@pytest.mark.parametrize("nbuf,min_parts", [(1, 1), (2, 3), (4, 1)])
@pytest.mark.parametrize("ac_where", ["pinned", "hbm"])
def test_knl_bitwise(case, nbuf, min_parts, ac_where):
    kind, n, frac = case
    print(f"chunkknl {case} nbuf={nbuf} min_parts={min_parts} A,C in {ac_where}", flush=True)
    A, B = case_inputs(kind, n)
    R, _ = oracle.spgemm(A, B)
    sB = op.range_bytes(B.row_ptr, 0, B.nrows)
    base = mls.chunked_plan(A.row_ptr, B.row_ptr, B.ncols, R.row_ptr, 10**10, knl=True).info
    budget = base["ws_bytes"] - base["chunk_bytes"] + int(sB * frac)
    try:
        plan = mls.chunked_plan(A.row_ptr, B.row_ptr, B.ncols, R.row_ptr, budget, nbuf=nbuf, min_parts=min_parts,
                                knl=True)
    except mls.SpgemmError as e:
        assert "BUDGET" in str(e)
        pytest.skip("budget below a single row")
    Cs = synth.Csr(R.nrows, R.ncols, R.row_ptr, R.col_idx, np.full(R.nnz, np.nan))
    place = mls.HostCsr.from_host if ac_where == "pinned" else mls.DeviceCsr.from_host
    Ax, Cx = place(A), place(Cs)
    mls.numeric_chunked(Ax, mls.HostCsr.from_host(B), Cx, plan)
    torch.cuda.synchronize()
    vals = Cx.values.numpy() if ac_where == "pinned" else Cx.values.cpu().numpy()
    assert np.array_equal(vals, R.values)
    info = plan.info
    assert info["algo"] == 3 and info["issued_h2d"] == info["h2d_bytes"] and info["issued_d2h"] == 0
    assert info["ws_bytes"] <= budget
    if frac < 1.0:
        assert info["n_b_parts"] > 1


def test_knl_refuses_pageable_a():
    A, B = case_inputs("poisson", 0)
    R, _ = oracle.spgemm(A, B)
    plan = mls.chunked_plan(A.row_ptr, B.row_ptr, B.ncols, R.row_ptr, 10**9, knl=True)
    Cd = mls.DeviceCsr.from_host(synth.Csr(R.nrows, R.ncols, R.row_ptr, R.col_idx, np.zeros(R.nnz)))
    Ad = mls.DeviceCsr.from_host(A)
    Bh = mls.HostCsr.from_host(B)
    import ctypes
    keep = np.ascontiguousarray(A.values)          # pageable host memory
    ha = mls.CsrT(A.nrows, A.ncols, A.nnz, Ad.row_ptr.data_ptr(), Ad.col_idx.data_ptr(), keep.ctypes.data)
    ws = mls.Workspace()
    nb = plan.info["ws_bytes"]
    st = mls.ChunkStreams()
    rc = mls.lib.spgemm_numeric_chunked(ctypes.byref(ha), ctypes.byref(Bh.handle()), ctypes.byref(Cd.handle()),
                                        plan._h, ws.get(nb), nb, st.compute.cuda_stream, st.h2d.cuda_stream,
                                        st.d2h.cuda_stream)
    assert rc == 1
