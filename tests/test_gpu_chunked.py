"""GPU parity of the chunked numeric phase (pinned host A, B, C; HBM budget).

For budgets from "everything fits" down to dozens of parts, with single and
double buffering: C's values must equal the oracle's bit for bit (and the
in-HBM GPU result), and the bytes the executor queued must equal the plan's
schedule (which equals the oracle planner's, see test_plan_parity)."""
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
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("nbuf,min_parts", [(1, 1), (2, 1), (2, 4)])
def test_chunked_bitwise(case, nbuf, min_parts):
    kind, n, frac = case
    if kind == "stencil":
        A = synth.stencil27_3d(n, amp=0.1)
        B = A
    elif kind == "rmat":
        G = synth.rmat_graph(n, 8, seed=5)
        A = synth.Csr(G.nrows, G.ncols, G.row_ptr, G.col_idx, synth.normal_values(len(G.col_idx), 8))
        B = A
    else:
        A = synth.poisson_csr(3000, 2500, 6.0, 41)
        B = synth.poisson_csr(2500, 2800, 9.0, 42)
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
