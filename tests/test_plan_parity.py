"""The library's chunk planner (C++, host only) against the oracle planner:
identical parts, branch, algorithm, byte counts and copy schedule, on
synthetic row-pointer shapes that drive every branch of Alg. "chunker"."""
import numpy as np
import pytest

import oracle
import oracle.plan as op
import synth
import paper_1804_00695_amd as mls


def shapes():
    g = synth.rng(77)
    out = []
    for nA, nB, la, lb, lc in [(1000, 100, 10, 5, 30), (100, 1000, 10, 30, 5), (3000, 3000, 9, 9, 40),
                               (3000, 3000, 30, 20, 60), (2000, 5000, 40, 30, 2), (300, 3000, 5, 40, 6),
                               (5000, 5000, 3, 3, 9)]:
        out.append((np.arange(nA + 1) * la, np.arange(nB + 1) * lb, np.arange(nA + 1) * lc))
    for _ in range(6):  # ragged rows
        nA, nB = int(g.integers(50, 2000)), int(g.integers(50, 2000))
        out.append((np.concatenate([[0], np.cumsum(g.poisson(8, nA))]),
                    np.concatenate([[0], np.cumsum(g.poisson(12, nB))]),
                    np.concatenate([[0], np.cumsum(g.poisson(40, nA))])))
    return out


def size(rp):
    return op.range_bytes(rp, 0, len(rp) - 1)


@pytest.mark.parametrize("case", range(13))
@pytest.mark.parametrize("frac", [10.0, 1.0, 0.5, 0.2, 0.07])
@pytest.mark.parametrize("nbuf,min_parts", [(1, 1), (2, 1), (2, 5), (3, 1), (4, 6)])
def test_planner_matches_oracle(case, frac, nbuf, min_parts):
    arp, brp, crp = shapes()[case]
    total = size(arp) + size(brp) + size(crp)
    budget = int(total * frac) + 100000
    try:
        p = mls.chunked_plan(arp, brp, 10**6, crp, budget, nbuf=nbuf, min_parts=min_parts)
    except mls.SpgemmError as e:
        assert "BUDGET" in str(e)
        # the reserve (budget - FastSize) does not depend on the budget
        big = mls.chunked_plan(arp, brp, 10**6, crp, 100 * total, nbuf=nbuf, min_parts=min_parts)
        fast = budget - (100 * total - big.info["fast_bytes"])
        if fast > 0:
            with pytest.raises(op.BudgetError):
                op.partition(arp, brp, crp, fast, nbuf=nbuf, min_parts=min_parts)
        return
    info = p.info
    ref = op.partition(arp, brp, crp, info["fast_bytes"], nbuf=nbuf, min_parts=min_parts)
    assert p.parts(0) == [tuple(x) for x in ref.p_ac]
    assert p.parts(1) == [tuple(x) for x in ref.p_b]
    assert (info["branch"], info["algo"], info["nbuf_inner"]) == (ref.branch, ref.algo, ref.nbuf_inner)
    assert (info["h2d_bytes"], info["d2h_bytes"]) == (ref.h2d, ref.d2h)
    assert (info["cost_chunk1"], info["cost_chunk2"]) == (ref.cost1, ref.cost2)
    assert info["chunk_bytes"] == ref.ws_chunks
    assert p.steps() == [tuple(s) for s in ref.steps]
    assert info["ws_bytes"] <= budget


def test_budget_too_small():
    arp, brp, crp = shapes()[0]
    with pytest.raises(mls.SpgemmError, match="BUDGET"):
        mls.chunked_plan(arp, brp, 10**6, crp, 1000)


def test_real_product_plan():
    A = synth.stencil27_3d(16, amp=0.1)
    C, _ = oracle.spgemm(A, A, with_abs=False)
    total = size(A.row_ptr) * 2 + size(C.row_ptr)
    for frac in (4.0, 0.6, 0.25):
        p = mls.chunked_plan(A.row_ptr, A.row_ptr, A.ncols, C.row_ptr, int(total * frac) + 2_000_000, nbuf=2)
        ref = op.partition(A.row_ptr, A.row_ptr, C.row_ptr, p.info["fast_bytes"], nbuf=2)
        assert p.steps() == [tuple(s) for s in ref.steps]


@pytest.mark.parametrize("case", range(13))
@pytest.mark.parametrize("frac", [4.0, 1.0, 0.3, 0.08])
@pytest.mark.parametrize("nbuf,min_parts", [(1, 1), (2, 1), (3, 4), (4, 1)])
def test_knl_planner_matches_oracle(case, frac, nbuf, min_parts):
    arp, brp, crp = shapes()[case]
    budget = int(size(brp) * frac) + 100000
    try:
        p = mls.chunked_plan(arp, brp, 10**6, crp, budget, nbuf=nbuf, min_parts=min_parts, knl=True)
    except mls.SpgemmError as e:
        assert "BUDGET" in str(e)
        big = mls.chunked_plan(arp, brp, 10**6, crp, 100 * size(brp) + 10**8, nbuf=nbuf, knl=True)
        fast = budget - (100 * size(brp) + 10**8 - big.info["fast_bytes"])
        if fast > 0:
            with pytest.raises(op.BudgetError):
                op.partition_knl(arp, brp, crp, fast, nbuf=nbuf, min_parts=min_parts)
        return
    info = p.info
    ref = op.partition_knl(arp, brp, crp, info["fast_bytes"], nbuf=nbuf, min_parts=min_parts)
    assert info["algo"] == 3 and info["branch"] == 0
    assert p.parts(0) == [tuple(x) for x in ref.p_ac]
    assert p.parts(1) == [tuple(x) for x in ref.p_b]
    assert (info["h2d_bytes"], info["d2h_bytes"], info["zero_copy_bytes"]) == (ref.h2d, ref.d2h, ref.zero_copy)
    assert info["chunk_bytes"] == ref.ws_chunks and info["nbuf_inner"] == nbuf
    assert p.steps() == [tuple(s) for s in ref.steps]
    assert info["ws_bytes"] <= budget


def test_nbuf_range():
    arp, brp, crp = shapes()[0]
    for bad in (0, 5):
        with pytest.raises(mls.SpgemmError, match="INVALID_ARG"):
            mls.chunked_plan(arp, brp, 10**6, crp, 10**9, nbuf=bad)
