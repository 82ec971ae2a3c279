"""Hazard check of the chunked executor's copy / kernel / event sequence, on
the CPU (no GPU): the executor records what it would queue
(spgemm_numeric_chunked_trace) and a vector-clock model of its three streams
derives the happens-before order from stream order and event waits. Every
pair of accesses to overlapping bytes of the workspace (or of C's values in
host memory) of which one writes must be ordered: no part buffer is
overwritten while a kernel or a copy back still uses it, no kernel starts
before its parts arrived, no partial C value is copied back in before the
copy out that produced it, and no copy overwrites the workspace before the
work queued earlier on the compute stream is done. Plans of all three
algorithms, 1 to 4 inner buffers; a trace with one wait removed must fail."""
import numpy as np
import pytest

import oracle
import synth
import paper_1804_00695_amd as mls

WAIT, RECORD = 5, 4


def happens_before(trace):
    """Vector clock of every operation: {op: (stream, clock)}."""
    streams = {0: [0, 0, 0], 1: [0, 0, 0], 2: [0, 0, 0]}
    events, out = {}, {}
    seen = set()
    for op, kind, stream, event, *_ in trace:
        if op in seen:
            continue
        seen.add(op)
        vc = list(streams[stream])
        vc[stream] += 1
        if kind == WAIT and event in events:
            vc = [max(a, b) for a, b in zip(vc, events[event])]
        if kind == RECORD:
            events[event] = list(vc)
        streams[stream] = vc
        out[op] = (stream, vc)
    return out


def conflicts(trace):
    vcs = happens_before(trace)
    acc = [(op, space, write, lo, hi) for op, kind, stream, event, space, write, lo, hi in trace
           if space >= 0 and hi > lo]
    bad = []
    for x in range(len(acc)):
        ox, sx, wx, lx, hx = acc[x]
        for y in range(x + 1, len(acc)):
            oy, sy, wy, ly, hy = acc[y]
            if ox == oy or sx != sy or not (wx or wy) or hx <= ly or hy <= lx:
                continue
            s, vc = vcs[ox]
            if not vc[s] <= vcs[oy][1][s]:
                bad.append((acc[x], acc[y]))
    return bad


def operands(kind):
    if kind == "stencil":
        A = synth.stencil27_3d(9, amp=0.1)
        B = A
    elif kind == "wide":
        A = synth.poisson_csr(300, 2000, 10.0, 43)
        B = synth.poisson_csr(2000, 500, 5.0, 44)
    else:
        A = synth.poisson_csr(1500, 1200, 6.0, 41)
        B = synth.poisson_csr(1200, 1400, 9.0, 42)
    R, _ = oracle.spgemm(A, B, with_abs=False)
    return A, B, R


def sizes(A, B, R):
    f = lambda M: 4 * (M.nrows + 1) + 12 * M.nnz
    return f(A) + f(B) + f(R)


CASES = [(k, frac, nbuf, mp, knl) for k in ("stencil", "poisson", "wide")
         for frac in (3.0, 0.4, 0.12)
         for nbuf, mp in ((1, 1), (2, 1), (2, 4), (3, 1), (4, 3))
         for knl in (False, True)]


@pytest.mark.parametrize("kind,frac,nbuf,min_parts,knl", CASES)
def test_trace_has_no_unordered_conflict(kind, frac, nbuf, min_parts, knl):
    A, B, R = operands(kind)
    base = mls.chunked_plan(A.row_ptr, B.row_ptr, B.ncols, R.row_ptr, 10**10, knl=knl).info
    budget = base["ws_bytes"] - base["chunk_bytes"] + int(sizes(A, B, R) * frac)
    try:
        plan = mls.chunked_plan(A.row_ptr, B.row_ptr, B.ncols, R.row_ptr, budget, nbuf=nbuf, min_parts=min_parts,
                                knl=knl)
    except mls.SpgemmError:
        pytest.skip("budget below one row")
    trace = mls.chunked_trace(A, B, R, plan)
    info = plan.info
    assert info["n_steps"] > 0 and len(trace) > 0
    # the trace copies exactly the bytes of the schedule
    h2d = sum(hi - lo for op, kind_, st, ev, sp, w, lo, hi in trace if kind_ == 0 and sp == 0)
    d2h = sum(hi - lo for op, kind_, st, ev, sp, w, lo, hi in trace if kind_ == 1 and sp == 0)
    assert (h2d, d2h) == (info["h2d_bytes"], info["d2h_bytes"])
    assert conflicts(trace) == []


def test_checker_catches_a_missing_wait():
    A, B, R = operands("poisson")
    base = mls.chunked_plan(A.row_ptr, B.row_ptr, B.ncols, R.row_ptr, 10**10).info
    plan = mls.chunked_plan(A.row_ptr, B.row_ptr, B.ncols, R.row_ptr,
                            base["ws_bytes"] - base["chunk_bytes"] + sizes(A, B, R) // 8, nbuf=2)
    assert plan.info["n_ac_parts"] * plan.info["n_b_parts"] > 2
    trace = mls.chunked_trace(A, B, R, plan)
    waits = [op for op, kind, stream, *_ in trace if kind == WAIT and stream != 0]
    found = 0
    for drop in waits:
        t2 = [e for e in trace if e[0] != drop]
        found += bool(conflicts(t2))
    # removing any one of the copy streams' waits leaves some conflict open,
    # except waits already implied by stream order
    assert found >= len(waits) // 2
    # and without the first one (copies after earlier compute work) the
    # copies race with that work
    assert conflicts([e for e in trace if e[0] != waits[0]])
