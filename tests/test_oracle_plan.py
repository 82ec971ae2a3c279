"""Pins of the oracle's chunking heuristic and copy schedules (Sec. 3.3.1).

* BinarySearch against a linear scan (a different algorithm) and against the
  definition (contiguous, covering, within the limit, maximal);
* the paper's statements about Alg. "chunker": when B fits the big portion it
  is not partitioned and B-in-place runs; when A and C fit, they are not
  partitioned and AC-in-place runs; otherwise the cheaper copy order runs;
* the paper's statements about the schedules: AC-in-place copies A and C
  once and B once per part of A/C; B-in-place copies B once and A once per
  part of B; a problem that fits is copied in once and its result out once;
* executing a schedule on the CPU (row-range products C += A_r[:, b] B_b with
  the parts taken from the fast-memory buffers) gives A*B, and no buffer is
  overwritten while a pending step still needs its contents;
* Alg. "chunkknl": ceil(size(B) / FastSize) parts of at most the balanced
  size, B not cut when it fits (the data-placement case), B copied once, and
  its schedule executed on the CPU with A and C left in slow memory gives A*B.
"""
import numpy as np
import pytest

import oracle
import oracle.plan as op
import synth


def linear_scan_parts(sizes_prefix_fn, n, psize):
    parts, r0 = [], 0
    while r0 < n:
        r1 = r0
        while r1 < n and sizes_prefix_fn(r0, r1 + 1) <= psize:
            r1 += 1
        assert r1 > r0
        parts.append((r0, r1))
        r0 = r1
    return parts or [(0, 0)]


@pytest.mark.parametrize("seed", range(8))
def test_binary_search_vs_linear_scan(seed):
    g = synth.rng(seed)
    n = int(g.integers(1, 60))
    lens = g.integers(0, 20, n)
    rp = np.concatenate([[0], np.cumsum(lens)])
    fn = lambda a, b: op.range_bytes(rp, a, b)
    psize = int(g.integers(8 + 12 * lens.max(), 8 + 12 * lens.sum() + 50))
    parts = op.binary_search(fn, n, psize)
    assert parts == linear_scan_parts(fn, n, psize)
    assert parts[0][0] == 0 and parts[-1][1] == n
    for (a, b), (c, d) in zip(parts, parts[1:]):
        assert b == c
    for a, b in parts:
        assert fn(a, b) <= psize
        if b < n:
            assert fn(a, b + 1) > psize


def test_binary_search_row_too_big():
    rp = np.array([0, 1, 100, 101])
    with pytest.raises(op.BudgetError):
        op.binary_search(lambda a, b: op.range_bytes(rp, a, b), 3, 200)


def mats(nA, nB, lenA, lenB, lenC):
    arp = np.arange(nA + 1) * lenA
    brp = np.arange(nB + 1) * lenB
    crp = np.arange(nA + 1) * lenC
    return arp, brp, crp


def sizes(arp, brp, crp):
    return (op.range_bytes(arp, 0, len(arp) - 1), op.range_bytes(brp, 0, len(brp) - 1),
            op.range_bytes(crp, 0, len(crp) - 1))


def test_branch1_b_fits():
    arp, brp, crp = mats(1000, 100, 10, 5, 30)
    sA, sB, sC = sizes(arp, brp, crp)
    fast = 2 * sB
    p = op.partition(arp, brp, crp, fast)
    assert p.branch == 1 and p.algo == op.CHUNK2 and p.p_b == [(0, 100)]
    assert len(p.p_ac) > 1
    assert p.ws_chunks <= fast


def test_branch2_ac_fits():
    arp, brp, crp = mats(100, 1000, 10, 30, 5)
    sA, sB, sC = sizes(arp, brp, crp)
    fast = 2 * (sA + sC)
    p = op.partition(arp, brp, crp, fast)
    assert p.branch == 2 and p.algo == op.CHUNK1 and p.p_ac == [(0, 100)]
    assert len(p.p_b) > 1 and p.ws_chunks <= fast


def test_everything_fits_is_copied_once():
    arp, brp, crp = mats(500, 400, 7, 7, 20)
    sA, sB, sC = sizes(arp, brp, crp)
    p = op.partition(arp, brp, crp, 10 * (sA + sB + sC))
    assert p.branch == 1 and p.p_ac == [(0, 500)] and p.p_b == [(0, 400)]
    assert p.h2d == sA + sB + (sC - 8 * int(crp[-1]))     # C's structure in
    assert p.d2h == 8 * int(crp[-1])                      # C's values out


@pytest.mark.parametrize("shape", [(3000, 3000, 9, 9, 40), (3000, 3000, 30, 20, 60), (2000, 5000, 40, 30, 2)])
def test_branches_3_4_pick_cheaper(shape):
    arp, brp, crp = mats(*shape)
    sA, sB, sC = sizes(arp, brp, crp)
    fast = (sA + sB + sC) // 5
    p = op.partition(arp, brp, crp, fast)
    assert p.branch in (3, 4)
    assert (sA + 2 * sC > sB) == (p.branch == 3)
    assert p.h2d + p.d2h == min(p.cost1, p.cost2)
    assert p.ws_chunks <= fast


def count_bytes(steps, kind, mat):
    return sum(s[5] for s in steps if s[0] == kind and s[1] == mat)


def test_chunk1_copies_ac_once_b_per_ac_part():
    arp, brp, crp = mats(800, 2000, 10, 20, 15)
    sA, sB, sC = sizes(arp, brp, crp)
    p = op.partition(arp, brp, crp, (sA + sC) // 2 + sB // 3)
    assert p.algo == op.CHUNK1
    n_ac = len(p.p_ac)
    a_once = sum(op.range_bytes(arp, a, b) for a, b in p.p_ac)
    b_once = sum(op.range_bytes(brp, a, b) for a, b in p.p_b)
    assert count_bytes(p.steps, op.H2D, op.MAT_A) == a_once
    assert count_bytes(p.steps, op.H2D, op.MAT_B) == n_ac * b_once
    assert count_bytes(p.steps, op.D2H, op.MAT_CVAL) == 8 * int(crp[-1])
    assert count_bytes(p.steps, op.H2D, op.MAT_CVAL) == 0


def test_chunk2_copies_b_once_a_per_b_part():
    arp, brp, crp = mats(3000, 300, 5, 40, 6)
    p_ac = [(0, 1000), (1000, 2500), (2500, 3000)]
    p_b = [(0, 100), (100, 120), (120, 300)]
    for p in (op.Plan(op.CHUNK2, 0, 0, p_ac, p_b, 1), op.Plan(op.CHUNK2, 0, 0, p_ac, p_b, 2)):
        steps = op.schedule(p, arp, brp, crp)
        n_b = len(p_b)
        a_once = sum(op.range_bytes(arp, a, b) for a, b in p_ac)
        assert count_bytes(steps, op.H2D, op.MAT_B) == op.range_bytes(brp, 0, 300) + 4 * 2
        assert count_bytes(steps, op.H2D, op.MAT_A) == n_b * a_once
        assert count_bytes(steps, op.D2H, op.MAT_CVAL) == n_b * 8 * int(crp[-1])
        assert count_bytes(steps, op.H2D, op.MAT_CVAL) == (n_b - 1) * 8 * int(crp[-1])
        h2d, d2h = op.copy_bytes(op.CHUNK2, p_ac, p_b, arp, brp, crp)
        assert h2d == sum(s[5] for s in steps if s[0] == op.H2D)
        assert d2h == sum(s[5] for s in steps if s[0] == op.D2H)


def test_branch4_can_choose_b_in_place():
    arp, brp, crp = mats(300, 3000, 5, 40, 6)
    sA, sB, sC = sizes(arp, brp, crp)
    fast = int((sA + sC) / 0.8)
    p = op.partition(arp, brp, crp, fast)
    assert p.branch == 4
    assert p.algo == (op.CHUNK2 if p.cost2 < p.cost1 else op.CHUNK1)
    assert p.h2d + p.d2h == min(p.cost1, p.cost2)


def test_extensions_min_parts_and_double_buffer():
    arp, brp, crp = mats(1000, 100, 10, 5, 30)
    sA, sB, sC = sizes(arp, brp, crp)
    fast = 10 * (sA + sB + sC)
    p = op.partition(arp, brp, crp, fast, nbuf=2, min_parts=6)
    assert p.branch == 1 and p.nbuf_inner == 2
    assert len(p.p_ac) >= 6
    assert p.ws_chunks <= fast
    slots = [s[6] for s in p.steps if s[0] == op.KERNEL]
    assert slots == [i % 2 for i in range(len(slots))]


def simulate(plan, A, B, C_struct):
    """Run the schedule on the CPU with explicit fast-memory buffers.

    Buffers hold row ranges; a kernel step reads only what sits in the
    buffers and accumulates C_r += A_r[:, b0:b1] B_b in the C buffer of its
    slot. Checks that every kernel finds the ranges it needs in place.
    """
    Ad, Bd = synth.to_dense(A), synth.to_dense(B)
    slow_C = np.zeros((A.nrows, B.ncols))
    outer_is_ac = plan.algo in (op.CHUNK1, op.CHUNKKNL)
    buf_a, buf_c, buf_b = {}, {}, {}
    if plan.algo == op.CHUNKKNL:
        # A and C stay in slow memory and are used in place
        buf_a[0] = (0, A.nrows, Ad)
        buf_c[0] = [0, A.nrows, slow_C]
    for kind, mat, part, r0, r1, nbytes, slot in plan.steps:
        s_ac = 0 if outer_is_ac else slot
        s_b = slot if outer_is_ac else 0
        if kind == op.H2D and mat == op.MAT_A:
            buf_a[s_ac] = (r0, r1, Ad[r0:r1].copy())
        elif kind == op.H2D and mat == op.MAT_CSTRUCT:
            buf_c[s_ac] = [r0, r1, None]
        elif kind == op.ZERO:
            buf_c[s_ac][2] = np.zeros((r1 - r0, B.ncols))
        elif kind == op.H2D and mat == op.MAT_CVAL:
            buf_c[s_ac][2] = slow_C[r0:r1].copy()
        elif kind == op.H2D and mat == op.MAT_B:
            buf_b[s_b] = (r0, r1, Bd[r0:r1].copy())
        elif kind == op.KERNEL:
            a0, a1, Ablk = buf_a[s_ac]
            c = buf_c[s_ac]
            b0, b1, Bblk = buf_b[s_b]
            assert (b0, b1) == (r0, r1) and (c[0], c[1]) == (a0, a1) == plan.p_ac[part]
            c[2] += Ablk[:, b0:b1] @ Bblk
        elif kind == op.D2H:
            c = buf_c[s_ac]
            assert (c[0], c[1]) == (r0, r1)
            slow_C[r0:r1] = c[2]
    return slow_C


@pytest.mark.parametrize("budget_div", [1, 3, 6, 12])
@pytest.mark.parametrize("nbuf,min_parts", [(1, 1), (2, 1), (2, 4)])
def test_schedule_executes_to_product(budget_div, nbuf, min_parts):
    A = synth.poisson_csr(120, 90, 6.0, 60)
    B = synth.poisson_csr(90, 110, 7.0, 61)
    C, _ = oracle.spgemm(A, B)
    sA, sB, sC = sizes(A.row_ptr, B.row_ptr, C.row_ptr)
    fast = (sA + sB + sC) * 2 // budget_div
    try:
        p = op.partition(A.row_ptr, B.row_ptr, C.row_ptr, fast, nbuf=nbuf, min_parts=min_parts)
    except op.BudgetError:
        pytest.skip("budget below one row")
    got = simulate(p, A, B, C)
    ref = synth.to_dense(A) @ synth.to_dense(B)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    assert p.ws_chunks <= fast
    assert p.h2d == count_bytes(p.steps, op.H2D, op.MAT_A) + count_bytes(p.steps, op.H2D, op.MAT_B) + \
        count_bytes(p.steps, op.H2D, op.MAT_CSTRUCT) + count_bytes(p.steps, op.H2D, op.MAT_CVAL)
    assert p.d2h == count_bytes(p.steps, op.D2H, op.MAT_CVAL)


@pytest.mark.parametrize("lenB,nbuf", [(5, 1), (17, 1), (9, 2), (9, 3), (9, 4)])
def test_knl_parts_follow_the_algorithm(lenB, nbuf):
    arp, brp, crp = mats(400, 3000, 7, lenB, 20)
    sA, sB, sC = sizes(arp, brp, crp)
    for div in (1.0, 2.5, 7.0, 19.0):
        fast = int(sB / div) + 64
        p = op.partition_knl(arp, brp, crp, fast, nbuf=nbuf)
        np_ = -(-sB // (fast // nbuf))        # ceil(size(B) / portion)
        psize = -(-sB // np_)
        assert p.algo == op.CHUNKKNL and p.p_ac == [(0, 400)]
        assert p.p_b[0][0] == 0 and p.p_b[-1][1] == 3000
        assert all(b == c for (_, b), (c, _) in zip(p.p_b, p.p_b[1:]))
        assert all(op.range_bytes(brp, a, b) <= psize for a, b in p.p_b)
        # uniform rows: the balanced size is met by np or np + 1 greedy parts
        assert len(p.p_b) in (np_, np_ + 1)
        assert p.h2d == sum(op.range_bytes(brp, a, b) for a, b in p.p_b) and p.d2h == 0
        assert p.ws_chunks <= fast
        assert [s[6] for s in p.steps if s[0] == op.KERNEL] == [i % nbuf for i in range(len(p.p_b))]


def test_knl_b_fits_is_not_cut():
    arp, brp, crp = mats(400, 300, 7, 9, 20)
    sA, sB, sC = sizes(arp, brp, crp)
    p = op.partition_knl(arp, brp, crp, 4 * sB)
    assert p.p_b == [(0, 300)] and p.h2d == sB
    cval = 8 * int(crp[-1])
    assert p.zero_copy == sA + (sC - cval) + cval     # one pass: A, C's structure read, C's values written


@pytest.mark.parametrize("budget_div", [1, 3, 6, 12])
@pytest.mark.parametrize("nbuf,min_parts", [(1, 1), (2, 1), (3, 4)])
def test_knl_schedule_executes_to_product(budget_div, nbuf, min_parts):
    A = synth.poisson_csr(120, 90, 6.0, 62)
    B = synth.poisson_csr(90, 110, 7.0, 63)
    C, _ = oracle.spgemm(A, B)
    sB = op.range_bytes(B.row_ptr, 0, B.nrows)
    try:
        p = op.partition_knl(A.row_ptr, B.row_ptr, C.row_ptr, sB * 2 // budget_div, nbuf=nbuf, min_parts=min_parts)
    except op.BudgetError:
        pytest.skip("budget below one row")
    got = simulate(p, A, B, C)
    ref = synth.to_dense(A) @ synth.to_dense(B)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
