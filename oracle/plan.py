"""Oracle for the chunking decision and copy schedule -- TEST INFRASTRUCTURE ONLY.

Follows Sec. 3.3.1 of the paper (Alg. "chunker", the "Partition" heuristic;
Algs. "chunk1" = AC in place and "chunk2" = B in place) and Sec. 3.2.2
(Alg. "chunkknl": only B is partitioned, A and C stay in slow memory), in
plain Python, in the paper's order. Readings taken where the text is silent
or garbled:

* size of a row range [r0, r1) of a CSR matrix X = 4*(r1 - r0 + 1) bytes of
  row pointers + 12 bytes per stored entry (int32 index + fp64 value).
  C counts the same way (its structure is known from the symbolic phase and
  its values are accumulated in fast memory).
* BinarySearch(X, pSize): greedy maximal row ranges from row 0, each the
  longest range whose size is <= pSize (an upper bound search on the byte
  prefix). A single row larger than its portion is an error.
* "balanced partition size" for a total T and a portion S:
  ceil(T / max(ceil(T / S), min_parts)); if the largest single row is larger
  than that, the portion itself is used as the limit.
* "Add left over from big to small portion": the inner-loop matrix gets
  FastSize minus what the outer-loop matrix actually occupies (its largest
  part).
* BigPortion = floor(3/4 FastSize), SmallPortion = FastSize - BigPortion.
* Extensions (both off in the paper's setting nbuf=1, min_parts=1): ``nbuf``
  buffers for the inner-loop matrix (double buffering, so copies overlap the
  kernel; the inner portion is divided among them), and ``min_parts`` (the
  inner matrix is cut into at least that many parts so that copy-in, compute
  and copy-out of consecutive parts can overlap even when it fits whole).
* Copy cost = bytes actually moved, both directions (the formulas printed in
  the paper for chunk1 and chunk2 differ in how they count C):
    chunk1: H2D A and C's structure once per AC part, each B part once per AC
            part; D2H C's values once.
    chunk2: H2D each B part once; per B part, every AC part's A and C
            structure, plus C's partial values from the second B part on;
            D2H C's values once per B part.
  Ties go to the algorithm natural to the branch.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

CHUNK1, CHUNK2, CHUNKKNL = 1, 2, 3   # AC in place / B in place / only B moves
H2D, D2H, KERNEL, ZERO = 0, 1, 2, 3
MAT_A, MAT_B, MAT_CSTRUCT, MAT_CVAL = 0, 1, 2, 3


class BudgetError(ValueError):
    pass


def range_bytes(rp: np.ndarray, r0: int, r1: int) -> int:
    return 4 * (r1 - r0 + 1) + 12 * (int(rp[r1]) - int(rp[r0]))


def struct_bytes(rp: np.ndarray, r0: int, r1: int) -> int:
    return 4 * (r1 - r0 + 1) + 4 * (int(rp[r1]) - int(rp[r0]))


def binary_search(size_fn, n: int, psize: int) -> List[Tuple[int, int]]:
    """Greedy maximal ranges [r0, r1) with size_fn(r0, r1) <= psize."""
    if n == 0:
        return [(0, 0)]
    parts = []
    r0 = 0
    while r0 < n:
        lo, hi = r0, n          # largest r1 in (r0, n] with size <= psize
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if size_fn(r0, mid) <= psize:
                lo = mid
            else:
                hi = mid - 1
        if lo == r0:
            raise BudgetError(f"row {r0} does not fit a part of {psize} bytes")
        parts.append((r0, lo))
        r0 = lo
    return parts


def _ceil_div(a: int, b: int) -> int:
    return -(-a // b)


def balanced(total: int, portion: int, max_row: int, min_parts: int = 1) -> int:
    if portion <= 0:
        raise BudgetError("no memory left for a portion")
    nparts = max(_ceil_div(total, portion), min_parts, 1)
    p = _ceil_div(total, nparts) if total > 0 else 0
    if p < max_row:
        p = portion
    return p


@dataclass
class Plan:
    algo: int
    branch: int
    fast: int
    p_ac: List[Tuple[int, int]]
    p_b: List[Tuple[int, int]]
    nbuf_inner: int
    h2d: int = 0
    d2h: int = 0
    cost1: int = 0
    cost2: int = 0
    ws_chunks: int = 0
    steps: list = field(default_factory=list)
    zero_copy: int = 0       # chunkknl: bytes the kernels move in place in slow memory


def _sizes(arp, brp, crp):
    nA = len(arp) - 1
    nB = len(brp) - 1
    sA = range_bytes(arp, 0, nA)
    sB = range_bytes(brp, 0, nB)
    sC = range_bytes(crp, 0, nA)
    return nA, nB, sA, sB, sC


def copy_bytes(algo, p_ac, p_b, arp, brp, crp):
    """(h2d, d2h) bytes of the schedule of ``algo`` over the given parts."""
    a_c = sum(range_bytes(arp, r0, r1) + struct_bytes(crp, r0, r1) for r0, r1 in p_ac)
    cval = 8 * (int(crp[-1]) - int(crp[0]))
    b = sum(range_bytes(brp, b0, b1) for b0, b1 in p_b)
    if algo == CHUNK1:
        return a_c + len(p_ac) * b, cval
    return b + len(p_b) * a_c + (len(p_b) - 1) * cval, len(p_b) * cval


def partition(arp, brp, crp, fast: int, nbuf: int = 1, min_parts: int = 1) -> Plan:
    """Alg. "chunker" (Partition): row parts of A/C and of B, and the algorithm."""
    arp = np.asarray(arp, dtype=np.int64)
    brp = np.asarray(brp, dtype=np.int64)
    crp = np.asarray(crp, dtype=np.int64)
    nA, nB, sA, sB, sC = _sizes(arp, brp, crp)
    big = (3 * fast) // 4
    small = fast - big

    def size_ac(r0, r1):
        return range_bytes(arp, r0, r1) + range_bytes(crp, r0, r1)

    def size_b(r0, r1):
        return range_bytes(brp, r0, r1)

    # largest single row: 8 bytes of row pointers per matrix plus 12 per entry
    max_row_ac = int((16 + 12 * (np.diff(arp) + np.diff(crp))).max()) if nA else 0
    max_row_b = int((8 + 12 * np.diff(brp)).max()) if nB else 0

    def maxpart(parts, fn):
        return max(fn(r0, r1) for r0, r1 in parts)

    if sB < big:
        branch, natural = 1, CHUNK2
        p_b = [(0, nB)]
        portion = (fast - sB) // nbuf
        p_ac = binary_search(size_ac, nA, balanced(sA + sC, portion, max_row_ac, min_parts))
        algo = CHUNK2
    elif sA + sC < big:
        branch, natural = 2, CHUNK1
        p_ac = [(0, nA)]
        portion = (fast - sA - sC) // nbuf
        p_b = binary_search(size_b, nB, balanced(sB, portion, max_row_b, min_parts))
        algo = CHUNK1
    elif sA + 2 * sC > sB:
        branch, natural = 3, CHUNK1
        p_ac = binary_search(size_ac, nA, balanced(sA + sC, big, max_row_ac))
        portion = (small + big - maxpart(p_ac, size_ac)) // nbuf
        p_b = binary_search(size_b, nB, balanced(sB, portion, max_row_b, min_parts))
        algo = None
    else:
        branch, natural = 4, CHUNK2
        p_b = binary_search(size_b, nB, balanced(sB, big, max_row_b))
        portion = (small + big - maxpart(p_b, size_b)) // nbuf
        p_ac = binary_search(size_ac, nA, balanced(sA + sC, portion, max_row_ac, min_parts))
        algo = None

    c1 = sum(copy_bytes(CHUNK1, p_ac, p_b, arp, brp, crp))
    c2 = sum(copy_bytes(CHUNK2, p_ac, p_b, arp, brp, crp))
    if algo is None:
        if c1 < c2:
            algo = CHUNK1
        elif c2 < c1:
            algo = CHUNK2
        else:
            algo = natural
    nbuf_inner = nbuf if algo == natural else 1
    h2d, d2h = copy_bytes(algo, p_ac, p_b, arp, brp, crp)
    if algo == CHUNK1:
        ws = maxpart(p_ac, size_ac) + nbuf_inner * maxpart(p_b, size_b)
    else:
        ws = maxpart(p_b, size_b) + nbuf_inner * maxpart(p_ac, size_ac)
    plan = Plan(algo, branch, fast, p_ac, p_b, nbuf_inner, h2d, d2h, c1, c2, ws)
    plan.steps = schedule(plan, arp, brp, crp)
    return plan


def schedule(plan: Plan, arp, brp, crp):
    """The copy / kernel steps of chunk1 or chunk2 in issue order.

    Each step is (kind, matrix, part, r0, r1, bytes, slot); ``slot`` is the
    buffer of the inner-loop matrix (0 for outer-loop copies), counting inner
    iterations globally modulo nbuf_inner. Kernel steps carry the AC part in
    ``part``, the B row range in (r0, r1) and the inner slot.
    """
    steps = []
    it = 0
    if plan.algo == CHUNK1:
        for r, (r0, r1) in enumerate(plan.p_ac):
            steps.append((H2D, MAT_A, r, r0, r1, range_bytes(arp, r0, r1), 0))
            steps.append((H2D, MAT_CSTRUCT, r, r0, r1, struct_bytes(crp, r0, r1), 0))
            steps.append((ZERO, MAT_CVAL, r, r0, r1, 0, 0))
            for b, (b0, b1) in enumerate(plan.p_b):
                slot = it % plan.nbuf_inner
                steps.append((H2D, MAT_B, b, b0, b1, range_bytes(brp, b0, b1), slot))
                steps.append((KERNEL, MAT_CVAL, r, b0, b1, 0, slot))
                it += 1
            steps.append((D2H, MAT_CVAL, r, r0, r1, 8 * (int(crp[r1]) - int(crp[r0])), 0))
    else:
        for b, (b0, b1) in enumerate(plan.p_b):
            steps.append((H2D, MAT_B, b, b0, b1, range_bytes(brp, b0, b1), 0))
            for r, (r0, r1) in enumerate(plan.p_ac):
                slot = it % plan.nbuf_inner
                cv = 8 * (int(crp[r1]) - int(crp[r0]))
                steps.append((H2D, MAT_A, r, r0, r1, range_bytes(arp, r0, r1), slot))
                steps.append((H2D, MAT_CSTRUCT, r, r0, r1, struct_bytes(crp, r0, r1), slot))
                if b == 0:
                    steps.append((ZERO, MAT_CVAL, r, r0, r1, 0, slot))
                else:
                    steps.append((H2D, MAT_CVAL, r, r0, r1, cv, slot))
                steps.append((KERNEL, MAT_CVAL, r, b0, b1, 0, slot))
                steps.append((D2H, MAT_CVAL, r, r0, r1, cv, slot))
                it += 1
    return steps


def partition_knl(arp, brp, crp, fast: int, nbuf: int = 1, min_parts: int = 1) -> Plan:
    """Alg. "chunkknl": np = ceil(size(B) / FastSize) parts of balanced size
    size(B) / np, cut by BinarySearch; A and C are not copied (the kernels use
    them in slow memory). With nbuf buffers the portion of a part is
    FastSize / nbuf; min_parts cuts at least that many parts."""
    arp = np.asarray(arp, dtype=np.int64)
    brp = np.asarray(brp, dtype=np.int64)
    crp = np.asarray(crp, dtype=np.int64)
    nA, nB, sA, sB, sC = _sizes(arp, brp, crp)
    max_row_b = int((8 + 12 * np.diff(brp)).max()) if nB else 0

    def size_b(r0, r1):
        return range_bytes(brp, r0, r1)

    p_b = binary_search(size_b, nB, balanced(sB, fast // nbuf, max_row_b, min_parts))
    plan = Plan(CHUNKKNL, 0, fast, [(0, nA)], p_b, nbuf)
    plan.h2d = sum(size_b(b0, b1) for b0, b1 in p_b)
    plan.d2h = 0
    plan.ws_chunks = nbuf * max(size_b(b0, b1) for b0, b1 in p_b)
    nparts = len(p_b)
    cval = 8 * (int(crp[-1]) - int(crp[0]))
    # every pass reads A and C's structure where they are and writes C's
    # values; the passes after the first read the previous values back
    plan.zero_copy = nparts * (sA + struct_bytes(crp, 0, nA)) + nparts * cval + (nparts - 1) * cval
    plan.steps = []
    for q, (b0, b1) in enumerate(p_b):
        plan.steps.append((H2D, MAT_B, q, b0, b1, size_b(b0, b1), q % nbuf))
        plan.steps.append((KERNEL, MAT_CVAL, 0, b0, b1, 0, q % nbuf))
    return plan
