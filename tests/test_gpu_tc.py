"""GPU parity of triangle counting: per-row int64 counts and the total must
equal the oracle's bit for bit (integers), on closed-form families and R-MAT
graphs, through the LDS classes and the global spill path."""
import numpy as np
import pytest
import torch
from math import comb

import oracle
import synth

pytestmark = pytest.mark.gpu
mls = pytest.importorskip("paper_1804_00695_amd")


@pytest.fixture(autouse=True)
def _reset():
    yield
    mls.set_option(mls._abi.OPT_FORCE_SPILL, 0)
    mls.set_option(mls._abi.OPT_FORCE_CLASS, -1)


def gpu_tc(G):
    perm, (n, lrp, lci) = mls.tc_lower(G)
    L = synth.Csr(n, n, lrp, lci, None)
    counts, total = mls.triangle_count(mls.DeviceCsr.from_host(L))
    torch.cuda.synchronize()
    return counts.cpu().numpy(), total, L


def check(G):
    counts, total, L = gpu_tc(G)
    ref_total, ref_counts, _, RL = oracle.triangle_count(G)
    assert np.array_equal(L.col_idx, RL.col_idx)
    assert total == ref_total
    assert np.array_equal(counts, ref_counts)
    return total


def test_complete_graphs():
    for n in (3, 4, 17, 64):
        e = [(i, j) for i in range(n) for j in range(i + 1, n)]
        a = np.array(e)
        assert check(synth.graph_from_edges(n, a[:, 0], a[:, 1])) == comb(n, 3)


def test_wheel_and_cycle():
    n = 40
    cyc = [(i, (i + 1) % n) for i in range(n)]
    a = np.array(cyc + [(n, i) for i in range(n)])
    assert check(synth.graph_from_edges(n + 1, a[:, 0], a[:, 1])) == n
    a = np.array(cyc)
    assert check(synth.graph_from_edges(n, a[:, 0], a[:, 1])) == 0


@pytest.mark.parametrize("scale,ef,seed", [(10, 8, 1), (14, 16, 3), (16, 16, 4)])
def test_rmat(scale, ef, seed):
    check(synth.rmat_graph(scale, ef, seed=seed))


def test_long_spread_rows_and_spill():
    # a random core of 8000 vertices (degree ~300) plus low-degree "fans" tied
    # to ~280 core vertices each: the fans' rows of L hold ~180 distinct
    # 32-column words, which takes them out of the first LDS class
    g = synth.rng(9)
    nc, nf = 8000, 24
    m = nc * 150
    src, dst = g.integers(0, nc, m), g.integers(0, nc, m)
    fs = np.repeat(np.arange(nc, nc + nf), 280)
    fd = g.integers(0, nc, fs.size)
    G = synth.graph_from_edges(nc + nf, np.concatenate([src, fs]), np.concatenate([dst, fd]))
    check(G)
    mls.set_option(mls._abi.OPT_FORCE_SPILL, 1)
    check(synth.rmat_graph(11, 8, seed=2))


def lower_with_word_rows(targets, n, seed):
    """Strictly lower L: sparse random rows near the diagonal, plus one row per
    target w holding exactly w distinct 32-column words (1-3 columns each);
    rows named by a target's columns share some of them, so they close
    triangles."""
    g = synth.rng(seed)
    rows = [set() for _ in range(n)]
    for i in range(1, n):
        k = int(g.integers(0, 5))
        if k:
            rows[i].update(g.integers(max(0, i - 2000), i, k).tolist())
    special = {}
    for t, w in enumerate(targets):
        i = n - 1 - 7 * t
        words = g.choice(i >> 5, size=w, replace=False)
        cols = set()
        for q in words.tolist():
            cols.update((32 * q + g.choice(32, size=int(g.integers(1, 4)), replace=False)).tolist())
        rows[i] = cols
        special[i] = w
        sc = sorted(cols)
        for j in g.choice(sc, size=min(40, len(sc)), replace=False).tolist():
            below = [c for c in sc if c < j]
            if below:
                rows[j].update(g.choice(below, size=min(20, len(below)), replace=False).tolist())
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate([np.array(sorted(r), dtype=np.int32) for r in rows])
    for i, w in special.items():
        assert np.unique(ci[rp[i]:rp[i + 1]] >> 5).size == w
    return synth.Csr(n, n, rp, ci, None)


def test_class_boundaries():
    # own-word counts on both sides of every class limit (half the table of
    # 64, 256, 512, 1024 and 4096 slots); the row of 2049 words spills
    targets = [32, 33, 128, 129, 256, 257, 512, 513, 2048, 2049]
    L = lower_with_word_rows(targets, 70000, 23)
    counts, total = mls.triangle_count(mls.DeviceCsr.from_host(L))
    torch.cuda.synchronize()
    ref_counts, ref_total = oracle.tc_count(L)
    assert total == ref_total
    assert np.array_equal(counts.cpu().numpy(), ref_counts)
    assert ref_total > 0


@pytest.mark.parametrize("cls", [0, 1, 2, 3, 4])
def test_forced_class(cls):
    mls.set_option(mls._abi.OPT_FORCE_CLASS, cls)
    check(synth.rmat_graph(10, 8, seed=7))
    n = 30
    e = [(i, j) for i in range(n) for j in range(i + 1, n)]
    a = np.array(e)
    assert check(synth.graph_from_edges(n, a[:, 0], a[:, 1])) == comb(n, 3)
