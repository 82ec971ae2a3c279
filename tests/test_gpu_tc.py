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
