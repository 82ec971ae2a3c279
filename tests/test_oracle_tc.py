"""Pins of the oracle's triangle count (masked (L*L) o L, summed).

Closed forms (complete, cycle, wheel, bipartite graphs), trace(A^3)/6 from a
dense cube, and a second, different algorithm (merge intersection of sorted
adjacency lists over the edges of the original labelling).
"""
from math import comb

import numpy as np
import pytest

import oracle
import synth


def graph(n, edges):
    e = np.array(edges, dtype=np.int64).reshape(-1, 2)
    return synth.graph_from_edges(n, e[:, 0], e[:, 1])


def complete(n):
    return graph(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def cycle(n):
    return graph(n, [(i, (i + 1) % n) for i in range(n)])


def wheel(n):
    """Hub n joined to every vertex of the cycle 0..n-1."""
    return graph(n + 1, [(i, (i + 1) % n) for i in range(n)] + [(n, i) for i in range(n)])


def bipartite(m, n):
    return graph(m + n, [(i, m + j) for i in range(m) for j in range(n)])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 10, 23])
def test_complete(n):
    assert oracle.triangle_count(complete(n))[0] == comb(n, 3)


@pytest.mark.parametrize("n", [3, 4, 5, 9, 50])
def test_cycle(n):
    assert oracle.triangle_count(cycle(n))[0] == (1 if n == 3 else 0)


@pytest.mark.parametrize("n", [4, 5, 8, 31])
def test_wheel(n):
    assert oracle.triangle_count(wheel(n))[0] == n


@pytest.mark.parametrize("mn", [(1, 1), (3, 4), (10, 7)])
def test_bipartite(mn):
    assert oracle.triangle_count(bipartite(*mn))[0] == 0


def test_empty_graph():
    G = synth.Csr(5, 5, np.zeros(6, np.int32), np.zeros(0, np.int32), None)
    total, counts, perm, L = oracle.triangle_count(G)
    assert total == 0 and L.nnz == 0 and sorted(perm.tolist()) == list(range(5))


@pytest.mark.parametrize("seed", range(5))
def test_trace_cube(seed):
    g = synth.rng(seed)
    n = 40
    M = np.triu(g.random((n, n)) < 0.2, 1)
    i, j = np.nonzero(M)
    G = synth.graph_from_edges(n, i, j)
    Ad = synth.to_dense(G)
    assert oracle.triangle_count(G)[0] == int(round(np.trace(Ad @ Ad @ Ad))) // 6


def merge_intersection_count(G):
    """Second algorithm: for each edge u < v, |N(u) intersect N(v) restricted to w > v|."""
    adj = [G.row(i)[0] for i in range(G.nrows)]
    total = 0
    for u in range(G.nrows):
        for v in adj[u]:
            if v <= u:
                continue
            a, b = adj[u], adj[v]
            x = y = 0
            while x < len(a) and y < len(b):
                if a[x] < b[y]:
                    x += 1
                elif a[x] > b[y]:
                    y += 1
                else:
                    if a[x] > v:
                        total += 1
                    x += 1
                    y += 1
    return total


def test_rmat_vs_merge_intersection():
    G = synth.rmat_graph(9, 8, seed=5)
    assert oracle.triangle_count(G)[0] == merge_intersection_count(G)


def test_lower_triangle_properties():
    G = synth.rmat_graph(8, 8, seed=6)
    perm, L = oracle.tc_lower(G)
    deg = np.diff(G.row_ptr)
    d = deg[perm]
    # descending degree, ties by ascending original id
    assert np.all((d[:-1] > d[1:]) | ((d[:-1] == d[1:]) & (perm[:-1] < perm[1:])))
    assert L.nnz * 2 == G.nnz
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    rows = np.repeat(np.arange(L.nrows), np.diff(L.row_ptr))
    assert np.all(L.col_idx < rows)
    got = set(zip(perm[rows].tolist(), perm[L.col_idx].tolist()))
    grow = np.repeat(np.arange(G.nrows), np.diff(G.row_ptr))
    want = {(int(a), int(b)) for a, b in zip(grow, G.col_idx) if inv[a] > inv[b]}
    assert got == want
    assert oracle.csr_check(L) == 0


def test_row_counts_sum_and_subset():
    G = synth.rmat_graph(8, 8, seed=7)
    total, counts, perm, L = oracle.triangle_count(G, nthreads=3)
    assert counts.sum() == total
    rows = np.array([5, 0, 255, 5])
    sub, st = oracle.tc_count(L, rows=rows)
    assert np.array_equal(sub, counts[rows]) and st == counts[rows].sum()
