"""Host triangle-counting preprocessing of the library (degree relabelling and
strict lower triangle) against the oracle's, bit-exact, on graph families
with many degree ties. Host only: runs without a GPU."""
import numpy as np
import pytest

import oracle
import synth
import paper_1804_00695_amd as mls


@pytest.mark.parametrize("scale,ef,seed", [(6, 4, 1), (9, 8, 2), (11, 16, 3)])
def test_lower_matches_oracle(scale, ef, seed):
    G = synth.rmat_graph(scale, ef, seed=seed)
    perm, (n, lrp, lci) = mls.tc_lower(G)
    operm, L = oracle.tc_lower(G)
    assert np.array_equal(perm, operm)
    assert np.array_equal(lrp, L.row_ptr) and np.array_equal(lci, L.col_idx)


def test_lower_regular_graph_all_ties():
    n = 50
    G = synth.graph_from_edges(n, np.arange(n), (np.arange(n) + 1) % n)   # cycle: all degree 2
    perm, (_, lrp, lci) = mls.tc_lower(G)
    assert np.array_equal(perm, np.arange(n))
    operm, L = oracle.tc_lower(G)
    assert np.array_equal(lci, L.col_idx)


def test_lower_rejects_self_loop():
    G = synth.Csr(2, 2, np.array([0, 2, 3], np.int32), np.array([0, 1, 0], np.int32), None)
    with pytest.raises(mls.SpgemmError, match="BAD_CSR"):
        mls.tc_lower(G)
