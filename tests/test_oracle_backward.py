"""Pins of the oracle's adjoint of loss(A, B) = sum_ij W_ij (A*B)_ij.

* central finite differences through the oracle's forward product: the loss
  is linear in A.values and in B.values separately, so a step h = 1 is exact
  up to rounding;
* Euler's identity for a function homogeneous of degree 1 in each factor:
  <dA, A> = loss = <dB, B>;
* dense numpy adjoints (W B^T) o pat(A) and (A^T W) o pat(B).
"""
import numpy as np
import pytest

import oracle
import synth

TOL = 1e-10


def loss(A, B, W):
    C, _ = oracle.spgemm(A, B, with_abs=False)
    assert np.array_equal(C.col_idx, W.col_idx)
    return float(np.dot(C.values, W.values)), C


def setup(m, k, n, lam_a, lam_b, seed):
    A = synth.poisson_csr(m, k, lam_a, seed)
    B = synth.poisson_csr(k, n, lam_b, seed + 1)
    C, _ = oracle.spgemm(A, B, with_abs=False)
    W = synth.Csr(C.nrows, C.ncols, C.row_ptr, C.col_idx, synth.normal_values(C.nnz, seed + 2))
    return A, B, W


@pytest.mark.parametrize("seed", [8, 21])
def test_finite_differences_every_entry(seed):
    A, B, W = setup(40, 35, 45, 3.0, 3.0, seed)
    dA, dB, dAa, dBa = oracle.backward(A, B, W)
    for p in range(A.nnz):
        vp = A.values.copy(); vp[p] += 1.0
        vm = A.values.copy(); vm[p] -= 1.0
        lp, _ = loss(synth.Csr(A.nrows, A.ncols, A.row_ptr, A.col_idx, vp), B, W)
        lm, _ = loss(synth.Csr(A.nrows, A.ncols, A.row_ptr, A.col_idx, vm), B, W)
        fd = (lp - lm) / 2.0
        assert abs(fd - dA[p]) <= 1e-9 * (1.0 + np.abs(W.values).sum())
    for q in range(B.nnz):
        vp = B.values.copy(); vp[q] += 1.0
        vm = B.values.copy(); vm[q] -= 1.0
        lp, _ = loss(A, synth.Csr(B.nrows, B.ncols, B.row_ptr, B.col_idx, vp), W)
        lm, _ = loss(A, synth.Csr(B.nrows, B.ncols, B.row_ptr, B.col_idx, vm), W)
        fd = (lp - lm) / 2.0
        assert abs(fd - dB[q]) <= 1e-9 * (1.0 + np.abs(W.values).sum())


def test_euler_identity():
    A, B, W = setup(300, 250, 280, 6.0, 6.0, 30)
    dA, dB, _, _ = oracle.backward(A, B, W)
    L, _ = loss(A, B, W)
    scale = float(np.abs(W.values).sum() * (np.abs(A.values).max() * np.abs(B.values).max()) * 50)
    assert abs(np.dot(dA, A.values) - L) <= 1e-12 * scale
    assert abs(np.dot(dB, B.values) - L) <= 1e-12 * scale


@pytest.mark.parametrize("seed", [40, 41, 42])
def test_dense_adjoints(seed):
    A, B, W = setup(25, 30, 20, 4.0, 4.0, seed)
    dA, dB, dAa, dBa = oracle.backward(A, B, W)
    Ad, Bd, Wd = synth.to_dense(A), synth.to_dense(B), synth.to_dense(W)
    GA = Wd @ Bd.T
    GB = Ad.T @ Wd
    SA = np.abs(Wd) @ np.abs(Bd).T
    SB = np.abs(Ad).T @ np.abs(Wd)
    ar = np.repeat(np.arange(A.nrows), np.diff(A.row_ptr))
    br = np.repeat(np.arange(B.nrows), np.diff(B.row_ptr))
    assert np.all(np.abs(dA - GA[ar, A.col_idx]) <= TOL * SA[ar, A.col_idx] + 1e-300)
    assert np.all(np.abs(dB - GB[br, B.col_idx]) <= TOL * SB[br, B.col_idx] + 1e-300)
    assert np.allclose(dAa, SA[ar, A.col_idx], rtol=1e-13, atol=0)
    assert np.allclose(dBa, SB[br, B.col_idx], rtol=1e-13, atol=0)


def test_w_must_cover_pattern():
    A, B, W = setup(10, 10, 10, 3.0, 3.0, 50)
    if W.nnz == 0:
        pytest.skip("empty product")
    short = synth.Csr(W.nrows, W.ncols, np.zeros(W.nrows + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    with pytest.raises(ValueError):
        oracle.backward(A, B, short)
