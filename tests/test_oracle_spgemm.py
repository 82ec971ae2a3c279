"""Pins of the oracle's C = A*B against things other than itself.

* dense brute force (numpy) on tiny random pairs, rectangular, empty rows;
* the 13-point closed form of the squared 5-point Laplacian (64 x 64 grid);
* the closed form of the squared 27-point stencil, derived from the Kronecker
  structure A = 27 I - T (x) T (x) T, at small grids;
* the exact pattern counts nnz(C) = (5n-6)^3, madds = (9(n-2)+8)^3.
"""
import numpy as np
import pytest

import oracle
import synth

TOL = 1e-12


def dense_pattern(M):
    P = np.zeros((M.nrows, M.ncols), dtype=np.int64)
    rows = np.repeat(np.arange(M.nrows), np.diff(M.row_ptr.astype(np.int64)))
    P[rows, M.col_idx] = 1
    return P


def check_against_dense(A, B, C, cabs):
    Ad, Bd = synth.to_dense(A), synth.to_dense(B)
    pat = (dense_pattern(A) @ dense_pattern(B)) > 0
    assert np.array_equal(dense_pattern(C) > 0, pat)
    ref = Ad @ Bd
    scale = np.abs(Ad) @ np.abs(Bd)
    Cd = synth.to_dense(C)
    err = np.abs(Cd - ref)
    assert np.all(err <= TOL * scale + 1e-300), float((err - TOL * scale).max())
    # the oracle's own error scale equals sum |a||b| over the terms
    D = np.zeros_like(Cd)
    rows = np.repeat(np.arange(C.nrows), np.diff(C.row_ptr.astype(np.int64)))
    D[rows, C.col_idx] = cabs
    assert np.allclose(D, scale, rtol=1e-13, atol=0)


SHAPES = [(0, 0, 0), (1, 1, 1), (3, 4, 5), (7, 1, 9), (12, 12, 12), (40, 17, 33), (25, 40, 8), (5, 0, 6)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("density", [0.0, 0.1, 0.35, 1.0])
def test_dense_brute_force(shape, density):
    m, k, n = shape
    seed = 1000 * m + 10 * k + n + int(100 * density)
    A = synth.random_csr(m, k, density, seed, empty_rows=0.2)
    B = synth.random_csr(k, n, density, seed + 7, empty_rows=0.2)
    C, cabs = oracle.spgemm(A, B)
    assert oracle.csr_check(C) == 0
    check_against_dense(A, B, C, cabs)


@pytest.mark.parametrize("seed", range(6))
def test_integer_values_exact(seed):
    A = synth.random_csr(30, 20, 0.3, seed, integer=True)
    B = synth.random_csr(20, 25, 0.3, seed + 50, integer=True)
    C, _ = oracle.spgemm(A, B)
    ref = synth.to_dense(A) @ synth.to_dense(B)          # exact: small integers
    assert np.array_equal(synth.to_dense(C), ref)


def test_structural_zero_kept():
    A = synth.from_dense(np.array([[1.0, 1.0]]))
    B = synth.from_dense(np.array([[1.0], [-1.0]]))
    C, _ = oracle.spgemm(A, B)
    assert C.nnz == 1 and C.values[0] == 0.0


def test_row_subset_and_threads_match_full():
    A = synth.poisson_csr(300, 200, 5.0, 11)
    B = synth.poisson_csr(200, 250, 6.0, 12)
    C, cabs = oracle.spgemm(A, B)
    C4, cabs4 = oracle.spgemm(A, B, nthreads=4)
    assert np.array_equal(C.row_ptr, C4.row_ptr) and np.array_equal(C.col_idx, C4.col_idx)
    assert np.array_equal(C.values, C4.values) and np.array_equal(cabs, cabs4)
    rows = np.array([299, 0, 17, 17, 150])
    S, _ = oracle.spgemm(A, B, rows=rows)
    for t, i in enumerate(rows):
        ci, cv = C.row(int(i))
        si, sv = S.row(t)
        assert np.array_equal(ci, si) and np.array_equal(cv, sv)


def laplace13_expected(nx):
    """Square of the 5-point Dirichlet Laplacian from the grid geometry.

    (A^2)_ii = 16 + number of in-grid axis neighbours; distance-1 axis
    neighbours -8 (two paths a_ii a_ij + a_ij a_jj); diagonal neighbours +2
    (two paths through the two corner nodes); distance-2 axis neighbours +1.
    """
    N = nx * nx
    D = np.zeros((N, N))
    for y in range(nx):
        for x in range(nx):
            i = y * nx + x
            deg = sum(1 for dx, dy in [(1, 0), (-1, 0), (0, 1), (0, -1)]
                      if 0 <= x + dx < nx and 0 <= y + dy < nx)
            D[i, i] = 16 + deg
            for dx, dy, v in [(1, 0, -8), (-1, 0, -8), (0, 1, -8), (0, -1, -8),
                              (1, 1, 2), (1, -1, 2), (-1, 1, 2), (-1, -1, 2),
                              (2, 0, 1), (-2, 0, 1), (0, 2, 1), (0, -2, 1)]:
                if 0 <= x + dx < nx and 0 <= y + dy < nx:
                    D[i, (y + dy) * nx + (x + dx)] = v
    return D


def test_laplace2d_13pt_closed_form():
    A = synth.laplace2d_5pt(64)
    assert A.nnz == 20224
    C, _ = oracle.spgemm(A, A)
    assert C.nnz == 51972
    assert int(oracle.row_work(A, A).sum()) == 100104
    D = laplace13_expected(64)
    Cd = synth.to_dense(C)
    assert np.array_equal(Cd, D)                 # bit-exact: all integers
    assert np.array_equal(dense_pattern(C) > 0, D != 0)


def stencil27_square_expected(n):
    """(A^2) for A = 27 I - K, K = T (x) T (x) T with T = tridiag(1, 1, 1) (n x n).

    A^2 = 729 I - 54 K + (T^2) (x) (T^2) (x) (T^2); T^2 has 2 (ends) or 3 on
    the diagonal, 2 at offset +-1 and 1 at offset +-2.
    """
    T = np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    K = np.kron(np.kron(T, T), T)
    T2 = T @ T
    K2 = np.kron(np.kron(T2, T2), T2)
    return 729 * np.eye(n ** 3) - 54 * K + K2


@pytest.mark.parametrize("n", [2, 3, 4, 6, 7])
def test_stencil27_square_closed_form(n):
    A = synth.stencil27_3d(n, amp=0.0)
    assert A.nnz == (3 * n - 2) ** 3
    C, _ = oracle.spgemm(A, A)
    D = stencil27_square_expected(n)
    assert np.array_equal(synth.to_dense(C), D)
    assert C.nnz == (5 * n - 6) ** 3 if n >= 2 else True
    assert int(oracle.row_work(A, A).sum()) == (9 * (n - 2) + 8) ** 3


def test_stencil27_interior_diagonal_702():
    A = synth.stencil27_3d(6, amp=0.0)
    C, _ = oracle.spgemm(A, A)
    i = (3 * 6 + 3) * 6 + 3
    cols, vals = C.row(i)
    assert vals[list(cols).index(i)] == 702.0
    assert len(cols) == 125


def test_stencil27_perturbed_vs_dense():
    A = synth.stencil27_3d(5, amp=0.1, seed=2)
    C, cabs = oracle.spgemm(A, A)
    check_against_dense(A, A, C, cabs)


def test_csr_check_codes():
    A = synth.random_csr(6, 6, 0.5, 3)
    assert oracle.csr_check(A) == 0
    bad = synth.Csr(A.nrows, A.ncols, A.row_ptr.copy(), A.col_idx.copy(), A.values)
    bad.row_ptr[0] = 1
    assert oracle.csr_check(bad) == 1
    bad = synth.Csr(2, 3, np.array([0, 2, 1], np.int32), np.array([0, 1], np.int32), None)
    assert oracle.csr_check(bad) == 2
    bad = synth.Csr(1, 3, np.array([0, 1], np.int32), np.array([3], np.int32), None)
    assert oracle.csr_check(bad) == 3
    bad = synth.Csr(1, 3, np.array([0, 2], np.int32), np.array([1, 1], np.int32), None)
    assert oracle.csr_check(bad) == 4


def test_compress_definition():
    B = synth.poisson_csr(50, 300, 9.0, 4)
    rp, sets, masks = oracle.compress(B)
    for i in range(B.nrows):
        cols, _ = B.row(i)
        s = sets[rp[i]:rp[i + 1]]
        m = masks[rp[i]:rp[i + 1]]
        assert np.all(np.diff(s) > 0)
        expanded = sorted(int(si) * 32 + b for si, mi in zip(s, m) for b in range(32) if (int(mi) >> b) & 1)
        assert expanded == cols.tolist()
    assert int(sum(bin(int(x)).count("1") for x in masks)) == B.nnz


def test_row_work_dense():
    A = synth.random_csr(20, 15, 0.3, 9)
    B = synth.random_csr(15, 18, 0.4, 10)
    w = oracle.row_work(A, B)
    assert np.array_equal(w, (dense_pattern(A) @ dense_pattern(B)).sum(axis=1))
