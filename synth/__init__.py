"""Seeded synthetic inputs for the SpGEMM hot path.

This module only builds input matrices and random draws. It holds none of the
arithmetic of the method (no products, no accumulation, no triangle
counting): the oracle under ``oracle/`` and the HIP library under
``paper_1804_00695_amd/`` both take their inputs from here and from nowhere
else, so that neither has to import the other.

Every generator returns CSR with int32 row pointers and column indices,
columns strictly increasing inside each row, and float64 values (or no
values for pattern-only matrices). Random draws use numpy's PCG64 with an
explicit seed, so a (generator, arguments, seed) triple names one matrix.

Workloads (the paper's multigrid matrices and graphs are not available; these
seeded stand-ins have the same structure classes):

* ``laplace2d_5pt``     2D 5-point Dirichlet Laplacian (4 / -1).
* ``stencil27_3d``      3D 27-point stencil, diagonal 26, off-diagonals
                        -(1 + U(-amp, amp)), one draw per stored off-diagonal
                        entry in CSR order.
* ``laplace3d_7pt``     3D 7-point Dirichlet Laplacian (6 / -1), the fine
                        operator of the multigrid Galerkin products.
* ``amg_prolongator``   smoothed aggregation prolongator
                        P = (I - 2/3 D^-1 A) P0 with 2x2x2 aggregates,
                        written out in closed form (no product is formed).
* ``rmat_graph``        R-MAT graph, symmetrised, no self loops, no
                        duplicate edges (pattern only).
* ``poisson_csr``       rows with Poisson(lam) distinct uniform columns and
                        N(0, 1) values.
* ``random_csr``        tiny Bernoulli patterns for brute-force tests.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

__all__ = [
    "Csr", "laplace2d_5pt", "stencil27_3d", "laplace3d_7pt", "amg_prolongator",
    "amg_instance", "amg_batch_sizes", "transpose", "rmat_edges", "rmat_graph",
    "poisson_csr", "normal_values", "random_csr", "from_dense", "to_dense",
    "graph_from_edges", "rng",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Csr:
    """Compressed sparse row matrix (host arrays)."""
    nrows: int
    ncols: int
    row_ptr: np.ndarray            # int32 [nrows + 1]
    col_idx: np.ndarray            # int32 [nnz]
    values: Optional[np.ndarray]   # float64 [nnz] or None (pattern only)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row(self, i: int):
        s, e = int(self.row_ptr[i]), int(self.row_ptr[i + 1])
        v = None if self.values is None else self.values[s:e]
        return self.col_idx[s:e], v

    def nbytes(self) -> int:
        """4 bytes per row pointer, 4 per column index, 8 per value."""
        b = 4 * (self.nrows + 1) + 4 * self.nnz
        if self.values is not None:
            b += 8 * self.nnz
        return b


def _csr_from_sorted_coo(nrows, ncols, rows, cols, vals=None) -> Csr:
    counts = np.bincount(rows, minlength=nrows)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    if rp[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return Csr(nrows, ncols, rp.astype(np.int32), np.ascontiguousarray(cols, dtype=np.int32),
               None if vals is None else np.ascontiguousarray(vals, dtype=np.float64))


def _stencil(dims, offsets):
    """Rows of a structured-grid stencil, columns ascending.

    ``dims`` is the grid shape (slowest first); ``offsets`` is a list of
    integer offset tuples sorted so that the flat column offset increases.
    Returns (row_ptr int64, col_idx int32, which-offset int8) in CSR order.
    """
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    coords = np.indices(dims).reshape(len(dims), -1)
    strides = [int(np.prod(dims[d + 1:])) for d in range(len(dims))]
    valid = np.zeros((len(offsets), n), dtype=bool)
    for o, off in enumerate(offsets):
        ok = np.ones(n, dtype=bool)
        for d, od in enumerate(off):
            c = coords[d] + od
            ok &= (c >= 0) & (c < dims[d])
        valid[o] = ok
    counts = valid.sum(axis=0)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    nnz = int(rp[-1])
    col = np.empty(nnz, dtype=np.int32)
    which = np.empty(nnz, dtype=np.int8)
    cursor = rp[:-1].copy()
    rows = np.arange(n, dtype=np.int64)
    for o, off in enumerate(offsets):
        flat = sum(od * s for od, s in zip(off, strides))
        r = rows[valid[o]]
        pos = cursor[r]
        col[pos] = (r + flat).astype(np.int32)
        which[pos] = o
        cursor[r] += 1
    return rp, col, which


def _sorted_offsets(ndim, radius):
    rngs = [range(-radius, radius + 1)] * ndim
    offs = [tuple(t) for t in np.array(np.meshgrid(*rngs, indexing="ij")).reshape(ndim, -1).T]
    return sorted(offs)  # lexicographic on (slowest, ..., fastest) == ascending flat offset


def laplace2d_5pt(nx: int, ny: Optional[int] = None) -> Csr:
    """5-point Dirichlet Laplacian on an ny x nx grid, row = y*nx + x."""
    ny = nx if ny is None else ny
    offs = [(-1, 0), (0, -1), (0, 0), (0, 1), (1, 0)]
    rp, col, which = _stencil((ny, nx), offs)
    vals = np.where(which == 2, 4.0, -1.0)
    return Csr(ny * nx, ny * nx, rp.astype(np.int32), col, vals)


def laplace3d_7pt(n: int) -> Csr:
    """7-point Dirichlet Laplacian on an n^3 grid, row = (z*n + y)*n + x."""
    offs = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    rp, col, which = _stencil((n, n, n), offs)
    vals = np.where(which == 3, 6.0, -1.0)
    return Csr(n ** 3, n ** 3, rp.astype(np.int32), col, vals)


def stencil27_3d(n: int, amp: float = 0.1, seed: int = 2) -> Csr:
    """27-point stencil on an n^3 grid: diagonal 26, off-diagonal -(1+U(-amp, amp)).

    One uniform draw per stored off-diagonal entry, in CSR order, from
    PCG64(seed). With amp == 0 every off-diagonal value is exactly -1.
    """
    offs = _sorted_offsets(3, 1)
    rp, col, which = _stencil((n, n, n), offs)
    diag = which == 13
    vals = np.full(col.shape[0], 26.0)
    noff = int((~diag).sum())
    if amp == 0.0:
        vals[~diag] = -1.0
    else:
        u = rng(seed).uniform(-amp, amp, noff)
        vals[~diag] = -(1.0 + u)
    return Csr(n ** 3, n ** 3, rp.astype(np.int32), col, vals)


def amg_prolongator(n: int) -> Csr:
    """Smoothed-aggregation prolongator for the 7-point Laplacian on n^3.

    P0 maps fine node (x, y, z) to aggregate (x//2, y//2, z//2) with value 1
    (ceil(n/2) aggregates per dimension, so odd n leaves partial aggregates).
    S = I - (2/3) D^-1 A with D = diag(A) = 6, so S has 1/3 on the diagonal
    and 1/9 on each existing axis neighbour. P = S P0 therefore has, in row x,
    (3*[g == agg(x)] + #{neighbours y of x with agg(y) == g}) / 9 at column g:
    the integer weight is summed exactly and divided once.
    """
    nc = (n + 1) // 2
    N = n ** 3
    z, y, x = np.indices((n, n, n)).reshape(3, -1)
    fine = np.arange(N, dtype=np.int64)

    def agg(zz, yy, xx):
        return ((zz // 2) * nc + (yy // 2)) * nc + (xx // 2)

    rows = [fine]
    aggs = [agg(z, y, x)]
    wts = [np.full(N, 3, dtype=np.int64)]
    for dz, dy, dx in [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]:
        zz, yy, xx = z + dz, y + dy, x + dx
        ok = (zz >= 0) & (zz < n) & (yy >= 0) & (yy < n) & (xx >= 0) & (xx < n)
        rows.append(fine[ok])
        aggs.append(agg(zz[ok], yy[ok], xx[ok]))
        wts.append(np.ones(int(ok.sum()), dtype=np.int64))
    r = np.concatenate(rows)
    g = np.concatenate(aggs)
    w = np.concatenate(wts)
    ncoarse = nc ** 3
    key = r * ncoarse + g
    ukey, inv = np.unique(key, return_inverse=True)
    wsum = np.bincount(inv, weights=w).astype(np.int64)
    vals = wsum.astype(np.float64) / 9.0
    return _csr_from_sorted_coo(N, ncoarse, ukey // ncoarse, (ukey % ncoarse).astype(np.int32), vals)


def transpose(M: Csr) -> Csr:
    """Explicit CSR transpose (input preparation: R = P^T)."""
    rows = np.repeat(np.arange(M.nrows, dtype=np.int64), np.diff(M.row_ptr.astype(np.int64)))
    order = np.lexsort((rows, M.col_idx))
    vals = None if M.values is None else M.values[order]
    return _csr_from_sorted_coo(M.ncols, M.nrows, M.col_idx[order].astype(np.int64),
                                rows[order].astype(np.int32), vals)


def amg_batch_sizes(count: int = 256, lo: int = 16, hi: int = 64, seed: int = 4) -> np.ndarray:
    """Grid sizes n ~ U{lo..hi} for a batch of Galerkin products."""
    return rng(seed).integers(lo, hi + 1, count)


def amg_instance(n: int):
    """(A, P, R) for one Galerkin product Ac = R (A P), R = P^T."""
    A = laplace3d_7pt(n)
    P = amg_prolongator(n)
    return A, P, transpose(P)


def rmat_edges(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: int = 3, chunk: int = 1 << 22):
    """Plain recursive-quadrant R-MAT sampling: edge_factor * 2^scale samples.

    At each of ``scale`` levels one uniform draw picks quadrant (0,0) with
    probability a, (0,1) with b, (1,0) with c, (1,1) with d = 1-a-b-c.
    No noise, no vertex permutation. Returns directed (src, dst) int64.
    """
    m = edge_factor << scale
    g = rng(seed)
    src = np.empty(m, dtype=np.int64)
    dst = np.empty(m, dtype=np.int64)
    t1, t2, t3 = a, a + b, a + b + c
    for s in range(0, m, chunk):
        e = min(m, s + chunk)
        u = np.zeros(e - s, dtype=np.int64)
        v = np.zeros(e - s, dtype=np.int64)
        for _ in range(scale):
            r = g.random(e - s)
            ubit = r >= t2                      # quadrants (1,0) and (1,1)
            vbit = ((r >= t1) & (r < t2)) | (r >= t3)   # quadrants (0,1) and (1,1)
            u = (u << 1) | ubit
            v = (v << 1) | vbit
        src[s:e] = u
        dst[s:e] = v
    return src, dst


def graph_from_edges(nverts: int, src: np.ndarray, dst: np.ndarray) -> Csr:
    """Symmetric adjacency pattern: self loops dropped, both directions, deduplicated."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = np.unique(np.concatenate([src * nverts + dst, dst * nverts + src]))
    return _csr_from_sorted_coo(nverts, nverts, key // nverts, (key % nverts).astype(np.int32), None)


def rmat_graph(scale: int, edge_factor: int = 16, seed: int = 3, **kw) -> Csr:
    src, dst = rmat_edges(scale, edge_factor, seed=seed, **kw)
    return graph_from_edges(1 << scale, src, dst)


def poisson_csr(nrows: int, ncols: int, lam: float, seed: int) -> Csr:
    """Row i holds k_i ~ Poisson(lam) distinct uniform columns; values N(0,1) in CSR order."""
    g = rng(seed)
    k = g.poisson(lam, nrows).astype(np.int64)
    k = np.minimum(k, ncols)
    rows = np.repeat(np.arange(nrows, dtype=np.int64), k)
    cols = g.integers(0, ncols, rows.shape[0], dtype=np.int64)
    while True:
        order = np.lexsort((cols, rows))
        rows, cols = rows[order], cols[order]
        dup = np.zeros(rows.shape[0], dtype=bool)
        if rows.shape[0] > 1:
            dup[1:] = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        nd = int(dup.sum())
        if nd == 0:
            break
        cols[dup] = g.integers(0, ncols, nd, dtype=np.int64)
    vals = g.standard_normal(rows.shape[0])
    return _csr_from_sorted_coo(nrows, ncols, rows, cols.astype(np.int32), vals)


def normal_values(count: int, seed: int) -> np.ndarray:
    """``count`` N(0,1) draws (e.g. the loss weights W on the pattern of C)."""
    return rng(seed).standard_normal(int(count))


def random_csr(m: int, n: int, density: float, seed: int, integer: bool = False,
               empty_rows: float = 0.0) -> Csr:
    """Tiny Bernoulli(density) pattern; values N(0,1) or integers in [-3, 3]\\{0}."""
    g = rng(seed)
    mask = g.random((m, n)) < density
    if empty_rows > 0.0 and m > 0:
        mask[g.random(m) < empty_rows, :] = False
    if integer:
        vals = g.integers(1, 4, (m, n)) * np.where(g.random((m, n)) < 0.5, -1, 1)
        vals = vals.astype(np.float64)
    else:
        vals = g.standard_normal((m, n))
    return from_dense(np.where(mask, vals, 0.0), mask)


def from_dense(D: np.ndarray, mask: Optional[np.ndarray] = None) -> Csr:
    """CSR holding D's entries where ``mask`` (default D != 0) is set, zeros included."""
    D = np.asarray(D, dtype=np.float64)
    m, n = D.shape
    if mask is None:
        mask = D != 0
    r, c = np.nonzero(mask)
    return _csr_from_sorted_coo(m, n, r.astype(np.int64), c.astype(np.int32), D[r, c])


def to_dense(M: Csr) -> np.ndarray:
    D = np.zeros((M.nrows, M.ncols))
    rows = np.repeat(np.arange(M.nrows), np.diff(M.row_ptr.astype(np.int64)))
    D[rows, M.col_idx] = 1.0 if M.values is None else M.values
    return D
