"""Seeded stand-ins for the paper's four multigrid problem families (torch).

The paper's R x A and A x P products come from Laplace3D, BigStar2D, Brick3D
and Elasticity multigrid hierarchies with 7, 13, 27 and 81 entries per row of
A (Sec. 3.2); the matrices themselves are not available. These generators
build operators of the same structure classes on structured grids, with the
grid edge chosen so that A has a requested size in bytes (the paper scales A
from 1 GB up), plus a smoothed-aggregation prolongator P and R = P^T:

* ``laplace3d``     7-point stencil on an n^3 grid, one unknown per node.
* ``bigstar2d``     13-point stencil on an n^2 grid: the centre, the axis
                    neighbours at distance 1 and 2, and the four diagonal
                    neighbours.
* ``brick3d``       27-point stencil (the 3x3x3 box) on an n^3 grid.
* ``elasticity3d``  the 27-point box on an n^3 grid with 3 unknowns per node
                    coupled to all 3 unknowns of every neighbour (81 per row).

Values of A: diagonal ``points - 1 + 0.5`` and off-diagonals
``-(1 + ((31 r + 17 c) mod 201 - 100) / 1000)`` at row r, column c -- a
function of the position only, so the same matrix comes out on every device
and in any generation order, and sums of products round (bitwise comparisons
between two paths are meaningful).

Aggregation: 2 nodes per dimension per aggregate (ceil(n/2) per dimension;
an odd n leaves partial aggregates), unknown a of a node mapped to unknown a
of its aggregate. Smoothing: P = (I - (2/3) D^-1 L) P0 with L the
nearest-neighbour Laplacian of the grid (diagonal 2*dim, -1 on the 2*dim axis
neighbours), so P has 1/3 on its own aggregate plus 1/(3 dim) for each axis
neighbour in the same or in another aggregate: row x of P holds
(dim + #{axis neighbours of x in agg(x)}) / (3 dim) at agg(x) and
1 / (3 dim) at the aggregate of each axis neighbour outside it (at most one
per axis), so P has 1 + dim entries per row in the interior (delta of P = 4
in 3D, 3 in 2D, the paper's 3 to 4.5).

Everything is input preparation; none of the product's arithmetic is here.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Optional

import torch

from . import Csr

PROBLEMS = {
    # name: (grid dimensions, stencil kind, unknowns per node)
    "laplace3d": (3, "axis", 1),
    "bigstar2d": (2, "bigstar", 1),
    "brick3d": (3, "box", 1),
    "elasticity3d": (3, "box", 3),
}


@dataclass
class TCsr:
    """CSR matrix held in torch tensors (int32 indices, float64 values)."""
    nrows: int
    ncols: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    values: Optional[torch.Tensor]

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    def nbytes(self) -> int:
        """4 bytes per row pointer, 12 per entry (int32 index + fp64 value)."""
        return 4 * (self.nrows + 1) + 12 * self.nnz

    def to_csr(self) -> Csr:
        """Host numpy copy (for the oracle and for the CPU tests)."""
        v = None if self.values is None else self.values.cpu().numpy()
        return Csr(self.nrows, self.ncols, self.row_ptr.cpu().numpy(), self.col_idx.cpu().numpy(), v)


def stencil_offsets(kind: str, dim: int):
    """Node offsets of the stencil, sorted so that the flat offset ascends."""
    if kind == "axis":
        offs = [tuple(0 for _ in range(dim))]
        for d in range(dim):
            for s in (-1, 1):
                o = [0] * dim
                o[d] = s
                offs.append(tuple(o))
    elif kind == "box":
        offs = list(itertools.product((-1, 0, 1), repeat=dim))
    elif kind == "bigstar":
        if dim != 2:
            raise ValueError("bigstar is a 2D stencil")
        offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1), (-2, 0), (2, 0), (0, -2), (0, 2),
                (-1, -1), (-1, 1), (1, -1), (1, 1)]
    else:
        raise ValueError(kind)
    return sorted(offs)   # lexicographic on (slowest, ..., fastest)


def _coords(n: int, dim: int, device):
    idx = torch.arange(n ** dim, dtype=torch.int64, device=device)
    out = []
    for d in range(dim):
        stride = n ** (dim - 1 - d)
        out.append((idx // stride) % n)
    return idx, out


def _stencil_rows(n: int, dim: int, offs, dof: int, device):
    """Row pointer of the stencil matrix and, per offset, (valid nodes, rank)."""
    N = n ** dim
    idx, xs = _coords(n, dim, device)
    valid = []
    for off in offs:
        ok = torch.ones(N, dtype=torch.bool, device=device)
        for d, od in enumerate(off):
            c = xs[d] + od
            ok &= (c >= 0) & (c < n)
        valid.append(ok)
    count = torch.zeros(N, dtype=torch.int64, device=device)
    for ok in valid:
        count += ok
    row_len = (count * dof).repeat_interleave(dof)            # rows node-major, unknown-minor
    row_ptr = torch.zeros(N * dof + 1, dtype=torch.int64, device=device)
    torch.cumsum(row_len, 0, out=row_ptr[1:])
    return idx, valid, row_ptr


def operator(problem: str, n: int, device="cpu") -> TCsr:
    """The fine operator A of a problem on an n^dim grid."""
    dim, kind, dof = PROBLEMS[problem]
    offs = stencil_offsets(kind, dim)
    idx, valid, rp = _stencil_rows(n, dim, offs, dof, device)
    N = n ** dim
    nnz = int(rp[-1])
    if nnz >= 2 ** 31:
        raise ValueError(f"{problem} on n={n}: {nnz} entries do not fit int32 indices")
    col = torch.empty(nnz, dtype=torch.int32, device=device)
    rank = torch.zeros(N, dtype=torch.int64, device=device)   # valid offsets before the current one
    ar = torch.arange(dof, dtype=torch.int64, device=device)
    for off, ok in zip(offs, valid):
        flat = sum(od * n ** (dim - 1 - d) for d, od in enumerate(off))
        nodes = idx[ok]
        nbr = nodes + flat
        # rows (node, a): entries (nbr, b) at rank*dof + b
        rows = nodes[:, None] * dof + ar[None, :]                          # [v, a]
        base = rp[rows] + rank[nodes][:, None] * dof                       # [v, a]
        pos = base[:, :, None] + ar[None, None, :]                         # [v, a, b]
        cval = (nbr[:, None] * dof + ar[None, :])[:, None, :].expand_as(pos)
        col[pos.reshape(-1)] = cval.reshape(-1).to(torch.int32)
        rank[nodes] += 1
    rows = torch.repeat_interleave(torch.arange(N * dof, dtype=torch.int64, device=device), torch.diff(rp))
    c64 = col.to(torch.int64)
    vals = -(1.0 + ((31 * rows + 17 * c64) % 201 - 100).to(torch.float64) / 1000.0)
    diag = rows == c64
    vals[diag] = float(len(offs) * dof - 1) + 0.5
    return TCsr(N * dof, N * dof, rp.to(torch.int32), col, vals)


def prolongator(problem: str, n: int, device="cpu") -> TCsr:
    """Smoothed-aggregation prolongator P (fine unknowns x coarse unknowns)."""
    dim, _, dof = PROBLEMS[problem]
    nc = (n + 1) // 2
    N, Nc = n ** dim, nc ** dim
    idx, xs = _coords(n, dim, device)
    agg = torch.zeros(N, dtype=torch.int64, device=device)
    for d in range(dim):
        agg = agg * nc + xs[d] // 2
    # candidates in ascending coarse order: -axis (slowest first), own, +axis (fastest first)
    same = torch.zeros(N, dtype=torch.int64, device=device)
    minus, plus = [], []
    for d in range(dim):
        x = xs[d]
        cstride = nc ** (dim - 1 - d)
        lo_in = (x >= 1) & (x % 2 == 1)          # x-1 inside the grid and in the same aggregate
        hi_in = (x + 1 < n) & (x % 2 == 0)       # x+1 inside the grid and in the same aggregate
        same += lo_in.to(torch.int64) + hi_in.to(torch.int64)
        minus.append(((x >= 1) & (x % 2 == 0), -cstride))      # x-1 in the previous aggregate
        plus.append(((x + 1 < n) & (x % 2 == 1), cstride))     # x+1 in the next aggregate
    cands = minus + [(torch.ones(N, dtype=torch.bool, device=device), 0)] + plus[::-1]
    # plus[::-1] lists the fastest axis first, whose coarse offset is the smallest positive one
    cnt = torch.zeros(N, dtype=torch.int64, device=device)
    for ok, _ in cands:
        cnt += ok
    row_len = cnt.repeat_interleave(dof)
    rp = torch.zeros(N * dof + 1, dtype=torch.int64, device=device)
    torch.cumsum(row_len, 0, out=rp[1:])
    nnz = int(rp[-1])
    col = torch.empty(nnz, dtype=torch.int32, device=device)
    val = torch.empty(nnz, dtype=torch.float64, device=device)
    rank = torch.zeros(N, dtype=torch.int64, device=device)
    ar = torch.arange(dof, dtype=torch.int64, device=device)
    w_other = 1.0 / (3 * dim)
    for ok, coff in cands:
        nodes = idx[ok]
        rows = nodes[:, None] * dof + ar[None, :]
        pos = rp[rows] + rank[nodes][:, None]
        g = agg[nodes] + coff
        col[pos.reshape(-1)] = (g[:, None] * dof + ar[None, :]).reshape(-1).to(torch.int32)
        if coff == 0:
            w = (dim + same[nodes]).to(torch.float64) / (3 * dim)
            val[pos.reshape(-1)] = w[:, None].expand(-1, dof).reshape(-1)
        else:
            val[pos.reshape(-1)] = w_other
        rank[nodes] += 1
    return TCsr(N * dof, Nc * dof, rp.to(torch.int32), col, val)


def transpose(M: TCsr) -> TCsr:
    """Explicit transpose (R = P^T), columns of each row ascending."""
    dev = M.col_idx.device
    c = M.col_idx.to(torch.int64)
    order = torch.argsort(c, stable=True)            # entries are in ascending row order already
    rows = torch.repeat_interleave(torch.arange(M.nrows, dtype=torch.int64, device=dev),
                                   torch.diff(M.row_ptr.to(torch.int64)))
    cnt = torch.bincount(c, minlength=M.ncols)
    rp = torch.zeros(M.ncols + 1, dtype=torch.int64, device=dev)
    torch.cumsum(cnt, 0, out=rp[1:])
    vals = None if M.values is None else M.values[order]
    return TCsr(M.ncols, M.nrows, rp.to(torch.int32), rows[order].to(torch.int32), vals)


def bytes_per_row(problem: str) -> float:
    dim, kind, dof = PROBLEMS[problem]
    return 4 + 12 * len(stencil_offsets(kind, dim)) * dof


def grid_for_bytes(problem: str, nbytes: float) -> int:
    """Even grid edge n for which A takes about ``nbytes`` (interior rows)."""
    dim, _, dof = PROBLEMS[problem]
    rows = nbytes / bytes_per_row(problem)
    n = int(round((rows / dof) ** (1.0 / dim)))
    return max(6, n + (n % 2))


def problem(name: str, n: int, device="cpu"):
    """(A, P, R) of one problem on an n^dim grid."""
    A = operator(name, n, device)
    P = prolongator(name, n, device)
    return A, P, transpose(P)


def random_rhs(nrows: int, ncols: int, delta: int, seed: int, device="cpu") -> TCsr:
    """Right-hand side of the density study (Table "expdensity"): every row
    holds exactly ``delta`` distinct uniform columns (delta <= ncols), values
    N(0, 1); torch's generator on ``device`` seeded with ``seed`` (the same
    seed gives the same matrix on the same kind of device)."""
    if delta > ncols:
        raise ValueError("delta exceeds the number of columns")
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    cols = torch.randint(0, ncols, (nrows, delta), generator=g, device=device, dtype=torch.int64)
    while True:
        cols, _ = torch.sort(cols, dim=1)
        dup = torch.zeros_like(cols, dtype=torch.bool)
        if delta > 1:
            dup[:, 1:] = cols[:, 1:] == cols[:, :-1]
        nd = int(dup.sum())
        if nd == 0:
            break
        cols[dup] = torch.randint(0, ncols, (nd,), generator=g, device=device, dtype=torch.int64)
    vals = torch.randn(nrows * delta, generator=g, device=device, dtype=torch.float64)
    rp = torch.arange(nrows + 1, dtype=torch.int64, device=device) * delta
    return TCsr(nrows, ncols, rp.to(torch.int32), cols.reshape(-1).to(torch.int32), vals)
