"""Seeded synthetic inputs: CSR test matrices and dense operands.

This module builds inputs only.  It computes no sparse product, solve or
gradient, so both the HIP path and the FP64 CPU oracle can be fed from it
without sharing any of the method's arithmetic.

Every matrix is returned as a ``Csr`` of NumPy arrays: ``rowptr`` and
``colind`` are int32 (column indices ascending and unique within each row),
``vals`` is float64.  Callers cast values to float32 where a run needs it;
the float32 cast of an exactly representable stencil is exact.

Matrices follow the paper's test problems:
* the 1D finite-difference Poisson matrix A_N (tridiagonal 2/-1), Section 4,
  Eq. (mat_1d_fd);
* its 2D Kronecker form A_Nx (x) I_Ny + I_Nx (x) A_Ny, Section 4,
  Eq. (mat_2d_fd), and the 3D analogue with three Kronecker terms;
* the 9x3 aggregation example of Fig. 2 (Section 3) generalised to
  P[i, floor(i/a)] = 1.
Anisotropic diffusion and random geometric-graph Laplacians are not in the
paper; their recipes are stated in the functions below.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Csr:
    nrows: int
    ncols: int
    rowptr: np.ndarray  # int32 [nrows+1]
    colind: np.ndarray  # int32 [nnz]
    vals: np.ndarray    # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def todense(self) -> np.ndarray:
        d = np.zeros((self.nrows, self.ncols), dtype=self.vals.dtype)
        rows = np.repeat(np.arange(self.nrows), np.diff(self.rowptr))
        d[rows, self.colind] = self.vals
        return d

    def row_of_entry(self) -> np.ndarray:
        return np.repeat(np.arange(self.nrows, dtype=np.int32),
                         np.diff(self.rowptr)).astype(np.int32)

    def astype(self, dt) -> "Csr":
        return Csr(self.nrows, self.ncols, self.rowptr, self.colind,
                   self.vals.astype(dt))


def _from_coo(nrows: int, ncols: int, rows: np.ndarray, cols: np.ndarray,
              vals: np.ndarray) -> Csr:
    """Sort COO triplets into CSR (rows, then columns ascending).

    Triplets must already be unique; this only orders them."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], np.asarray(vals, np.float64)[order]
    counts = np.bincount(rows, minlength=nrows)
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    assert rowptr[-1] < 2**31, "int32 CSR index space exceeded"
    return Csr(nrows, ncols, rowptr.astype(np.int32), cols.astype(np.int32),
               vals.astype(np.float64))


def _stencil(shape, offsets, weights) -> Csr:
    """Constant-coefficient stencil on a grid with homogeneous Dirichlet
    boundary nodes eliminated (neighbours outside the grid are dropped).

    ``shape`` lists grid extents, slowest index first; a node's linear index
    is the row-major index over ``shape``.  ``offsets`` are per-axis integer
    displacements, ``weights`` their coefficients."""
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64)
    coords = np.unravel_index(idx, shape)
    rows_l, cols_l, vals_l = [], [], []
    for off, w in zip(offsets, weights):
        ok = np.ones(n, dtype=bool)
        nb = []
        for ax, d in enumerate(off):
            c = coords[ax] + d
            ok &= (c >= 0) & (c < shape[ax])
            nb.append(c)
        nbi = np.ravel_multi_index(tuple(np.where(ok, c, 0) for c in nb), shape)
        rows_l.append(idx[ok])
        cols_l.append(nbi[ok])
        vals_l.append(np.full(int(ok.sum()), float(w)))
    return _from_coo(n, n, np.concatenate(rows_l), np.concatenate(cols_l),
                     np.concatenate(vals_l))


def poisson1d(n: int) -> Csr:
    """A_N: 2 on the diagonal, -1 on both off-diagonals (Eq. mat_1d_fd)."""
    return _stencil((n,), [(-1,), (0,), (1,)], [-1.0, 2.0, -1.0])


def poisson2d(nx: int, ny: int) -> Csr:
    """A_{Nx x Ny} = A_Nx (x) I_Ny + I_Nx (x) A_Ny (Eq. mat_2d_fd).

    In the Kronecker form the row index is ix*Ny + iy, so iy is the fast
    index; the 5-point stencil has 4 on the diagonal and -1 to each grid
    neighbour."""
    return _stencil((nx, ny), [(-1, 0), (0, -1), (0, 0), (0, 1), (1, 0)],
                    [-1.0, -1.0, 4.0, -1.0, -1.0])


def poisson3d(n: int) -> Csr:
    """Three-term Kronecker analogue of Eq. mat_2d_fd on an n^3 grid:
    7-point stencil, 6 on the diagonal, -1 per neighbour, last index fastest."""
    offs = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1),
            (0, 1, 0), (1, 0, 0)]
    w = [-1.0, -1.0, -1.0, 6.0, -1.0, -1.0, -1.0]
    return _stencil((n, n, n), offs, w)


def aggregation(n: int, agg: int = 8) -> Csr:
    """Prolongator with one unit entry per row: P[i, floor(i/agg)] = 1."""
    ncols = (n + agg - 1) // agg
    rows = np.arange(n, dtype=np.int64)
    return _from_coo(n, ncols, rows, rows // agg, np.ones(n))


def fig2_pair() -> tuple[Csr, Csr]:
    """The operands drawn in Fig. 2 (Section 3): the 9x9 5-point pattern of a
    3x3 grid times a 9x3 aggregation pattern with aggregates {1,2,4},
    {3,5,6}, {7,8,9} (1-based).  Values: Poisson stencil for A, ones for B."""
    a = poisson2d(3, 3)
    agg_of = np.array([0, 0, 1, 0, 1, 1, 2, 2, 2])
    b = _from_coo(9, 3, np.arange(9), agg_of, np.ones(9))
    return a, b


def anisotropic_q1(n: int, eps: float, theta: float) -> Csr:
    """Bilinear (Q1) finite elements for -div(K grad u) on an n x n interior
    grid, Dirichlet nodes eliminated, x fastest (index iy*n + ix).

    K = R(theta) diag(1, eps) R(theta)^T, so a = cos^2 + eps sin^2,
    c = sin^2 + eps cos^2, b = (1 - eps) cos sin.  The stencil is the tensor
    product of the 1D stiffness [-1 2 -1] and mass [1 4 1]/6 for the a and c
    terms, plus the cross term on the diagonal neighbours:
      centre 4(a+c)/3; E/W -2a/3 + c/3; N/S a/3 - 2c/3;
      NE/SW -(a+c)/6 - b/2; NW/SE -(a+c)/6 + b/2.
    """
    cs, sn = np.cos(theta), np.sin(theta)
    a = cs * cs + eps * sn * sn
    c = sn * sn + eps * cs * cs
    b = (1.0 - eps) * cs * sn
    offs = [(0, 0), (0, 1), (0, -1), (1, 0), (-1, 0), (1, 1), (-1, -1),
            (1, -1), (-1, 1)]  # (dy, dx)
    w = [4 * (a + c) / 3, -2 * a / 3 + c / 3, -2 * a / 3 + c / 3,
         a / 3 - 2 * c / 3, a / 3 - 2 * c / 3,
         -(a + c) / 6 - b / 2, -(a + c) / 6 - b / 2,
         -(a + c) / 6 + b / 2, -(a + c) / 6 + b / 2]
    return _stencil((n, n), offs, w)


def geometric_graph_laplacian(block: int, shift: float = 1e-2,
                              n_range=(1024, 65536), k_range=(6, 14)) -> Csr:
    """Random geometric-graph Laplacian D - W + shift*I for one block of the
    batched workload.

    rng = default_rng([3, block]); n ~ U{n_range}, k ~ U{k_range};
    points ~ U[0,1)^2; exact k nearest neighbours, union-symmetrised,
    unit weights."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng([3, block])
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    k = int(rng.integers(k_range[0], k_range[1] + 1))
    pts = rng.random((n, 2))
    _, nbr = cKDTree(pts).query(pts, k=k + 1)
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    dst = nbr[:, 1:].reshape(-1).astype(np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = np.unique(np.concatenate([src * n + dst, dst * n + src]))
    r, c = key // n, key % n
    deg = np.bincount(r, minlength=n).astype(np.float64)
    rows = np.concatenate([r, np.arange(n)])
    cols = np.concatenate([c, np.arange(n)])
    vals = np.concatenate([-np.ones(len(r)), deg + shift])
    return _from_coo(n, n, rows, cols, vals)


def geometric_graph(n: int, k: int, seed) -> Csr:
    """Adjacency of a random geometric graph: points ~ U[0,1)^2 from
    default_rng(seed), exact k nearest neighbours, union-symmetrised, unit
    weights, no self loops (k = 4 gives about 5 incident edges per node)."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    _, nbr = cKDTree(pts).query(pts, k=k + 1)
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    dst = nbr[:, 1:].reshape(-1).astype(np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = np.unique(np.concatenate([src * n + dst, dst * n + src]))
    g = _from_coo(n, n, key // n, key % n, np.ones(len(key)))
    g.points = pts
    return g


def node_classes(points: np.ndarray, nclass: int, seed) -> np.ndarray:
    """Class of each point: its nearest of nclass centres ~ U[0,1)^2 drawn
    from default_rng(seed) (spatially coherent labels on a geometric graph)."""
    from scipy.spatial import cKDTree

    centres = np.random.default_rng(seed).random((nclass, 2))
    return cKDTree(centres).query(points, k=1)[1].astype(np.int64)


def block_diag(blocks: list[Csr]) -> tuple[Csr, np.ndarray]:
    """Concatenate square CSR blocks block-diagonally.

    Returns the combined matrix and block_rowptr[nb+1] (first row of each
    block)."""
    offs = np.zeros(len(blocks) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([b.nrows for b in blocks])
    noffs = np.zeros(len(blocks) + 1, dtype=np.int64)
    noffs[1:] = np.cumsum([b.nnz for b in blocks])
    assert noffs[-1] < 2**31 and offs[-1] < 2**31
    rowptr = np.concatenate([[0]] + [b.rowptr[1:].astype(np.int64) + noffs[i]
                                     for i, b in enumerate(blocks)])
    colind = np.concatenate([b.colind.astype(np.int64) + offs[i]
                             for i, b in enumerate(blocks)])
    vals = np.concatenate([b.vals for b in blocks])
    n = int(offs[-1])
    return (Csr(n, n, rowptr.astype(np.int32), colind.astype(np.int32), vals),
            offs.astype(np.int32))


def _select(a: Csr, keep: np.ndarray) -> Csr:
    """Entries where keep is set, in their CSR order (selection keeps rows
    and columns sorted, so no re-sort is needed)."""
    kept = np.zeros(len(keep) + 1, dtype=np.int64)
    np.cumsum(keep, out=kept[1:])
    rowptr = kept[a.rowptr.astype(np.int64)]
    return Csr(a.nrows, a.ncols, rowptr.astype(np.int32), a.colind[keep].astype(np.int32),
               a.vals[keep])


def tril(a: Csr, k: int = 0) -> Csr:
    """Entries with col <= row + k (pattern selection, values copied)."""
    return _select(a, a.colind <= a.row_of_entry() + k)


def triu(a: Csr, k: int = 0) -> Csr:
    return _select(a, a.colind >= a.row_of_entry() + k)


def permute_sym(a: Csr, perm: np.ndarray) -> Csr:
    """P A P^T for the permutation new_index = position of old index in
    ``perm`` (row perm[i] of A becomes row i)."""
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    rows = inv[a.row_of_entry()]
    cols = inv[a.colind]
    return _from_coo(a.nrows, a.ncols, rows, cols, a.vals)


def four_color_2d(n: int) -> np.ndarray:
    """Ordering of an n x n grid (index iy*n + ix) by the 2x2 colouring
    color = (ix % 2) + 2*(iy % 2), natural order within each colour.
    Returns perm with perm[new] = old."""
    iy, ix = np.divmod(np.arange(n * n), n)
    color = (ix % 2) + 2 * (iy % 2)
    return np.argsort(color, kind="stable")


def red_black_3d(n: int) -> np.ndarray:
    """Red-black ordering of an n^3 grid: perm[new] = old."""
    i = np.arange(n ** 3)
    iz, rem = np.divmod(i, n * n)
    iy, ix = np.divmod(rem, n)
    return np.argsort((ix + iy + iz) % 2, kind="stable")


def random_csr(m: int, n: int, density: float, seed, empty_rows: float = 0.0,
               long_rows: int = 0, long_len: int = 0) -> Csr:
    """Uniformly random pattern with N(0,1) values; optional empty rows and a
    few long rows to exercise skewed row lengths."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    if empty_rows > 0:
        mask[rng.random(m) < empty_rows, :] = False
    for _ in range(long_rows):
        r = int(rng.integers(0, m))
        mask[r, rng.choice(n, size=min(long_len, n), replace=False)] = True
    rows, cols = np.nonzero(mask)
    return _from_coo(m, n, rows, cols, rng.standard_normal(len(rows)))


def random_rows(m: int, n: int, per_row: int, seed) -> Csr:
    """per_row uniform column draws in [0, n) for every row (repeats
    dropped, so a row holds at most per_row entries) with N(0,1) values.
    Built row-vectorised, for matrices too large for a dense mask."""
    rng = np.random.default_rng(seed)
    cols = np.sort(rng.integers(0, n, size=(m, per_row), dtype=np.int64), axis=1)
    keep = np.ones(cols.shape, dtype=bool)
    keep[:, 1:] = cols[:, 1:] != cols[:, :-1]
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(keep.sum(axis=1), out=rowptr[1:])
    assert rowptr[-1] < 2**31, "int32 CSR index space exceeded"
    colind = cols[keep].astype(np.int32)
    return Csr(m, n, rowptr.astype(np.int32), colind, rng.standard_normal(len(colind)))


def power_law_rows(n: int, seed, alpha: float = 1.2, min_len: int = 1,
                   max_len: int | None = None, empty: float = 0.0) -> Csr:
    """Square n x n matrix whose row lengths follow a heavy-tailed (Zipf-like)
    law: each row draws len = min(max_len, floor(min_len * u^(-1/alpha))),
    u ~ U(0,1], then that many uniform columns (repeats dropped), so most
    rows hold a few entries and a handful hold thousands (the uneven rows of
    scale-free graphs); a fraction `empty` of the rows is empty.  N(0,1)
    values; everything from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    max_len = n if max_len is None else min(max_len, n)
    u = 1.0 - rng.random(n)
    lens = np.minimum(max_len, np.floor(min_len * u ** (-1.0 / alpha))).astype(np.int64)
    lens[rng.random(n) < empty] = 0
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    cols = rng.integers(0, n, size=len(rows), dtype=np.int64)
    key = np.unique(rows * n + cols)
    return _from_coo(n, n, key // n, key % n, rng.standard_normal(len(key)))


def random_lower(n: int, density: float, seed, diag_shift: float = 2.0) -> Csr:
    """Random lower-triangular matrix with a full, well-conditioned
    diagonal (|L_ii| >= diag_shift) and N(0,1)/sqrt(row length) below it."""
    rng = np.random.default_rng(seed)
    mask = np.tril(rng.random((n, n)) < density, -1)
    rows, cols = np.nonzero(mask)
    cnt = np.bincount(rows, minlength=n) + 1
    off = rng.standard_normal(len(rows)) / np.sqrt(cnt[rows])
    dia = (diag_shift + rng.random(n)) * rng.choice([-1.0, 1.0], size=n)
    return _from_coo(n, n, np.concatenate([rows, np.arange(n)]),
                     np.concatenate([cols, np.arange(n)]),
                     np.concatenate([off, dia]))


def normal(shape, seed, dtype=np.float64) -> np.ndarray:
    """N(0,1) array from default_rng(seed), drawn in float64 then cast."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)
