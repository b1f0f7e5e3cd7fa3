"""Finite-difference diffusion problems on regular grids (seeded, synthetic).

Problem definition (a stand-in for the paper's inhomogeneous Poisson and
elasticity workloads of Section 6, which need deal.II meshes and the Florida
collection and are not available here):

* unknowns are the interior points of an ``n_0 x n_1 [x n_2]`` grid, numbered
  lexicographically with the first axis fastest;
* for axis ``d`` the parameter ``k_d(c)`` is the coefficient of the face
  between cell ``c`` and ``c + e_d``; when ``c_d = n_d - 1`` that face touches
  the (Dirichlet) boundary ghost.  Faces between the low boundary and cells with
  ``c_d = 0`` have the fixed coefficient 1, so each parameter owns exactly one
  face;
* ``A[c, c] = sum of the coefficients of all 2d faces of c`` and
  ``A[c, c + e_d] = A[c + e_d, c] = -k_d(c)``; with all ``k = 1`` this is the
  classic 4/-1 (2D) or 6/-1 (3D) stencil, without ``h^2`` scaling;
* random draws come from ``numpy.random.default_rng(seed)`` in this order:
  the coefficient arrays (axis-major, each lexicographic) as
  ``exp(sigma * N(0, 1))``, then ``b ~ N(0, 1)``, then ``x_target ~ N(0, 1)``.

The matrix is returned as a full symmetric CSR pattern (sorted, no duplicates,
diagonal present) with int64 row pointers and int32 column indices.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class GridProblem:
    dims: tuple
    sigma: float
    seed: int
    n: int
    rowptr: np.ndarray
    colind: np.ndarray
    values: np.ndarray
    coef: np.ndarray            # (d, N) face coefficients k_d(c)
    face_i: np.ndarray          # (d*N,) low-side cell of each parameter's face
    face_j: np.ndarray          # (d*N,) high-side cell, -1 for a boundary face
    b: np.ndarray
    x_target: np.ndarray
    value_map: sp.csr_matrix = field(repr=False)   # values = value_map @ coef.ravel() + value_const
    value_const: np.ndarray = field(repr=False)

    @property
    def nnz(self) -> int:
        return int(self.colind.size)

    def matrix(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.values, self.colind, self.rowptr), shape=(self.n, self.n))

    def values_from_coef(self, coef: np.ndarray) -> np.ndarray:
        return self.value_map @ np.asarray(coef, dtype=np.float64).ravel() + self.value_const


def _strides(dims):
    s = [1]
    for d in dims[:-1]:
        s.append(s[-1] * d)
    return s


def _build_pattern(dims):
    """Pattern of the stencil plus the linear map coefficients -> CSR values."""
    dims = tuple(int(x) for x in dims)
    nd = len(dims)
    N = int(np.prod(dims))
    strides = _strides(dims)
    cells = np.arange(N, dtype=np.int64)
    # coordinate of every cell along every axis
    coords = [(cells // strides[d]) % dims[d] for d in range(nd)]

    rows, cols, par, sgn, const = [], [], [], [], []
    # diagonal contributions: own +d face (parameter d*N + c) ...
    for d in range(nd):
        rows.append(cells); cols.append(cells)
        par.append(d * N + cells); sgn.append(np.ones(N)); const.append(np.zeros(N))
        # ... and the -d face: parameter of the lower neighbour, or the fixed 1
        low = coords[d] > 0
        rows.append(cells[low]); cols.append(cells[low])
        par.append(d * N + cells[low] - strides[d]); sgn.append(np.ones(int(low.sum())))
        const.append(np.zeros(int(low.sum())))
        rows.append(cells[~low]); cols.append(cells[~low])
        par.append(np.full(int((~low).sum()), -1)); sgn.append(np.zeros(int((~low).sum())))
        const.append(np.ones(int((~low).sum())))
        # off-diagonal couplings across interior +d faces
        up = coords[d] < dims[d] - 1
        c = cells[up]
        for (r_, c_) in ((c, c + strides[d]), (c + strides[d], c)):
            rows.append(r_); cols.append(c_)
            par.append(d * N + c); sgn.append(-np.ones(c.size)); const.append(np.zeros(c.size))
    rows = np.concatenate(rows); cols = np.concatenate(cols)
    par = np.concatenate(par); sgn = np.concatenate(sgn); const = np.concatenate(const)

    # CSR order: sort entries by (row, col); duplicates (the diagonal) merge
    key = rows * N + cols
    order = np.argsort(key, kind="stable")
    key_s = key[order]
    uniq, first = np.unique(key_s, return_index=True)
    slot = np.empty(key.size, dtype=np.int64)
    slot[order] = np.searchsorted(uniq, key_s)
    nnz = uniq.size
    r_u = (uniq // N).astype(np.int64)
    colind = (uniq % N).astype(np.int32)
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(rowptr, r_u + 1, 1)
    rowptr = np.cumsum(rowptr)

    has_par = par >= 0
    value_map = sp.csr_matrix((sgn[has_par], (slot[has_par], par[has_par])), shape=(nnz, nd * N))
    value_const = np.zeros(nnz)
    np.add.at(value_const, slot, const)

    face_i = np.concatenate([cells for _ in range(nd)]).astype(np.int32)
    face_j = np.concatenate([np.where(coords[d] < dims[d] - 1, cells + strides[d], -1)
                             for d in range(nd)]).astype(np.int32)
    return N, rowptr, colind, value_map, value_const, face_i, face_j


def grid_coordinates(dims) -> np.ndarray:
    """Positions of the unknowns (``N x 3`` FP64, the cell's integer grid coordinates,
    zero beyond the grid's dimension), in the unknowns' lexicographic numbering."""
    dims = tuple(int(x) for x in dims)
    N = int(np.prod(dims))
    strides = _strides(dims)
    cells = np.arange(N, dtype=np.int64)
    xyz = np.zeros((N, 3))
    for d in range(len(dims)):
        xyz[:, d] = (cells // strides[d]) % dims[d]
    return xyz


def clique_separator(na: int, nb: int, m: int, lam_min: float, seed: int):
    """Two cliques of ``na`` and ``nb`` unknowns joined through a separator clique of ``m``
    (every separator unknown coupled to every other unknown): a pattern whose dissection
    (leaves of at most ``max(na, nb)``) makes the ``m`` unknowns one separator.  The
    separator block is ``Q diag(lambda) Q^T`` with ``Q`` a seeded random orthogonal matrix
    and ``lambda`` geometric from ``lam_min`` to 1 (a dense, unstructured, nearly singular
    block); the cliques' blocks are ``2 I + 0.1``; their couplings to the separator are
    1e-6.  Returns ``(n, rowptr, colind, values)`` of the full symmetric CSR."""
    rng = np.random.default_rng(seed)
    n = na + nb + m
    A = np.zeros((n, n))
    a, b, s = np.arange(na), np.arange(na, na + nb), np.arange(na + nb, n)
    A[np.ix_(a, a)] = 2.0 * np.eye(na) + 0.1
    A[np.ix_(b, b)] = 2.0 * np.eye(nb) + 0.1
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    A[np.ix_(s, s)] = Q @ np.diag(np.geomspace(lam_min, 1.0, m)) @ Q.T
    for blk in (a, b):
        A[np.ix_(blk, s)] = 1e-6
        A[np.ix_(s, blk)] = 1e-6
    A = 0.5 * (A + A.T)
    pat = (A != 0) | np.eye(n, dtype=bool)
    rowptr = np.concatenate(([0], np.cumsum(pat.sum(axis=1)))).astype(np.int64)
    colind = np.nonzero(pat)[1].astype(np.int32)
    return n, rowptr, colind, A[pat]


def grid_problem(dims, sigma: float = 0.0, seed: int = 0, unit: bool = False) -> GridProblem:
    """One seeded diffusion problem; ``unit=True`` sets every coefficient to 1."""
    dims = tuple(int(x) for x in dims)
    N, rowptr, colind, vmap, vconst, face_i, face_j = _build_pattern(dims)
    rng = np.random.default_rng(seed)
    nd = len(dims)
    if unit:
        coef = np.ones((nd, N))
    else:
        coef = np.exp(sigma * rng.standard_normal((nd, N)))
    b = rng.standard_normal(N)
    x_target = rng.standard_normal(N)
    values = vmap @ coef.ravel() + vconst
    return GridProblem(dims=dims, sigma=float(sigma), seed=int(seed), n=N, rowptr=rowptr,
                       colind=colind, values=values, coef=coef, face_i=face_i, face_j=face_j,
                       b=b, x_target=x_target, value_map=vmap, value_const=vconst)


def batched_problems(count: int, side_lo: int, side_hi: int, sigma: float, seed: int):
    """Independent 2D problems of uneven size: the sides are drawn first
    (``integers(side_lo, side_hi + 1)``), then each system draws its own
    coefficients and right-hand side from a generator seeded ``(seed, i)``."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, size=count)
    probs = []
    for i, s in enumerate(sides):
        sub_seed = int(np.random.SeedSequence([seed, i]).generate_state(1)[0])
        probs.append(grid_problem((int(s), int(s)), sigma=sigma, seed=sub_seed))
    return probs


def block_diagonal(probs):
    """Concatenate independent systems into one block-diagonal CSR."""
    offs = np.cumsum([0] + [p.n for p in probs])
    rowptr = [np.zeros(1, dtype=np.int64)]
    colind, values = [], []
    base = 0
    for p, o in zip(probs, offs[:-1]):
        rowptr.append(p.rowptr[1:] + base)
        colind.append(p.colind.astype(np.int64) + o)
        values.append(p.values)
        base += p.nnz
    return (int(offs[-1]), np.concatenate(rowptr), np.concatenate(colind).astype(np.int32),
            np.concatenate(values), offs)


# The five benchmark workloads (sizes, coefficient laws and solver settings).
WORKLOADS = {
    "poisson2d_64": dict(dims=(64, 64), sigma=0.0, unit=True, seed=1, tol=1e-2, rtol=1e-8),
    "diffusion3d_64": dict(dims=(64, 64, 64), sigma=1.0, unit=False, seed=2, tol=1e-2, rtol=1e-8),
    "diffusion3d_96": dict(dims=(96, 96, 96), sigma=1.5, unit=False, seed=3, tol=1e-2, rtol=1e-8),
    "batched2d_64": dict(count=64, side_lo=128, side_hi=512, sigma=1.0, seed=4, tol=1e-2, rtol=1e-8),
    "adjoint3d_80": dict(dims=(80, 80, 80), sigma=1.0, unit=False, seed=5, tol=1e-2, rtol=1e-8),
}


def workload_config(name: str) -> dict:
    return dict(WORKLOADS[name])
