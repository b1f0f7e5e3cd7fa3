"""Oracle: triangular solves with the factor and preconditioned CG (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this module; the product path never does.

* ``apply_preconditioner``: the two triangular solves of §1 with the (exact or
  rank-structured) factor of the permuted matrix, ``z = P^T L^{-T} L^{-1} P r``.
  The paper does not spell the supernodal sweeps out; forward, for ``j``
  ascending: ``y_C = (L^D_j)^{-1} y_C`` then ``y_R -= L^O_j y_C`` (or
  ``V_j (U_j^T y_C)`` for a compressed supernode); backward, for ``j`` descending:
  ``z_C = (L^D_j)^{-T} (z_C - (L^O_j)^T z_R)`` (or ``U_j (V_j^T z_R)``).
* ``apply_preconditioner(..., interior=True)``: the same solves with the interior blocks
  of §5.1.  An interior block ``B`` is a maximal subtree of the elimination tree without a
  compressed supernode (a contiguous range of supernodes and columns ``C^B``: the
  subdomains the compressed separators cut out); its rows ``R^B`` are the rows of its
  supernodes outside ``C^B``.  The block ``L(R^B, C^B)`` is not used; its products come
  from the closed form ``L(R^B, C^B) = A(R^B, C^B) L(C^B, C^B)^{-T}`` (nothing outside the
  subtree enters those columns' Schur complements): forward, once the block's columns are
  solved, ``y_{R^B} -= A(R^B, C^B) (L^B)^{-T} w^B``; backward, before them,
  ``y_{C^B} -= (L^B)^{-1} A(C^B, R^B) z_{R^B}`` -- a sparse product and a triangular solve
  with the block's own factor ``L^B = L(C^B, C^B)`` each, as in eq. interiorBlockMult.
* ``pcg``: conjugate gradients preconditioned by the factor (§5.2, §6.1.1),
  started from ``x = 0`` and stopped when the recursive residual satisfies
  ``||r_k|| / ||b|| <= rtol`` (the relative l2 residual criterion of §6.1.1);
  the true residual ``||b - A x|| / ||b||`` is reported beside it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .factor import Factor, diag_solve


def interior_blocks(F: Factor):
    """Interior blocks (§5.1) of a rank-structured factor: ``(s0, s1)`` supernode ranges,
    each a maximal subtree of the elimination tree without a compressed supernode (the
    supernodes of a subtree are consecutive in the dissection order, its root last)."""
    sym = F.sym
    M = sym.M
    clean = np.zeros(M, dtype=bool)
    size = np.ones(M, dtype=np.int64)
    kids = [[] for _ in range(M)]
    for k in range(M):
        if sym.parent[k] >= 0:
            kids[int(sym.parent[k])].append(k)
    for k in range(M):                    # children come before their parent
        clean[k] = F.LO[k] is not None and all(clean[x] for x in kids[k])
        size[k] += sum(int(size[x]) for x in kids[k])
    out = []
    for k in range(M):
        p = int(sym.parent[k])
        if clean[k] and (p < 0 or not clean[p]):
            out.append((k - int(size[k]) + 1, k))
    return out


def _block_factor(F: Factor, s0: int, s1: int):
    """``L^B = L(C^B, C^B)`` of an interior block as a sparse lower-triangular matrix."""
    sym = F.sym
    a, b = int(sym.first[s0]), int(sym.first[s1 + 1])
    L = np.zeros((b - a, b - a))
    for k in range(s0, s1 + 1):
        lo, hi = int(sym.first[k]), int(sym.first[k + 1])
        L[lo - a:hi - a, lo - a:hi - a] = F.LD[k]
        R = sym.rows[k]
        head = R < b
        L[np.ix_(R[head] - a, np.arange(lo - a, hi - a))] = F.LO[k][head]
    return sp.csr_matrix(L), a, b


def apply_preconditioner(F: Factor, r: np.ndarray, interior: bool = False) -> np.ndarray:
    sym = F.sym
    y = np.asarray(r, dtype=np.float64)[sym.perm].copy()
    blocks = {}
    if interior:
        for s0, s1 in interior_blocks(F):
            LB, a, b = _block_factor(F, s0, s1)
            Rb = np.unique(np.concatenate([sym.rows[k] for k in range(s0, s1 + 1)]))
            Rb = Rb[Rb >= b]
            blocks[s1] = (s0, LB, a, b, Rb, F.Ap[Rb][:, a:b])
    in_block = np.full(sym.M, -1, dtype=np.int64)
    for s1, (s0, *_rest) in blocks.items():
        in_block[s0:s1 + 1] = s1

    def rows_of(j):
        """The rows of L^O_j the sweeps use: within its interior block only, else all."""
        R = sym.rows[j]
        if in_block[j] < 0:
            return R, F.LO[j]
        head = R < blocks[int(in_block[j])][3]
        return R[head], F.LO[j][head]

    for j in range(sym.M):
        lo, hi = int(sym.first[j]), int(sym.first[j + 1])
        y[lo:hi] = diag_solve(F.LD[j], y[lo:hi], transpose=False)
        if F.LO[j] is not None:
            R, LO = rows_of(j)
            if R.size:
                y[R] -= LO @ y[lo:hi]
        elif sym.rows[j].size:
            y[sym.rows[j]] -= F.V[j] @ (F.U[j].T @ y[lo:hi])
        if j in blocks:                   # eq. interiorBlockMult, forward
            s0, LB, a, b, Rb, ARC = blocks[j]
            t = spla.spsolve_triangular(LB.T.tocsr(), y[a:b], lower=False)
            y[Rb] -= ARC @ t
    for j in range(sym.M - 1, -1, -1):
        if j in blocks:                   # eq. interiorBlockMult, backward
            s0, LB, a, b, Rb, ARC = blocks[j]
            y[a:b] -= spla.spsolve_triangular(LB, ARC.T @ y[Rb], lower=True)
        lo, hi = int(sym.first[j]), int(sym.first[j + 1])
        w = y[lo:hi].copy()
        if F.LO[j] is not None:
            R, LO = rows_of(j)
            if R.size:
                w -= LO.T @ y[R]
        elif sym.rows[j].size:
            w -= F.U[j] @ (F.V[j].T @ y[sym.rows[j]])
        y[lo:hi] = diag_solve(F.LD[j], w, transpose=True)
    z = np.empty_like(y)
    z[sym.perm] = y
    return z


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    rel_residual: float        # recursive
    true_residual: float
    history: list


def pcg(A: sp.spmatrix, b: np.ndarray, apply_M, rtol: float = 1e-8, max_iter: int = 1000) -> PCGResult:
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return PCGResult(x, 0, True, 0.0, 0.0, [])
    r = b.copy()
    z = apply_M(r)
    p = z.copy()
    rz = float(r @ z)
    hist = []
    it = 0
    rel = 1.0
    converged = False
    while it < max_iter:
        Ap = A @ p
        pAp = float(p @ Ap)
        if pAp <= 0.0 or rz <= 0.0:
            break
        alpha = rz / pAp
        x += alpha * p
        r -= alpha * Ap
        it += 1
        rel = float(np.linalg.norm(r)) / bnorm
        hist.append(rel)
        if rel <= rtol:
            converged = True
            break
        z = apply_M(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    true = float(np.linalg.norm(b - A @ x)) / bnorm
    return PCGResult(x, it, converged, rel, true, hist)


def solve(F: Factor, A: sp.spmatrix, b, rtol=1e-8, max_iter=1000) -> PCGResult:
    return pcg(A, b, lambda v: apply_preconditioner(F, v), rtol, max_iter)
