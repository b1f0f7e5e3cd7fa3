"""Oracle: triangular solves with the factor and preconditioned CG (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this module; the product path never does.

* ``apply_preconditioner``: the two triangular solves of §1 with the (exact or
  rank-structured) factor of the permuted matrix, ``z = P^T L^{-T} L^{-1} P r``.
  The paper does not spell the supernodal sweeps out; forward, for ``j``
  ascending: ``y_C = (L^D_j)^{-1} y_C`` then ``y_R -= L^O_j y_C`` (or
  ``V_j (U_j^T y_C)`` for a compressed supernode); backward, for ``j`` descending:
  ``z_C = (L^D_j)^{-T} (z_C - (L^O_j)^T z_R)`` (or ``U_j (V_j^T z_R)``).
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

from .factor import Factor, diag_solve


def apply_preconditioner(F: Factor, r: np.ndarray) -> np.ndarray:
    sym = F.sym
    y = np.asarray(r, dtype=np.float64)[sym.perm].copy()
    for j in range(sym.M):
        lo, hi = int(sym.first[j]), int(sym.first[j + 1])
        y[lo:hi] = diag_solve(F.LD[j], y[lo:hi], transpose=False)
        R = sym.rows[j]
        if R.size:
            if F.LO[j] is not None:
                y[R] -= F.LO[j] @ y[lo:hi]
            else:
                y[R] -= F.V[j] @ (F.U[j].T @ y[lo:hi])
    for j in range(sym.M - 1, -1, -1):
        lo, hi = int(sym.first[j]), int(sym.first[j + 1])
        R = sym.rows[j]
        w = y[lo:hi].copy()
        if R.size:
            if F.LO[j] is not None:
                w -= F.LO[j].T @ y[R]
            else:
                w -= F.U[j] @ (F.V[j].T @ y[R])
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
