"""Oracle: adjoint of the solve (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this module; the product path never does.

For ``x = A^{-1} b`` and a loss ``L(x)`` with gradient ``g = dL/dx``:
``lambda = A^{-T} g = A^{-1} g`` (A symmetric), ``dL/db = lambda`` and
``dL/dA_p = -lambda_row(p) x_col(p)`` on every stored entry ``p`` of A's pattern.
Through ``values = value_map @ coef + const`` the coefficient gradient is
``value_map^T dL/dA``; for a face between cells i and j this is
``-(lambda_i - lambda_j)(x_i - x_j)``, and ``-lambda_i x_i`` for a boundary face.
Not in the paper: this differentiates the solve its method computes.
"""
from __future__ import annotations

import numpy as np


def dense_adjoint(A_dense: np.ndarray, b: np.ndarray, x_target: np.ndarray):
    """Loss ``0.5 ||x - x_target||^2`` with dense LAPACK solves (tiny grids)."""
    x = np.linalg.solve(A_dense, b)
    lam = np.linalg.solve(A_dense, x - x_target)
    loss = 0.5 * float((x - x_target) @ (x - x_target))
    return x, lam, loss


def grad_values(rowptr, colind, lam, x):
    """``-lambda_row(p) x_col(p)`` for every pattern entry, CSR order."""
    rows = np.repeat(np.arange(rowptr.size - 1), np.diff(rowptr))
    return -lam[rows] * x[np.asarray(colind, dtype=np.int64)]


def grad_faces(face_i, face_j, lam, x):
    """Face-coefficient gradient written out per face."""
    fi = np.asarray(face_i, dtype=np.int64)
    fj = np.asarray(face_j, dtype=np.int64)
    g = -lam[fi] * x[fi]
    inner = fj >= 0
    g[inner] = -(lam[fi[inner]] - lam[fj[inner]]) * (x[fi[inner]] - x[fj[inner]])
    return g
