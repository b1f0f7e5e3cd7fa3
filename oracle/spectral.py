"""Oracle: spectral coordinates of a matrix's graph (§4.3) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may
import this module; the library never does, and it imports nothing from the library.

§4.3 assigns each matrix index a position in three dimensions when the problem supplies
none: the entries of the three lowest eigenvectors of the graph Laplacian of the pattern
(off-diagonal entry -1 for every stored off-diagonal entry, diagonal entry the number of
those in the row), computed to low accuracy by Arnoldi iteration.

Readings:
* the lowest eigenvector of a connected graph's Laplacian is the constant vector
  (eigenvalue 0), which puts every index at one point; the coordinates are the three
  lowest eigenvectors orthogonal to it (the iteration keeps the constant vector as the
  first basis vector, so every later vector is orthogonal to it);
* the iteration is the symmetric (Lanczos) form of Arnoldi with a block of three
  vectors: the three coordinates may belong to one eigenvalue of multiplicity three (the
  three axis modes of a cubic grid), which a single-vector Krylov space never resolves;
  every new block is orthogonalised against all earlier basis vectors, twice;
* the start block is drawn from the counter-based generator of ``philox`` under key
  ``(seed mod 2^32, (seed >> 32) XOR 0xFFFFFFFF)`` with third counter word 2 (entry
  ``(i, c)`` for index ``i`` and column ``c``);
* the coordinates are the Ritz vectors of the three smallest Ritz values of the projected
  block-tridiagonal matrix, each signed so that ``sum_i (i + 1) y_i >= 0``.

Parity status: pinned by the closed-form spectrum of grid graphs (the Laplacian of an
``n1 x n2 x n3`` grid has eigenvalues ``sum_d 2 - 2 cos(pi k_d / n_d)`` with cosine
eigenvectors), by a dense eigen-decomposition on small graphs, and by the explicit
Laplacian of a hand-built graph.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .philox import gaussian_sample

BLOCK = 3


def graph_laplacian(n: int, rowptr, colind) -> sp.csr_matrix:
    """The graph Laplacian of a CSR pattern (§4.3): -1 per stored off-diagonal entry,
    the row's count of them on the diagonal."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    off = rows != colind
    L = sp.csr_matrix((-np.ones(int(off.sum())), (rows[off], colind[off])), shape=(n, n))
    deg = np.bincount(rows[off], minlength=n).astype(float)
    return (L + sp.diags(deg)).tocsr()


def start_block(n: int, seed: int) -> np.ndarray:
    return gaussian_sample(seed, 0xFFFFFFFF, n, BLOCK, c2=2)


def _orthonormalise(W: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """W = Q R with R upper triangular, positive diagonal (Householder QR, signs fixed)."""
    Q, R = np.linalg.qr(W)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s, R * s[:, None]


def block_lanczos(Lap: sp.csr_matrix, X0: np.ndarray, steps: int):
    """``steps`` blocks of the block Lanczos iteration from the start block ``X0``, the
    constant vector as the basis' first vector.  Returns the basis ``Q`` (``n x (1 + 3
    steps)``, orthonormal) and the projected block-tridiagonal matrix ``T`` (``3 steps``
    square) on the blocks."""
    n = Lap.shape[0]
    e = np.full((n, 1), 1.0 / np.sqrt(n))
    basis = [e]
    W = X0.copy()
    for _ in range(2):
        B = np.hstack(basis)
        W = W - B @ (B.T @ W)
    X, _ = _orthonormalise(W)
    T = np.zeros((BLOCK * steps, BLOCK * steps))
    for k in range(steps):
        basis.append(X)
        LX = Lap @ X
        T[BLOCK * k:BLOCK * (k + 1), BLOCK * k:BLOCK * (k + 1)] = X.T @ LX
        if k + 1 == steps:
            break
        W = LX
        for _ in range(2):
            B = np.hstack(basis)
            W = W - B @ (B.T @ W)
        Xn, R = _orthonormalise(W)
        # X_{k+1} R = L X_k - (projections): the off-diagonal block X_{k+1}^T L X_k = R
        T[BLOCK * (k + 1):BLOCK * (k + 2), BLOCK * k:BLOCK * (k + 1)] = R
        T[BLOCK * k:BLOCK * (k + 1), BLOCK * (k + 1):BLOCK * (k + 2)] = R.T
        X = Xn
    return np.hstack(basis), T


def spectral_coordinates(n: int, rowptr, colind, steps: int = 20, seed: int = 0):
    """Positions ``(n, 3)`` of §4.3 and the three Ritz values they belong to."""
    Lap = graph_laplacian(n, rowptr, colind)
    Q, T = block_lanczos(Lap, start_block(n, seed), steps)
    theta, S = np.linalg.eigh(T)
    Y = Q[:, 1:] @ S[:, :BLOCK]
    w = np.arange(1, n + 1, dtype=float)
    Y = Y * np.where(w @ Y < 0, -1.0, 1.0)
    return Y, theta[:BLOCK]
