"""Pins of the spectral-coordinates oracle (§4.3): closed-form grid spectra, a dense
eigen-decomposition, and a hand-built Laplacian."""
import numpy as np
import pytest

from oracle.spectral import block_lanczos, graph_laplacian, spectral_coordinates, start_block
from workloads import grid_problem


def _grid_modes(dims, count):
    """The `count` lowest nontrivial eigenpairs of an n1 x n2 (x n3) grid graph's
    Laplacian: eigenvalues sum_d 2 - 2 cos(pi k_d / n_d), eigenvectors products of
    cos(pi k_d (i_d + 1/2) / n_d) (axis 0 varies fastest in the index)."""
    ks = np.array(np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")).reshape(len(dims), -1).T
    lam = np.array([sum(2 - 2 * np.cos(np.pi * k[d] / dims[d]) for d in range(len(dims))) for k in ks])
    order = np.argsort(lam, kind="stable")[1:count + 1]
    N = int(np.prod(dims))
    cells = np.arange(N)
    strides = np.cumprod((1,) + tuple(dims[:-1]))
    coord = [(cells // strides[d]) % dims[d] for d in range(len(dims))]
    vecs = []
    for o in order:
        v = np.ones(N)
        for d in range(len(dims)):
            v *= np.cos(np.pi * ks[o][d] * (coord[d] + 0.5) / dims[d])
        vecs.append(v / np.linalg.norm(v))
    return lam[order], np.array(vecs).T


def _angles(A, B):
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    return np.linalg.svd(qa.T @ qb, compute_uv=False)


def test_laplacian_of_a_hand_built_pattern():
    # 4 indices: edges 0-1, 1-2, 1-3 (and the diagonal stored); row 3 also stores 3-1
    rowptr = [0, 2, 6, 8, 10]
    colind = [0, 1, 0, 1, 2, 3, 1, 2, 1, 3]
    L = graph_laplacian(4, rowptr, colind).toarray()
    want = np.array([[1, -1, 0, 0], [-1, 3, -1, -1], [0, -1, 1, 0], [0, -1, 0, 1]], dtype=float)
    assert np.array_equal(L, want)


def test_distinct_grid_modes_match_the_closed_form():
    dims = (12, 7, 5)                     # lowest modes (1,0,0), (0,1,0), (1,1,0): distinct
    p = grid_problem(dims, sigma=0.0, seed=0)
    Y, theta = spectral_coordinates(p.n, p.rowptr, p.colind, steps=60, seed=1)
    lam, V = _grid_modes(dims, 3)
    assert np.allclose(theta, lam, rtol=1e-10, atol=1e-12), (theta, lam)
    for c in range(3):
        assert abs(abs(Y[:, c] @ V[:, c]) - 1) < 1e-9, (c, Y[:, c] @ V[:, c])
    w = np.arange(1, p.n + 1)
    assert np.all(w @ Y >= 0)            # sign convention
    assert np.allclose(Y.T @ Y, np.eye(3), atol=1e-12)
    assert np.allclose(Y.sum(axis=0), 0, atol=1e-10)   # orthogonal to the constant vector


def test_cube_resolves_the_threefold_axis_mode():
    dims = (6, 6, 6)                      # 2 - 2 cos(pi/6) has multiplicity three
    p = grid_problem(dims, sigma=0.0, seed=0)
    Y, theta = spectral_coordinates(p.n, p.rowptr, p.colind, steps=30, seed=2)
    lam, V = _grid_modes(dims, 3)
    assert np.allclose(theta, 2 - 2 * np.cos(np.pi / 6), rtol=1e-10)
    assert np.allclose(lam, 2 - 2 * np.cos(np.pi / 6))
    assert _angles(Y, V).min() > 1 - 1e-9     # the same three-dimensional subspace


def test_full_krylov_space_gives_the_dense_spectrum():
    # an irregular graph: a 7 x 6 grid with long-range edges and one more vertex (43 in
    # all), so that 14 blocks of three and the constant vector span the whole space
    p = grid_problem((7, 6), sigma=0.0, seed=0)
    rows = [list(p.colind[p.rowptr[i]:p.rowptr[i + 1]]) for i in range(p.n)] + [[42]]
    for a, b in ((0, 40), (5, 30), (12, 41), (42, 3), (42, 20)):
        rows[a].append(b); rows[b].append(a)
    n = len(rows)
    rowptr = np.cumsum([0] + [len(r) for r in rows])
    colind = np.concatenate([np.sort(r) for r in rows])
    L = graph_laplacian(n, rowptr, colind).toarray()
    ev, U = np.linalg.eigh(L)
    Y, theta = spectral_coordinates(n, rowptr, colind, steps=14, seed=3)   # 1 + 42 = n
    assert np.allclose(theta, ev[1:4], rtol=1e-11, atol=1e-13), (theta - ev[1:4])
    assert _angles(Y, U[:, 1:4]).min() > 1 - 1e-10


def test_basis_is_orthonormal_and_start_block_is_seeded():
    p = grid_problem((9, 8, 7), sigma=0.0, seed=0)
    X0 = start_block(p.n, 5)
    assert np.array_equal(X0, start_block(p.n, 5)) and not np.array_equal(X0, start_block(p.n, 6))
    Q, T = block_lanczos(graph_laplacian(p.n, p.rowptr, p.colind), X0, 6)
    assert np.allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-12)
    assert np.allclose(T, T.T)
