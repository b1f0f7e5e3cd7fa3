"""Pins of the diagonal-block compression oracle (§4.1-4.2, §5.3): hand-worked
coordinate splits and tree labels, Algorithm 4 against a dense triangular solve,
full-rank sampling against the dense Cholesky factor, and the block-Cholesky
identities every leaf and every low-rank block must satisfy, checked on the
written-out factor rather than through Algorithms 5 and 6."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import diagonal as dg
from oracle.factor import NotSPDError, Options, factor, sample_count
from oracle.ordering import symbolic
from oracle.philox import gaussian_sample
from workloads import grid_coordinates, grid_problem


def test_coordinate_split_worked_example():
    # a 4 x 2 plane of points, listed scrambled: x in 0..3, y in 0..1
    pts = np.array([[3, 1, 0], [0, 0, 0], [2, 0, 0], [1, 1, 0],
                    [0, 1, 0], [3, 0, 0], [1, 0, 0], [2, 1, 0]], dtype=float)
    # depth 1: the x side (3) is longest; stable sort by x, first half x <= 1
    assert dg.coordinate_order(pts, 1).tolist() == [1, 4, 3, 6, 2, 7, 0, 5]
    # depth 2: each half has sides (1, 1): x wins the tie, each pair keeps its order
    assert dg.coordinate_order(pts, 2).tolist() == [1, 4, 3, 6, 2, 7, 0, 5]
    # a column of points along z: z is the longest side
    col = np.array([[0, 0, 2], [0, 0, 0], [0, 0, 3], [0, 0, 1]], dtype=float)
    assert dg.coordinate_order(col, 1).tolist() == [1, 3, 0, 2]
    assert dg.coordinate_order(col, 0).tolist() == [0, 1, 2, 3]


def test_tree_labels_and_ranges():
    # seven blocks (depth 2): root 4, its children 2 and 6, leaves 1 3 5 7
    assert [dg.height(s) for s in range(1, 8)] == [0, 1, 0, 2, 0, 1, 0]
    assert dg.children(4) == (2, 6) and dg.children(2) == (1, 3) and dg.children(6) == (5, 7)
    assert [dg.parent(s, 2) for s in range(1, 8)] == [2, 4, 2, None, 6, 4, 6]
    assert dg.leaf_bounds(10, 2).tolist() == [0, 2, 5, 7, 10]
    H = dg.HierDiag(c=10, d=2, bounds=dg.leaf_bounds(10, 2))
    assert H.span(4) == (0, 10) and H.cols(4) == (0, 5) and H.rows(4) == (5, 10)
    assert H.cols(6) == (5, 7) and H.rows(6) == (7, 10) and H.span(3) == (2, 5)
    assert [dg.split_depth(c, 8) for c in (8, 9, 16, 17, 33)] == [0, 1, 1, 2, 3]


def _random_tree(c, d, rank, seed):
    rng = np.random.default_rng(seed)
    H = dg.HierDiag(c=c, d=d, bounds=dg.leaf_bounds(c, d))
    for s in range(1, H.nblocks + 1):
        if dg.height(s) == 0:
            a, b = H.span(s)
            m = b - a
            H.D[s] = np.tril(rng.standard_normal((m, m))) + 3 * np.eye(m)
        else:
            (ca, cb), (ra, rb) = H.cols(s), H.rows(s)
            H.V[s] = rng.standard_normal((rb - ra, rank))
            H.U[s] = np.linalg.qr(rng.standard_normal((cb - ca, rank)))[0]
    return H


@pytest.mark.parametrize("c,d", [(9, 1), (23, 2), (40, 3)])
def test_diagonal_solve_is_a_triangular_solve(c, d):
    H = _random_tree(c, d, 2, seed=c)
    L = H.dense()
    G = np.random.default_rng(1).standard_normal((c, 3))
    assert np.allclose(dg.diagonal_solve(H, G, False), sla.solve_triangular(L, G, lower=True), atol=1e-12)
    assert np.allclose(dg.diagonal_solve(H, G, True), sla.solve_triangular(L, G, lower=True, trans="T"),
                       atol=1e-12)
    # a subtree's solve uses its own block of the factor
    a, b = H.span(2)
    Gs = G[a:b]
    assert np.allclose(dg.diagonal_solve(H, Gs, True, 2),
                       sla.solve_triangular(L[a:b, a:b], Gs, lower=True, trans="T"), atol=1e-12)


@pytest.mark.parametrize("dims,tau", [((30, 30), 8), ((12, 12, 12), 24)])
def test_full_rank_blocks_give_the_cholesky_factor(dims, tau):
    p = grid_problem(dims, sigma=1.0, seed=2)
    sym = symbolic(p.n, p.rowptr, p.colind, 64, tau, grid_coordinates(dims))
    assert int(sym.depth.max()) >= 2
    o = Options(tau_D=tau, alpha_D=1e6, alpha_O=1e6)
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, tol=1e-14, opts=o)
    A = p.matrix()[sym.perm][:, sym.perm].toarray()
    L = np.linalg.cholesky(A)
    Lt = F.dense_L()
    assert np.abs(Lt - L).max() <= 1e-11 * np.abs(L).max()


def _check_block_identities(F, j):
    """Every block of L^D_j against the Cholesky recurrences written on the dense
    factor: the Schur complement of supernode j's columns after all earlier columns
    (descendants, and the earlier blocks of L^D_j), then each leaf's D D^T and each
    low-rank block's V = (Schur block) L_{s1}^{-T} U, U orthonormal, U spanning the
    sample D_s^T Omega."""
    sym = F.sym
    lo, hi = int(sym.first[j]), int(sym.first[j + 1])
    L = F.dense_L()
    A = F.Ap.toarray()
    Sj = A[lo:hi, lo:hi] - L[lo:hi, :lo] @ L[lo:hi, :lo].T
    H = F.LD[j]
    Ld = H.dense()
    for s in range(1, H.nblocks + 1):
        if dg.height(s) == 0:
            a, b = H.span(s)
            want = Sj[a:b, a:b] - Ld[a:b, :a] @ Ld[a:b, :a].T
            assert np.allclose(H.D[s] @ H.D[s].T, want, rtol=0, atol=1e-10 * np.abs(want).max())
            continue
        (ca, cb), (ra, rb) = H.cols(s), H.rows(s)
        schur = Sj[ra:rb, ca:cb] - Ld[ra:rb, :ca] @ Ld[ca:cb, :ca].T
        Ds = sla.solve_triangular(Ld[ca:cb, ca:cb], schur.T, lower=True).T      # schur L_{s1}^{-T}
        U, V = H.U[s], H.V[s]
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-10)
        assert np.allclose(V, Ds @ U, atol=1e-9 * max(1.0, np.abs(Ds).max()))
        ell = sample_count(rb - ra, cb - ca, F.alpha_D, F.opts.oversample)
        assert U.shape[1] == ell == H.ell[s]
        Y = Ds.T @ gaussian_sample(F.opts.seed, j, rb - ra, ell, c2=4 + s)
        assert np.allclose(U @ (U.T @ Y), Y, atol=1e-9 * np.abs(Y).max())


@pytest.mark.parametrize("dims,tau,over", [((40, 40), 8, 2), ((14, 14, 14), 32, 10)])
def test_blocks_satisfy_the_cholesky_recurrences(dims, tau, over):
    p = grid_problem(dims, sigma=1.0, seed=4)
    sym = symbolic(p.n, p.rowptr, p.colind, 64, tau, grid_coordinates(dims))
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, tol=1e-2,
               opts=Options(tau_D=tau, oversample=over))
    trees = [j for j in range(sym.M) if sym.depth[j] > 0]
    assert trees and F.alpha_D == 0.5 and F.restarts == 0
    # at least one block is a true approximation (fewer samples than its size)
    assert any(H.ell[s] < min(H.rows(s)[1] - H.rows(s)[0], H.cols(s)[1] - H.cols(s)[0])
               for H in (F.LD[j] for j in trees) for s in H.ell)
    for j in trees[-3:]:
        _check_block_identities(F, j)


def test_restart_raises_alpha_by_a_quarter(monkeypatch):
    # the failure is planted: a leaf whose Schur complement is "indefinite" until
    # alpha_D reaches 1.0; the factorization must restart with 0.5, 0.625, 0.78125,
    # 0.9765625, 1.220703125 and succeed there
    dims, tau = (14, 14, 14), 32
    p = grid_problem(dims, sigma=1.0, seed=1)
    sym = symbolic(p.n, p.rowptr, p.colind, 64, tau, grid_coordinates(dims))
    real = dg.factor_hierarchical
    seen = []

    def planted(F, j, bounds, d, alpha_D, opts, key):
        seen.append(alpha_D)
        if alpha_D < 1.0:
            raise np.linalg.LinAlgError("planted")
        return real(F, j, bounds, d, alpha_D, opts, key)

    import oracle.factor as of
    monkeypatch.setattr(of, "factor_hierarchical", planted)
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, tol=1e-2, opts=Options(tau_D=tau))
    assert F.restarts == 4 and F.alpha_D == pytest.approx(0.5 * 1.25 ** 4)
    assert sorted(set(seen)) == pytest.approx([0.5 * 1.25 ** k for k in range(5)])


def test_restart_on_an_indefinite_approximation():
    """A separator whose block is dense, unstructured and nearly singular: rank-one blocks
    make a leaf's Schur complement indefinite.  Every single attempt below the final
    alpha_D (0.05 x 1.25^k) meets a non-positive pivot, the final one does not, and the
    factorization restarts exactly through that sequence (§5.3)."""
    from oracle.factor import _factor_once
    from workloads import clique_separator
    n, rp, ci, v = clique_separator(8, 8, 32, 1e-3, 0)
    sym = symbolic(n, rp, ci, 8, 4)
    assert [int(d) for d in sym.depth] == [0, 0, 3] and int(sym.kind[2]) == 1
    o = Options(tau_D=4, alpha_D=0.05, oversample=0, leaf_max=8)
    F = factor(sym, n, rp, ci, v, tol=1e-2, opts=o)
    assert F.restarts >= 5 and F.alpha_D == pytest.approx(0.05 * 1.25 ** F.restarts)
    for k in range(F.restarts):
        with pytest.raises(NotSPDError):
            _factor_once(sym, n, rp, ci, v, 1e-2, o, 0.05 * 1.25 ** k, None, None)
    L = F.dense_L()
    assert np.all(np.diag(L) > 0)
    A = F.Ap.toarray()
    assert np.linalg.eigvalsh(L @ L.T).min() > 0 and np.abs(L @ L.T - A).max() < np.abs(A).max()


def test_restart_stops_once_every_block_is_exact(monkeypatch):
    dims, tau = (16, 16), 4
    p = grid_problem(dims, sigma=1.0, seed=1)
    sym = symbolic(p.n, p.rowptr, p.colind, 64, tau, grid_coordinates(dims))

    def always(F, j, bounds, d, alpha_D, opts, key):
        raise np.linalg.LinAlgError("planted")

    import oracle.factor as of
    monkeypatch.setattr(of, "factor_hierarchical", always)
    with pytest.raises(NotSPDError):
        factor(sym, p.n, p.rowptr, p.colind, p.values, tol=1e-2, opts=Options(tau_D=tau))


def test_tree_preconditioner_converges_like_the_dense_one():
    from oracle.solve import solve
    dims = (20, 20, 20)
    p = grid_problem(dims, sigma=1.0, seed=3)
    xyz = grid_coordinates(dims)
    it = []
    for tau in (0, 48):
        sym = symbolic(p.n, p.rowptr, p.colind, 64, tau, xyz)
        F = factor(sym, p.n, p.rowptr, p.colind, p.values, tol=1e-2, opts=Options(tau_D=tau))
        r = solve(F, p.matrix(), p.b, rtol=1e-8)
        assert r.converged and r.true_residual < 1e-7
        it.append(r.iters)
    assert it[1] <= it[0] + 3, it
