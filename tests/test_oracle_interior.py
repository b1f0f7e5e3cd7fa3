"""Pins of the interior blocks (§5.1) in the oracle: the closed form
L(R^B, C^B) = A(R^B, C^B) L(C^B, C^B)^{-T} against the block the factorization computes,
the blocks as maximal compression-free subtrees, and the preconditioner applied through
eq. interiorBlockMult against the one applied with the stored blocks."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.factor import Options, factor
from oracle.ordering import symbolic
from oracle.solve import _block_factor, apply_preconditioner, interior_blocks
from workloads import grid_problem


def _factor(dims, tol=1e-2, seed=1):
    p = grid_problem(dims, sigma=1.0, seed=seed)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    return p, sym, factor(sym, p.n, p.rowptr, p.colind, p.values, tol, Options())


@pytest.mark.parametrize("dims", [(64, 64), (14, 13, 12)])
def test_closed_form_of_the_interior_off_diagonal_block(dims):
    p, sym, F = _factor(dims)
    blocks = interior_blocks(F)
    assert len(blocks) > 3 and any(s1 > s0 for s0, s1 in blocks)
    A = F.Ap.toarray()
    L = F.dense_L()
    for s0, s1 in blocks:
        a, b = int(sym.first[s0]), int(sym.first[s1 + 1])
        LB = L[a:b, a:b]
        assert np.allclose(LB @ LB.T, A[a:b, a:b], atol=1e-10 * np.abs(A).max())   # chol(A(C^B, C^B))
        # every column of the block: rows beyond C^B come from A alone
        tail = sla.solve_triangular(LB, A[b:, a:b].T, lower=True).T
        assert np.abs(L[b:, a:b] - tail).max() <= 1e-11 * max(1.0, np.abs(tail).max())
        # maximal: the parent of the root is compressed (or there is none)
        par = int(sym.parent[s1])
        assert par < 0 or F.LO[par] is None
        assert all(F.LO[k] is not None for k in range(s0, s1 + 1))


@pytest.mark.parametrize("dims", [(72, 70), (16, 15, 14), (20, 20, 20)])
def test_interior_apply_equals_the_stored_block_apply(dims):
    p, sym, F = _factor(dims)
    r = np.random.default_rng(2).standard_normal(p.n)
    z0 = apply_preconditioner(F, r)
    z1 = apply_preconditioner(F, r, interior=True)
    assert np.abs(z1 - z0).max() <= 1e-11 * np.abs(z0).max()


def test_block_factor_is_the_blocks_own_cholesky():
    p, sym, F = _factor((64, 64))
    for s0, s1 in interior_blocks(F)[:20]:
        LB, a, b = _block_factor(F, s0, s1)
        A = F.Ap[a:b][:, a:b].toarray()
        assert np.allclose(np.linalg.cholesky(A), LB.toarray(), atol=1e-12 * np.abs(A).max())


def test_exact_factor_is_one_interior_block():
    p, sym, F = _factor((12, 12), tol=0.0)
    assert interior_blocks(F) == [(0, sym.M - 1)]
