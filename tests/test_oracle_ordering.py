"""Pins of the oracle's ordering and symbolic analysis (CPU only)."""
import json

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import golden_path
from oracle.ordering import (LEAF, SEPARATOR, check_pattern, gather_rows, nested_dissection,
                             scatter_rows, symbolic)
from workloads import grid_problem


def path_graph(n):
    rows, cols = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i); cols.append(j)
    A = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    return A.indptr.astype(np.int64), A.indices.astype(np.int32)


def test_scatter_rows_worked_example():
    g = json.load(open(golden_path("scatter_rows_example.json")))
    out = scatter_rows(np.array(g["B"]), g["R1"], g["R2"])
    assert out.tolist() == g["expected"]
    # gatherRows reverses scatterRows (paper Sec. 2.1)
    assert gather_rows(out, g["R2"], g["R1"]).tolist() == g["B"]


def test_nd_path_graph_hand_worked():
    g = json.load(open(golden_path("nd_path200.json")))
    rp, ci = path_graph(g["n"])
    perm, first, kind = nested_dissection(g["n"], rp, ci, g["leaf_max"])
    got = []
    for j in range(first.size - 1):
        seg = perm[first[j]:first[j + 1]]
        assert np.all(np.diff(seg) == 1)
        got.append([int(seg[0]), int(seg[-1]), "leaf" if kind[j] == LEAF else "separator"])
    assert got == g["supernodes"]
    # row sets, elimination tree and levels of the same dissection, worked by hand
    sym = symbolic(g["n"], rp, ci, g["leaf_max"])
    assert [list(map(int, r)) for r in sym.rows] == g["rows"]
    assert [int(v) for v in sym.parent] == g["parent"]
    assert [int(v) for v in sym.level] == g["level"]


def test_nd_square_grid_top_separator_is_antidiagonal():
    # From corner 0 the BFS levels of an n x n 5-point grid are anti-diagonals
    # x + y = t; the corner is already pseudo-peripheral (the far corner has the
    # same eccentricity), the balanced level is t = n - 1 and every vertex on it
    # has a neighbour on t = n, so the last supernode is that anti-diagonal.
    n = 16
    p = grid_problem((n, n), unit=True)
    perm, first, kind = nested_dissection(p.n, p.rowptr, p.colind, 64)
    top = perm[first[-2]:first[-1]]
    x, y = top % n, top // n
    assert kind[-1] == SEPARATOR
    assert np.all(x + y == n - 1) and top.size == n


@pytest.mark.parametrize("dims", [(9, 7), (20, 20), (6, 7, 5), (12, 12, 12)])
def test_nd_valid_and_separating(dims):
    p = grid_problem(dims, sigma=1.0, seed=3)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    assert np.array_equal(np.sort(sym.perm), np.arange(p.n))
    # Every coupling of A points from a supernode to one of its ancestors: the
    # separators really separate (no edge joins two unrelated subtrees).
    anc = [set() for _ in range(sym.M)]
    for j in range(sym.M - 1, -1, -1):
        q = sym.parent[j]
        anc[j] = ({int(q)} | anc[q]) if q >= 0 else set()
    A = p.matrix().tocoo()
    u = sym.iperm[A.row]; v = sym.iperm[A.col]
    lo = np.minimum(u, v); hi = np.maximum(u, v)
    for a, b in zip(sym.owner[lo], sym.owner[hi]):
        assert a == b or int(b) in anc[int(a)]


@pytest.mark.parametrize("dims", [(10, 10), (5, 6, 7), (8, 8, 8)])
def test_union_pattern_contains_cholesky_pattern(dims):
    p = grid_problem(dims, sigma=0.5, seed=2)
    sym = symbolic(p.n, p.rowptr, p.colind, 16)
    Ap = p.matrix()[sym.perm][:, sym.perm].toarray()
    L = np.linalg.cholesky(Ap)
    allowed = np.zeros_like(L, dtype=bool)
    for j in range(sym.M):
        lo, hi = sym.first[j], sym.first[j + 1]
        allowed[lo:hi, lo:hi] = True
        allowed[np.ix_(sym.rows[j], np.arange(lo, hi))] = True
    assert not np.any((np.abs(L) > 0) & ~np.tril(allowed))


@pytest.mark.parametrize("dims", [(30, 30), (10, 10, 10)])
def test_descendant_row_property(dims):
    # Sec. 2.1: for a descendant k of j, R_k restricted to columns after C_j lies in R_j.
    p = grid_problem(dims, sigma=1.0, seed=1)
    sym = symbolic(p.n, p.rowptr, p.colind, 32)
    for j in range(sym.M):
        hi = sym.first[j + 1]
        Rj = set(sym.rows[j].tolist())
        for (k, p0, nD) in sym.pairs[j]:
            Rk = sym.rows[k]
            assert np.all(sym.owner[Rk[p0:p0 + nD]] == j)
            tail = Rk[p0 + nD:]
            assert np.all(tail >= hi) and set(tail.tolist()) <= Rj
            assert k < j


def test_nested_dissection_reduces_fill():
    # The point of the ordering (Sec. 2.2): far less fill than the natural
    # (banded) order of a 2D grid.
    n = 48
    p = grid_problem((n, n), unit=True)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    A = p.matrix().toarray()
    fill_nd = np.count_nonzero(np.linalg.cholesky(A[np.ix_(sym.perm, sym.perm)]))
    fill_nat = np.count_nonzero(np.linalg.cholesky(A))
    assert fill_nd < 0.6 * fill_nat


def test_check_pattern_rejects_bad_input():
    rp, ci = path_graph(5)
    check_pattern(5, rp, ci)
    with pytest.raises(ValueError):
        check_pattern(5, rp, ci[::-1].copy())
    bad = ci.copy(); bad[0] = 1            # drop the (0,0) diagonal
    with pytest.raises(ValueError):
        check_pattern(5, rp, bad)
