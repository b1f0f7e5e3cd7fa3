"""Oracle: hierarchical compression of diagonal blocks (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this module; the product path never does.  Plain FP64 NumPy /
LAPACK, written from §4.1-4.2 and §5.2-5.3 of the paper.

What is computed
----------------
* Ordering inside a large separator (§4.1): the positions of its indices are split
  recursively in two, along the longest side of their bounding box, until every
  piece has at most ``tau_D`` indices; the pieces, in the order of the recursion,
  become the dense diagonal blocks (leaves) of ``L^D_j``.
* Block structure (§4.1-4.2): the blocks of ``L^D_j`` are the nodes of a complete
  binary tree numbered in order (leaves odd, the root ``2^d``).  A leaf ``s`` is a
  dense lower-triangular block on its own index range; an internal node ``s`` is
  the block ``L(R_s, C_s) ~ V_s U_s^T`` whose columns ``C_s`` are the indices of its
  left subtree and whose rows ``R_s`` are those of its right subtree.
* ``diagonal_solve`` (Algorithm 4): a solve with the sub-factor rooted at ``s``.
* ``diagonal_multiply`` (Algorithm 5) and its transpose: ``L(R_s, C_s) G`` without
  forming the block -- a solve with the left subtree's factor, the matrix block,
  every descendant of ``j`` and every earlier block of ``L^D_j`` above ``s``.
* ``approximate_diagonal_block``: the randomized range finder of Algorithm 3
  driven by the two products above, at the rank of the §5.2 rank function with
  ``alpha_D`` (the paper fixes this rank; no truncation follows).
* ``factor_diagonal`` (Algorithm 6): a leaf's Schur complement (matrix block,
  descendants, earlier blocks above it) and its Cholesky factor.

Readings (the paper is terse or misprinted here):
* The tree is complete: every leaf sits at depth ``d = ceil(log2(c / tau_D))``, which
  is what the in-order labels of §4.2 presuppose.  A piece of ``m`` indices splits
  into its first ``m // 2`` (smaller coordinates) and the rest; the sort along an
  axis is stable; of equally long sides the first axis (x, then y, then z) wins.
* The root of the seven-block example has children 2 and 6 (the text prints 3).
* Algorithm 4's two branches are printed exchanged: with ``transpose`` the solve is
  with ``L^T`` (backward: the right part first, then ``G_1 -= U_s (V_s^T G_2)``);
  otherwise with ``L`` (forward: the left part first, then ``G_2 -= V_s (U_s^T G_1)``).
  Each leaf applies ``D_s^{-T}`` or ``D_s^{-1}`` as the flag says.
* Algorithm 6's descendant term uses each descendant's off-diagonal factor rows
  that fall in the leaf (``L^O_k``, or ``V_k`` when compressed; the printed
  ``L^D_k`` has no rows in ``C_j``), and its loop over earlier blocks moves to the
  parent on every pass, as Algorithm 5's does.
* A separator supernode is hierarchical when the factor is rank-structured
  (``tol > 0``), ``tau_D > 0`` and it has more than ``tau_D`` columns.
* Sample of block ``s`` of supernode ``j``: the Philox stream of ``j`` with third
  counter word ``4 + s``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .philox import gaussian_sample


# ---------------------------------------------------------------- ordering (§4.1)

def split_depth(c: int, tau_D: int) -> int:
    """Depth ``d`` of the complete tree over ``c`` indices: the smallest ``d`` whose
    pieces (``floor`` or ``ceil`` of ``c / 2^d`` indices) have at most ``tau_D``."""
    if tau_D <= 0:
        return 0
    d = 0
    while (c + (1 << d) - 1) >> d > tau_D:
        d += 1
    return d


def coordinate_order(xyz: np.ndarray, d: int) -> np.ndarray:
    """Order of the rows of ``xyz`` (m x 3) after ``d`` rounds of splitting each piece
    in two along the longest side of its bounding box (§4.1).  Returns positions."""
    order = np.arange(xyz.shape[0])

    def rec(idx, depth):
        if depth == 0 or idx.size < 2:
            return idx
        P = xyz[idx]
        ext = P.max(axis=0) - P.min(axis=0)
        axis = int(np.argmax(ext))            # first of the longest sides
        idx = idx[np.argsort(P[:, axis], kind="stable")]
        h = idx.size // 2
        return np.concatenate((rec(idx[:h], depth - 1), rec(idx[h:], depth - 1)))

    return rec(order, d)


def leaf_bounds(c: int, d: int) -> np.ndarray:
    """Boundaries of the ``2^d`` leaves of a piece of ``c`` indices (first half
    ``m // 2`` at every split), as ``2^d + 1`` offsets."""
    def rec(lo, m, depth):
        if depth == 0:
            return [lo]
        h = m // 2
        return rec(lo, h, depth - 1) + rec(lo + h, m - h, depth - 1)

    return np.array(rec(0, c, d) + [c], dtype=np.int64)


# ---------------------------------------------------------------- the block tree (§4.2)

def height(s: int) -> int:
    """Height of in-order node ``s`` (leaves 0): its number of trailing zero bits."""
    return (s & -s).bit_length() - 1


def children(s: int):
    h = height(s)
    return s - (1 << (h - 1)), s + (1 << (h - 1))


def parent(s: int, d: int):
    """In-order parent of ``s`` in the complete tree of depth ``d`` (None at the root)."""
    h = height(s)
    if h == d:
        return None
    return s + (1 << h) if ((s >> (h + 1)) & 1) == 0 else s - (1 << h)


@dataclass
class HierDiag:
    """``L^D_j`` of a hierarchical supernode: leaf factors and low-rank blocks."""
    c: int
    d: int
    bounds: np.ndarray                  # leaf boundaries (2^d + 1), relative to C_j
    D: dict = field(default_factory=dict)   # leaf s -> dense lower-triangular block
    V: dict = field(default_factory=dict)   # internal s -> V_s (|R_s| x l_s)
    U: dict = field(default_factory=dict)   # internal s -> U_s (|C_s| x l_s)
    ell: dict = field(default_factory=dict)

    @property
    def nblocks(self):
        return (1 << (self.d + 1)) - 1

    def span(self, s: int):
        """Index range ``[lo, hi)`` (relative to ``C_j``) of the subtree rooted at ``s``."""
        h = height(s)
        first_leaf = (s - ((1 << h) - 1)) // 2      # leaves numbered 0 .. 2^d - 1
        return int(self.bounds[first_leaf]), int(self.bounds[first_leaf + (1 << h)])

    def cols(self, s: int):
        """``C_s``: the left subtree's range (a leaf: its own range)."""
        if height(s) == 0:
            return self.span(s)
        return self.span(children(s)[0])

    def rows(self, s: int):
        """``R_s``: the right subtree's range (a leaf: its own range)."""
        if height(s) == 0:
            return self.span(s)
        return self.span(children(s)[1])

    def dense(self) -> np.ndarray:
        """The approximate ``L^D_j`` written out densely."""
        L = np.zeros((self.c, self.c))
        for s in range(1, self.nblocks + 1):
            if height(s) == 0:
                a, b = self.span(s)
                L[a:b, a:b] = self.D[s]
            else:
                (ca, cb), (ra, rb) = self.cols(s), self.rows(s)
                L[ra:rb, ca:cb] = self.V[s] @ self.U[s].T
        return L


def diagonal_solve(H: HierDiag, G: np.ndarray, transpose: bool, s: int | None = None) -> np.ndarray:
    """Algorithm 4: solve with the sub-factor of ``L^D_j`` rooted at block ``s`` (the
    whole of it when ``s`` is None); ``G`` has that subtree's rows."""
    if s is None:
        s = 1 << H.d
    if height(s) == 0:
        return sla.solve_triangular(H.D[s], G, lower=True, trans="T" if transpose else "N")
    s1, s2 = children(s)
    nc = H.cols(s)[1] - H.cols(s)[0]
    G1, G2 = G[:nc], G[nc:]
    if transpose:       # backward substitution with L^T
        G2 = diagonal_solve(H, G2, True, s2)
        G1 = G1 - H.U[s] @ (H.V[s].T @ G2)
        G1 = diagonal_solve(H, G1, True, s1)
    else:               # forward substitution with L
        G1 = diagonal_solve(H, G1, False, s1)
        G2 = G2 - H.V[s] @ (H.U[s].T @ G1)
        G2 = diagonal_solve(H, G2, False, s2)
    return np.concatenate((G1, G2), axis=0)


# ---------------------------------------------------------------- products and factors

def _desc_rows(F, j: int, k: int, p0: int, nD: int):
    """Descendant ``k``'s operand rows inside ``C_j``: positions relative to ``C_j``
    and the operand (``L^O_k`` rows, or ``V_k`` rows) with its ``U_prod``."""
    sym = F.sym
    lo = int(sym.first[j])
    pos = sym.rows[k][p0:p0 + nD] - lo
    if F.LO[k] is not None:
        return pos, F.LO[k][p0:p0 + nD], None
    return pos, F.V[k][p0:p0 + nD], F.U[k].T @ F.U[k]


def _in_range(pos: np.ndarray, a: int, b: int):
    m = (pos >= a) & (pos < b)
    return m, pos[m] - a


def diagonal_multiply(F, j: int, H: HierDiag, G: np.ndarray, s: int, transpose: bool = False):
    """Algorithm 5 (``transpose`` False): ``L(R_s, C_s) G`` for ``G`` of ``|C_s|`` rows;
    its transpose (``transpose`` True): ``L(R_s, C_s)^T G`` for ``G`` of ``|R_s|`` rows --
    the same terms in reverse order, the left subtree's solve applied last."""
    sym, Ap = F.sym, F.Ap
    lo = int(sym.first[j])
    (ca, cb), (ra, rb) = H.cols(s), H.rows(s)
    s1 = children(s)[0]
    if not transpose:
        G = diagonal_solve(H, G, True, s1)
        W = Ap[lo + ra:lo + rb][:, lo + ca:lo + cb] @ G
    else:
        W = Ap[lo + ra:lo + rb][:, lo + ca:lo + cb].T @ G
    W = np.array(W)
    for (k, p0, nD) in sym.pairs[j]:
        pos, X, Uprod = _desc_rows(F, j, k, p0, nD)
        mc, pc = _in_range(pos, ca, cb)
        mr, pr = _in_range(pos, ra, rb)
        if not mc.any() or not mr.any():
            continue
        XC, XR = X[mc], X[mr]
        if not transpose:
            T = XC.T @ G[pc]
            if Uprod is not None:
                T = Uprod @ T
            W[pr] -= XR @ T
        else:
            T = XR.T @ G[pr]
            if Uprod is not None:
                T = Uprod @ T
            W[pc] -= XC @ T
    p = parent(s, H.d)
    while p is not None:
        if p < s:
            base = H.rows(p)[0]
            Rsub = np.arange(ra, rb) - base
            Csub = np.arange(ca, cb) - base
            Uprod = H.U[p].T @ H.U[p]
            if not transpose:
                T = H.V[p][Csub].T @ G
                W -= H.V[p][Rsub] @ (Uprod @ T)
            else:
                T = H.V[p][Rsub].T @ G
                W -= H.V[p][Csub] @ (Uprod @ T)
        p = parent(p, H.d)
    if transpose:
        W = diagonal_solve(H, W, False, s1)
    return W


def approximate_diagonal_block(F, j: int, H: HierDiag, s: int, alpha_D: float, oversample: int,
                               power_iters: int, seed: int, sn_key: int):
    """Algorithm 3's range finder on the block ``L(R_s, C_s)`` through the products
    above, at ``l = min(k, ceil(alpha_D sqrt(k) log2 k) + p)``, ``k = min(|R_s|, |C_s|)``."""
    from .factor import sample_count
    (ca, cb), (ra, rb) = H.cols(s), H.rows(s)
    nr, nc = rb - ra, cb - ca
    ell = sample_count(nr, nc, alpha_D, oversample)
    Om = gaussian_sample(seed, sn_key, nr, ell, c2=4 + s)
    Y = diagonal_multiply(F, j, H, Om, s, transpose=True)
    for _ in range(power_iters):
        Y = diagonal_multiply(F, j, H, diagonal_multiply(F, j, H, Y, s), s, transpose=True)
    U, _ = np.linalg.qr(Y)
    V = diagonal_multiply(F, j, H, U, s)
    H.V[s], H.U[s], H.ell[s] = V, U, ell
    return ell


def factor_diagonal(F, j: int, H: HierDiag, s: int):
    """Algorithm 6: the dense leaf ``s`` of ``L^D_j`` (raises LinAlgError when its
    Schur complement is not positive definite)."""
    sym, Ap = F.sym, F.Ap
    lo = int(sym.first[j])
    a, b = H.span(s)
    S = Ap[lo + a:lo + b][:, lo + a:lo + b].toarray()
    for (k, p0, nD) in sym.pairs[j]:
        pos, X, Uprod = _desc_rows(F, j, k, p0, nD)
        m, p = _in_range(pos, a, b)
        if not m.any():
            continue
        Xs = X[m]
        upd = Xs @ Xs.T if Uprod is None else Xs @ (Uprod @ Xs.T)
        S[np.ix_(p, p)] -= upd
    q = parent(s, H.d)
    while q is not None:
        if q < s:
            sub = np.arange(a, b) - H.rows(q)[0]
            Uprod = H.U[q].T @ H.U[q]
            S -= H.V[q][sub] @ (Uprod @ H.V[q][sub].T)
        q = parent(q, H.d)
    D = np.linalg.cholesky(S)
    if not np.all(np.isfinite(D)):
        raise np.linalg.LinAlgError("non-finite leaf factor")
    H.D[s] = D


def factor_hierarchical(F, j: int, bounds: np.ndarray, d: int, alpha_D: float, opts, sn_key: int):
    """Every block of ``L^D_j`` in increasing order: leaves by Algorithm 6, the
    blocks between them by the range finder (§4.2)."""
    H = HierDiag(c=int(bounds[-1]), d=d, bounds=bounds)
    for s in range(1, H.nblocks + 1):
        if height(s) == 0:
            factor_diagonal(F, j, H, s)
        else:
            approximate_diagonal_block(F, j, H, s, alpha_D, opts.oversample, opts.power_iters,
                                       opts.seed, sn_key)
    return H
