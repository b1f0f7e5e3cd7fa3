"""Oracle: left-looking supernodal Cholesky, exact and rank-structured (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this module; the product path never does.  Plain FP64 NumPy /
LAPACK, supernodes in ascending order, no blocking or fusion beyond what the
paper states.

Exact mode (``tol == 0``): Algorithm 1 (``factorSupernode``) for every
supernode, with the Schur-complement assembly equations of §2.1: start from
``A(C_j, C_j)`` and ``A(R_j, C_j)`` (the second assignment in Algorithm 1 is
printed with the wrong left-hand side; it initialises the off-diagonal block),
subtract ``scatter(X_D X_D^T)`` and ``scatter(X_O X_D^T)`` for every descendant,
then ``L^D_j = chol(U^D_j)`` and ``L^O_j = U^O_j (L^D_j)^{-T}``.  Its result is
the unique Cholesky factor of the permuted matrix.

Rank-structured mode (``tol > 0``): after Algorithm 1, a separator supernode with
``c_j >= tau_O`` columns and ``r_j > 0`` rows (§3.1, §3.3) is replaced by
``L^O_j ~ V_j U_j^T`` from the randomized range finder of Algorithm 3, applied to
the explicitly formed ``L^O_j``:

1. ``l_j = min(k, ceil(alpha_O sqrt(k) log2 k) + p)``, ``k = min(r_j, c_j)``
   (the rank function of §5.2, used as the number of samples);
2. ``G = randomMatrix(r_j, l_j)``; ``Y = (L^O_j)^T G`` (the product Algorithm 3
   labels ``offDiagonalMultiplyTrans``: a row-space sample);
3. ``s_pow`` power iterations ``Y = (L^O_j)^T (L^O_j Y)``;
4. ``U = makeOrthonormal(Y)`` (Householder QR);
5. ``V = L^O_j U`` (the projection of Algorithm 3);
6. truncation (the paper fixes ranks; this tolerance is an addition): with
   ``V^T V = Z diag(lambda) Z^T`` (descending) and ``sigma_i = sqrt(lambda_i)``,
   keep ``q_j = #{sigma_i > tol sigma_1}`` (``q_j = 0`` when ``sigma_1 = 0``),
   ``U_j = U Z_q``, ``V_j = V Z_q``.

``U_j`` stays orthonormal and ``V_j = L^O_j U_j``, which is the condition of §3.2
under which every later Schur complement stays positive definite.  A compressed
descendant updates its ancestors through ``V_k`` (§3.4, the low-rank product with
``U_k^T U_k = I``).

Implicit products (``Options.implicit``): the same steps 2-5 without forming
``L^O_j`` -- Algorithm 2 (``offdiag_multiply``: ``L^O_j G`` from ``(L^D_j)^{-T} G``,
the block ``A(R_j, C_j)`` and every descendant's two products, a compressed
descendant through ``V_k`` with ``U_prod = U_k^T U_k``, eq. lowRankMult) and its
transpose (``offdiag_multiply_transpose``, the same terms in reverse order), as
Algorithm 3 calls them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .diagonal import HierDiag, diagonal_solve, factor_hierarchical, height, leaf_bounds
from .ordering import SEPARATOR, Symbolic, symbolic
from .philox import gaussian_sample


class NotSPDError(RuntimeError):
    def __init__(self, supernode):
        super().__init__(f"non-positive pivot in supernode {supernode}")
        self.supernode = supernode


@dataclass
class Options:
    leaf_max: int = 64
    tau_O: int = 32
    oversample: int = 10
    power_iters: int = 0
    alpha_O: float = 1.0
    seed: int = 0
    implicit: bool = False   # Algorithm 3 through Algorithm 2 (L^O_j of compressed supernodes never formed)
    keep_lo: bool = False    # explicit path: also keep the dense L^O_j of compressed supernodes (LO_dense)
    tau_D: int = 0           # largest dense diagonal block (0: no diagonal compression)
    alpha_D: float = 0.5     # rank constant of the diagonal blocks, raised by 1.25 on failure (§5.3)


def sample_count(r: int, c: int, alpha: float, p: int) -> int:
    """Rank function of §5.2, ``alpha sqrt(k) log2(k) + p`` with ``k = min(r, c)``,
    rounded up and capped at ``k``."""
    k = min(r, c)
    if k <= 0:
        return 0
    return int(min(k, math.ceil(alpha * math.sqrt(k) * math.log2(k)) + p))


def compressible(sym: Symbolic, j: int, opts: Options, tol: float) -> bool:
    return (tol > 0 and sym.kind[j] == SEPARATOR and sym.c(j) >= opts.tau_O and sym.r(j) > 0)


def hierarchical(sym: Symbolic, j: int, tol: float) -> bool:
    """Whether ``L^D_j`` is stored as a block tree (§4): rank-structured factor and a
    diagonal block tree from the symbolic phase."""
    return tol > 0 and sym.depth is not None and int(sym.depth[j]) > 0


def diag_solve(LD, G: np.ndarray, transpose: bool) -> np.ndarray:
    """``(L^D_j)^{-1} G``, or ``(L^D_j)^{-T} G``: a dense triangular solve, or
    Algorithm 4 for a block tree."""
    if isinstance(LD, HierDiag):
        return diagonal_solve(LD, G, transpose)
    return sla.solve_triangular(LD, G, lower=True, trans="T" if transpose else "N")


@dataclass
class Factor:
    sym: Symbolic
    tol: float
    opts: Options
    LD: list = field(default_factory=list)     # dense L^D_j, or a HierDiag block tree
    LO: list = field(default_factory=list)     # dense L^O_j, or None when compressed
    V: list = field(default_factory=list)
    U: list = field(default_factory=list)
    ell: list = field(default_factory=list)    # samples drawn (0 when not compressed)
    q: list = field(default_factory=list)      # kept rank
    flops: dict = field(default_factory=dict)
    LO_dense: dict = field(default_factory=dict)   # with Options.keep_lo: L^O_j before compression
    Ap: object = None                          # the permuted matrix P A P^T (CSR)
    alpha_D: float = 0.0                       # the diagonal rank constant that succeeded
    restarts: int = 0                          # factorizations restarted with a larger alpha_D

    def offdiag(self, j):
        """The stored off-diagonal operand ``X`` used by ancestors: ``L^O_j`` or ``V_j``."""
        return self.LO[j] if self.LO[j] is not None else self.V[j]

    def dense_L(self):
        """The (approximate) factor as a dense lower-triangular matrix."""
        n = self.sym.n
        L = np.zeros((n, n))
        for j in range(self.sym.M):
            lo, hi = int(self.sym.first[j]), int(self.sym.first[j + 1])
            L[lo:hi, lo:hi] = self.LD[j].dense() if isinstance(self.LD[j], HierDiag) else self.LD[j]
            R = self.sym.rows[j]
            if R.size:
                L[np.ix_(R, np.arange(lo, hi))] = (self.LO[j] if self.LO[j] is not None
                                                   else self.V[j] @ self.U[j].T)
        return L


def permuted_matrix(sym: Symbolic, n, rowptr, colind, values) -> sp.csr_matrix:
    A = sp.csr_matrix((np.asarray(values, dtype=np.float64), colind, rowptr), shape=(n, n))
    return A[sym.perm][:, sym.perm].tocsr()


def _truncate(V: np.ndarray, U: np.ndarray, tol: float):
    """Keep the directions of ``V`` with singular value ``> tol sigma_1``: eigen-
    decomposition of ``V^T V`` (descending); returns ``V Z_q, U Z_q, q``."""
    lam, Z = np.linalg.eigh(V.T @ V)
    order = np.argsort(lam)[::-1]
    lam, Z = lam[order], Z[:, order]
    sig = np.sqrt(np.maximum(lam, 0.0))
    q = 0 if sig.size == 0 or sig[0] == 0.0 else int(np.count_nonzero(sig > tol * sig[0]))
    return V @ Z[:, :q], U @ Z[:, :q], q


def compress(LO: np.ndarray, j: int, opts: Options, tol: float):
    """Algorithm 3 on an explicit ``L^O_j`` followed by the truncation above."""
    r, c = LO.shape
    ell = sample_count(r, c, opts.alpha_O, opts.oversample)
    G = gaussian_sample(opts.seed, j, r, ell)
    Y = LO.T @ G
    for _ in range(opts.power_iters):
        Y = LO.T @ (LO @ Y)
    U, _ = np.linalg.qr(Y)
    V = LO @ U
    Vq, Uq, q = _truncate(V, U, tol)
    return Vq, Uq, ell, q


def _pair_rows(sym: Symbolic, j: int, k: int, p0: int, nD: int):
    """Rows of descendant ``k``'s operand that meet supernode ``j``: ``C_j``-local
    positions of ``R^D_{k->j}`` and ``R_j``-local positions of ``R^O_{k->j}`` (§2.1)."""
    lo = int(sym.first[j])
    Rk = sym.rows[k]
    return Rk[p0:p0 + nD] - lo, np.searchsorted(sym.rows[j], Rk[p0 + nD:])


def _descendant_term(F: Factor, k: int, p0: int, nD: int, G: np.ndarray, transpose: bool):
    """One descendant's product of Algorithm 2 (lines 10-11, or eq. lowRankMult for a
    compressed ``k``): ``L^O_k(r^O) [L^O_k(r^D)]^T G`` (``G`` on the ``r^D`` rows), or
    with ``transpose`` ``L^O_k(r^D) [L^O_k(r^O)]^T G`` (``G`` on the ``r^O`` rows)."""
    if F.LO[k] is not None:
        X = F.LO[k][p0:]
        XD, XO = X[:nD], X[nD:]
        return XD @ (XO.T @ G) if transpose else XO @ (XD.T @ G)
    Vk = F.V[k][p0:]
    VD, VO = Vk[:nD], Vk[nD:]
    Uprod = F.U[k].T @ F.U[k]
    return VD @ (Uprod @ (VO.T @ G)) if transpose else VO @ (Uprod @ (VD.T @ G))


def offdiag_multiply(F: Factor, j: int, G: np.ndarray) -> np.ndarray:
    """Algorithm 2 (offDiagonalMultiply): ``L^O_j G`` for ``G`` of ``c_j`` rows, from
    ``(L^D_j)^{-T} G``, the block ``A(R_j, C_j)`` and the descendants of ``j``; needs
    ``L^D_j`` and the factored descendants, never ``L^O_j`` itself."""
    sym, Ap = F.sym, F.Ap
    lo, hi = int(sym.first[j]), int(sym.first[j + 1])
    R = sym.rows[j]
    G = diag_solve(F.LD[j], G, transpose=True)
    W = Ap[R][:, lo:hi] @ G
    for (k, p0, nD) in sym.pairs[j]:
        cols, orow = _pair_rows(sym, j, k, p0, nD)
        if orow.size:
            W[orow] -= _descendant_term(F, k, p0, nD, G[cols], transpose=False)
    return W


def offdiag_multiply_transpose(F: Factor, j: int, G: np.ndarray) -> np.ndarray:
    """The transpose product ``(L^O_j)^T G`` for ``G`` of ``r_j`` rows (the function
    the paper names offDiagonalMultiplyTranspose): ``A(R_j, C_j)^T G`` minus every
    descendant's term gathered from the ``r^O`` rows and scattered to the ``r^D``
    columns, then ``(L^D_j)^{-1}`` applied."""
    sym, Ap = F.sym, F.Ap
    lo, hi = int(sym.first[j]), int(sym.first[j + 1])
    R = sym.rows[j]
    S = Ap[R][:, lo:hi].T @ G
    for (k, p0, nD) in sym.pairs[j]:
        cols, orow = _pair_rows(sym, j, k, p0, nD)
        if orow.size:
            S[cols] -= _descendant_term(F, k, p0, nD, G[orow], transpose=True)
    return diag_solve(F.LD[j], S, transpose=False)


def compress_implicit(F: Factor, j: int, opts: Options, tol: float):
    """Algorithm 3 through Algorithm 2 and its transpose, then the truncation."""
    sym = F.sym
    r, c = sym.r(j), sym.c(j)
    ell = sample_count(r, c, opts.alpha_O, opts.oversample)
    G = gaussian_sample(opts.seed, j, r, ell)
    Y = offdiag_multiply_transpose(F, j, G)
    for _ in range(opts.power_iters):
        Y = offdiag_multiply_transpose(F, j, offdiag_multiply(F, j, Y))
    U, _ = np.linalg.qr(Y)
    V = offdiag_multiply(F, j, U)
    Vq, Uq, q = _truncate(V, U, tol)
    return Vq, Uq, ell, q


def _all_blocks_exact(sym: Symbolic, alpha_D: float, opts: Options) -> bool:
    """Whether every block of every diagonal block tree is sampled at full rank."""
    for j in range(sym.M):
        d = int(sym.depth[j]) if sym.depth is not None else 0
        if d == 0:
            continue
        b = leaf_bounds(sym.c(j), d)
        H = HierDiag(c=sym.c(j), d=d, bounds=b)
        for s in range(2, H.nblocks + 1, 2):
            (ca, cb), (ra, rb) = H.cols(s), H.rows(s)
            if sample_count(rb - ra, cb - ca, alpha_D, opts.oversample) < min(rb - ra, cb - ca):
                return False
    return True


def factor(sym: Symbolic, n, rowptr, colind, values, tol: float = 0.0,
           opts: Options | None = None, stop_after: int | None = None, progress=None) -> Factor:
    """Factor supernodes ``0 .. M-1`` (or the first ``stop_after``) in order.
    ``progress(j, M)``, if given, is called after each supernode (reporting only).

    With diagonal block trees the factorization may meet a Schur complement that is
    not positive definite; it then restarts with ``alpha_D`` multiplied by 1.25
    (§5.3), until it succeeds or every diagonal block is already sampled at full rank
    (then the factor is exact in those blocks and the failure is the matrix's)."""
    opts = opts or Options()
    use_tree = any(hierarchical(sym, j, tol) for j in range(sym.M))
    alpha = opts.alpha_D
    restarts = 0
    while True:
        try:
            F = _factor_once(sym, n, rowptr, colind, values, tol, opts, alpha, stop_after, progress)
        except NotSPDError:
            if not use_tree or _all_blocks_exact(sym, alpha, opts):
                raise
            alpha *= 1.25
            restarts += 1
            continue
        F.alpha_D = alpha if use_tree else 0.0
        F.restarts = restarts
        return F


def _factor_once(sym: Symbolic, n, rowptr, colind, values, tol, opts, alpha_D, stop_after,
                 progress) -> Factor:
    Ap = permuted_matrix(sym, n, rowptr, colind, values)
    F = Factor(sym=sym, tol=tol, opts=opts, Ap=Ap)
    M = sym.M if stop_after is None else min(sym.M, stop_after)
    fl = dict(potrf=0.0, trsm=0.0, update=0.0, sample=0.0, orth=0.0, trunc=0.0)
    for j in range(M):
        lo, hi = int(sym.first[j]), int(sym.first[j + 1])
        c = hi - lo
        R = sym.rows[j]
        comp = compressible(sym, j, opts, tol)
        implicit = comp and opts.implicit   # the off-diagonal block is only used through Algorithm 2
        tree = hierarchical(sym, j, tol)    # L^D_j by Algorithms 4-6 (its leaves form their own Schur blocks)
        # Initialise the Schur complement blocks (Algorithm 1)
        UD = Ap[lo:hi][:, lo:hi].toarray() if not tree else None
        UO = Ap[R][:, lo:hi].toarray() if (R.size and not implicit) else np.zeros((0, c))
        for (k, p0, nD) in sym.pairs[j]:
            X = F.offdiag(k)[p0:]
            XD = X[:nD]
            Rk = sym.rows[k]
            cols = Rk[p0:p0 + nD] - lo                       # R^D_{k->j} within C_j
            orow = np.searchsorted(R, Rk[p0 + nD:])          # R^O_{k->j} within R_j
            if not tree:
                UD[np.ix_(cols, cols)] -= XD @ XD.T
            if orow.size and not implicit:
                UO[np.ix_(orow, cols)] -= X[nD:] @ XD.T
            fl["update"] += 2.0 * X.shape[1] * (nD * (nD + 1) / 2.0 + float(X.shape[0] - nD) * nD)
        if tree:
            d = int(sym.depth[j])
            try:
                LD = factor_hierarchical(F, j, leaf_bounds(c, d), d, alpha_D, opts, j)
            except np.linalg.LinAlgError:
                raise NotSPDError(j) from None
        else:
            try:
                LD = np.linalg.cholesky(UD)
            except np.linalg.LinAlgError:
                raise NotSPDError(j) from None
            if not np.all(np.isfinite(LD)):
                raise NotSPDError(j)
        LO = (diag_solve(LD, UO.T, transpose=False).T if (R.size and not implicit)
              else np.zeros((0, c)))
        fl["potrf"] += c ** 3 / 3.0
        if not implicit:
            fl["trsm"] += float(R.size) * c * c
        F.LD.append(LD)
        if comp:
            if implicit:
                V, U, ell, q = compress_implicit(F, j, opts, tol)
            else:
                if opts.keep_lo:
                    F.LO_dense[j] = LO
                V, U, ell, q = compress(LO, j, opts, tol)
            F.LO.append(None); F.V.append(V); F.U.append(U); F.ell.append(ell); F.q.append(q)
            fl["sample"] += 4.0 * R.size * c * ell * (1 + opts.power_iters)
            fl["orth"] += 2.0 * c * ell * ell
            fl["trunc"] += 2.0 * R.size * ell * ell
        else:
            F.LO.append(LO); F.V.append(None); F.U.append(None); F.ell.append(0); F.q.append(0)
        if progress is not None:
            progress(j, M)
    F.flops = fl
    return F


def analyze_and_factor(n, rowptr, colind, values, tol=0.0, opts: Options | None = None, coords=None):
    opts = opts or Options()
    sym = symbolic(n, rowptr, colind, opts.leaf_max, opts.tau_D, coords)
    return factor(sym, n, rowptr, colind, values, tol, opts)
