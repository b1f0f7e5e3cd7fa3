"""Pins of the oracle's numeric factorization, preconditioner, PCG and adjoint (CPU only)."""
import json
import math

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import golden_path
from oracle.adjoint import dense_adjoint, grad_faces, grad_values
from oracle.factor import NotSPDError, Options, compress, factor, sample_count
from oracle.ordering import symbolic
from oracle.philox import gaussian_sample, philox4x32_10
from oracle.solve import apply_preconditioner, pcg, solve
from workloads import grid_problem

SMALL = [((8, 8), 0.0), ((16, 16), 1.0), ((4, 4, 4), 0.0), ((7, 6, 5), 1.5), ((8, 8, 8), 1.0)]


def _prob(dims, sigma, seed=1):
    return grid_problem(dims, sigma=sigma, seed=seed, unit=(sigma == 0.0))


@pytest.mark.parametrize("dims,sigma", SMALL)
@pytest.mark.parametrize("leaf", [8, 64])
def test_exact_factor_is_dense_cholesky(dims, sigma, leaf):
    # Sec. 1: the Cholesky factor is unique, so the supernodal left-looking
    # result must equal LAPACK's dense factor of the permuted matrix.
    p = _prob(dims, sigma)
    sym = symbolic(p.n, p.rowptr, p.colind, leaf)
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0, Options(leaf_max=leaf))
    Ap = p.matrix()[sym.perm][:, sym.perm].toarray()
    L = F.dense_L()
    Lref = np.linalg.cholesky(Ap)
    assert np.abs(L - Lref).max() <= 1e-13 * np.abs(Lref).max()
    assert np.linalg.norm(Ap - L @ L.T) / np.linalg.norm(Ap) <= 1e-12


def test_exact_preconditioner_is_inverse_and_pcg_one_step():
    p = _prob((9, 8, 7), 1.0)
    sym = symbolic(p.n, p.rowptr, p.colind, 32)
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0)
    A = p.matrix()
    z = apply_preconditioner(F, p.b)
    x = np.linalg.solve(A.toarray(), p.b)
    assert np.linalg.norm(z - x) <= 1e-12 * np.linalg.norm(x)
    res = solve(F, A, p.b, rtol=1e-12)
    assert res.converged and res.iters <= 2 and res.true_residual <= 1e-12


def test_sample_count_rank_function():
    # Sec. 5.2: alpha sqrt(k) log2(k) + p, k = min(m, n); capped at k.
    assert sample_count(200, 64, 1.0, 10) == 8 * 6 + 10
    assert sample_count(100, 300, 1.0, 10) == math.ceil(10 * math.log2(100)) + 10
    assert sample_count(5, 40, 1.0, 10) == 5
    assert sample_count(1, 1, 1.0, 10) == 1
    assert sample_count(1000, 4000, 0.5, 5) == math.ceil(0.5 * math.sqrt(1000) * math.log2(1000)) + 5


def test_compress_recovers_exact_low_rank():
    rng = np.random.default_rng(0)
    B = rng.standard_normal((300, 6)) @ rng.standard_normal((6, 80))
    V, U, ell, q = compress(B, 7, Options(seed=11), 1e-8)
    assert q == 6 and ell == sample_count(300, 80, 1.0, 10)
    assert np.abs(U.T @ U - np.eye(q)).max() <= 1e-13
    assert np.abs(V - B @ U).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.norm(B - V @ U.T) <= 1e-12 * np.linalg.norm(B)


def test_compress_error_within_range_finder_bound():
    # Randomized range finder bound (Halko, Martinsson, Tropp; cited by Sec. 3.4):
    # ||B - B U U^T|| <= (1 + 11 sqrt(k + p) sqrt(min(m, n))) sigma_{k+1}, plus the
    # truncation, which drops directions with sigma <= tol sigma_1.
    rng = np.random.default_rng(1)
    m, n = 400, 120
    Q1, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = 0.7 ** np.arange(n)
    B = (Q1 * s) @ Q2.T
    tol = 1e-3
    V, U, ell, q = compress(B, 3, Options(seed=5), tol)
    k = ell - 10
    bound = (1 + 11 * math.sqrt(ell) * math.sqrt(n)) * s[k] + tol * s[0]
    err = np.linalg.norm(B - V @ U.T, 2)
    assert err <= bound
    # and truncation kept exactly the singular values above the tolerance
    assert abs(q - np.count_nonzero(s > tol * s[0])) <= 1


def test_power_iterations_reach_best_rank_ell_error():
    # Algorithm 3's power iterations are subspace iteration on B^T B: with a spectral
    # gap after the l-th singular value the sampled subspace converges to the top-l
    # right singular subspace, so ||B - V U^T||_2 falls to sigma_{l+1}, the smallest
    # any rank-l approximation reaches (Eckart-Young-Mirsky).  Without the iterations
    # the same sample stays about twice as far off, so a dropped or mis-transposed
    # product fails one side or the other.
    rng = np.random.default_rng(2)
    m, n = 400, 120
    ell = sample_count(m, n, 1.0, 10)
    assert ell == 86
    Q1, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.where(np.arange(n) < ell, 1.0, 0.5) * 0.999 ** np.arange(n)
    B = (Q1 * s) @ Q2.T
    err = {}
    for q in (0, 6):
        V, U, l, k = compress(B, 4, Options(seed=6, power_iters=q), 0.0)
        assert l == ell and k == ell
        assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-12
        assert np.abs(V - B @ U).max() <= 1e-12 * s[0]
        err[q] = np.linalg.norm(B - V @ U.T, 2)
        assert err[q] >= s[ell] * (1 - 1e-12)
    assert err[6] <= s[ell] * (1 + 1e-4)
    assert err[0] >= 1.5 * s[ell]


@pytest.mark.parametrize("dims,sigma", [((10, 10, 10), 1.0), ((40, 40), 1.0), ((12, 11, 10), 1.5)])
def test_full_sampling_reproduces_exact_factor(dims, sigma):
    # With l_j = min(r_j, c_j) samples and nothing truncated, V_j U_j^T = L^O_j,
    # so the rank-structured path must give the exact factor (Sec. 3.2).
    p = _prob(dims, sigma)
    opts = Options(leaf_max=32, tau_O=8, alpha_O=1e9)
    sym = symbolic(p.n, p.rowptr, p.colind, 32)
    Fe = factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0, opts)
    Fc = factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-13, opts)
    assert any(e > 0 for e in Fc.ell)
    Le, Lc = Fe.dense_L(), Fc.dense_L()
    assert np.abs(Le - Lc).max() <= 1e-11 * np.abs(Le).max()


@pytest.mark.parametrize("dims,sigma,tol", [((12, 12, 12), 1.0, 1e-2), ((14, 13, 12), 1.5, 1e-1),
                                            ((64, 64), 1.0, 1e-2)])
def test_compressed_invariants_and_pd(dims, sigma, tol):
    p = _prob(dims, sigma, seed=7)
    opts = Options(leaf_max=64, tau_O=16, seed=9)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, tol, opts)   # never NotSPD (Sec. 3.2)
    nc = 0
    for j in range(sym.M):
        assert np.all(np.diag(F.LD[j]) > 0)
        if F.U[j] is not None:
            nc += 1
            q = F.q[j]
            assert F.U[j].shape == (sym.c(j), q) and F.V[j].shape == (sym.r(j), q)
            assert np.abs(F.U[j].T @ F.U[j] - np.eye(q)).max() <= 1e-12
    assert nc > 0
    # The preconditioner is symmetric positive definite.
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal(p.n), rng.standard_normal(p.n)
    Mu, Mv = apply_preconditioner(F, u), apply_preconditioner(F, v)
    assert abs(Mu @ v - u @ Mv) <= 1e-12 * abs(Mu @ v) + 1e-12 * np.linalg.norm(Mu) * np.linalg.norm(v)
    assert u @ Mu > 0 and v @ Mv > 0


def test_compressed_v_is_projection_of_exact_block():
    # V_j = L^O_j U_j for the block the supernode actually formed: rerun compress
    # on a supernode's block and check the projection identity.
    p = _prob((12, 12, 12), 1.0)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0)
    j = max(range(sym.M), key=lambda t: sym.c(t) * (sym.r(t) > 0))
    V, U, ell, q = compress(F.LO[j], j, Options(), 1e-2)
    assert np.abs(V - F.LO[j] @ U).max() <= 1e-13 * np.abs(F.LO[j]).max()


def test_indefinite_matrix_raises_not_spd():
    p = _prob((6, 6, 6), 1.0)
    vals = p.values.copy()
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    d = np.nonzero(rows == p.colind)[0]
    vals[d[100]] = -vals[d[100]]
    sym = symbolic(p.n, p.rowptr, p.colind, 16)
    with pytest.raises(NotSPDError) as e:
        factor(sym, p.n, p.rowptr, p.colind, vals, 0.0)
    # the failing supernode is the one holding the flipped column, or an ancestor
    j0 = sym.owner[sym.iperm[100]]
    anc = [j0]
    while sym.parent[anc[-1]] >= 0:
        anc.append(int(sym.parent[anc[-1]]))
    assert e.value.supernode in anc


@pytest.mark.parametrize("dims,sigma", [((16, 16, 16), 1.0), ((96, 96), 1.5)])
def test_pcg_manufactured_solution(dims, sigma):
    p = _prob(dims, sigma, seed=5)
    A = p.matrix()
    x_star = np.random.default_rng(3).standard_normal(p.n)
    b = A @ x_star
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-2, Options(seed=2))
    res = solve(F, A, b, rtol=1e-10)
    assert res.converged and res.true_residual <= 1e-9
    # forward error bounded by kappa(A) times the residual
    ev = np.linalg.eigvalsh(A.toarray()) if p.n <= 5000 else None
    kappa = ev[-1] / ev[0] if ev is not None else 1e6
    assert np.linalg.norm(res.x - x_star) <= 2 * kappa * 1e-9 * np.linalg.norm(x_star)


def test_pcg_identity_preconditioner_is_plain_cg():
    # With M = I, PCG is textbook CG, which in exact arithmetic terminates after at
    # most as many steps as A has distinct eigenvalues.  The unit 6 x 6 5-point
    # Laplacian has eigenvalues 4 - 2 cos(i pi/7) - 2 cos(j pi/7), i, j = 1..6.
    p = grid_problem((6, 6), unit=True)
    A = p.matrix()
    t = 2 * np.cos(np.arange(1, 7) * np.pi / 7)
    distinct = np.unique(np.round(4 - t[:, None] - t[None, :], 9)).size
    res = pcg(A, p.b, lambda v: v.copy(), rtol=1e-12, max_iter=100)
    assert res.converged and res.iters <= distinct
    assert abs(res.iters - distinct) <= 1


def test_philox_known_answer_vectors():
    g = json.load(open(golden_path("philox4x32_10_kat.json")))
    for v in g["vectors"]:
        c = [int(x, 16) for x in v["ctr"]]
        k = [int(x, 16) for x in v["key"]]
        out = philox4x32_10(*c, *k)
        assert [int(o) for o in out] == [int(x, 16) for x in v["out"]]


def test_gaussian_sample_moments_and_layout():
    G = gaussian_sample(123, 4, 2000, 250)
    assert G.shape == (2000, 250)
    assert abs(G.mean()) < 0.01 and abs(G.var() - 1.0) < 0.01
    # distinct supernodes and seeds give distinct streams; the layout is by entry
    assert not np.allclose(G[:5, :5], gaussian_sample(123, 5, 5, 5))
    assert np.array_equal(G[:7, :9], gaussian_sample(123, 4, 7, 9))


def test_adjoint_matches_finite_differences():
    p = grid_problem((3, 3, 3), sigma=1.0, seed=4)
    x, lam, loss = dense_adjoint(p.matrix().toarray(), p.b, p.x_target)
    gv = grad_values(p.rowptr, p.colind, lam, x)
    gf = grad_faces(p.face_i, p.face_j, lam, x)
    assert np.allclose(gf, p.value_map.T @ gv, rtol=1e-12, atol=1e-14)
    h = 1e-6
    coef = p.coef.ravel()
    for f in range(coef.size):
        cp, cm = coef.copy(), coef.copy()
        cp[f] += h; cm[f] -= h
        Lp = dense_adjoint(sp.csr_matrix((p.values_from_coef(cp), p.colind, p.rowptr)).toarray(),
                           p.b, p.x_target)[2]
        Lm = dense_adjoint(sp.csr_matrix((p.values_from_coef(cm), p.colind, p.rowptr)).toarray(),
                           p.b, p.x_target)[2]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gf[f]) <= 1e-6 * max(1.0, abs(gf[f]))
    # dL/db = lambda
    e = np.zeros(p.n); e[5] = 1.0
    Lp = dense_adjoint(p.matrix().toarray(), p.b + h * e, p.x_target)[2]
    Lm = dense_adjoint(p.matrix().toarray(), p.b - h * e, p.x_target)[2]
    assert abs((Lp - Lm) / (2 * h) - lam[5]) <= 1e-6 * max(1.0, abs(lam[5]))


# ---------------------------------------------------------------- Algorithm 2

def _offdiag_worst(F, blocks, rng, k=6):
    from oracle.factor import offdiag_multiply, offdiag_multiply_transpose
    worst = 0.0
    for j, LO in blocks:
        G = rng.standard_normal((LO.shape[1], k))
        H = rng.standard_normal((LO.shape[0], k))
        a, b = offdiag_multiply(F, j, G), LO @ G
        at, bt = offdiag_multiply_transpose(F, j, H), LO.T @ H
        worst = max(worst, np.abs(a - b).max() / np.abs(b).max(), np.abs(at - bt).max() / np.abs(bt).max())
    return worst


def test_offdiag_multiply_is_the_explicit_block_product():
    # Algorithm 2 and its transpose against L^O_j = U^O_j (L^D_j)^{-T} formed by the
    # triangular solve of Algorithm 1 (the exact factor): the same block applied two
    # ways, equal to rounding for every supernode with off-diagonal rows.
    p = grid_problem((14, 13, 12), sigma=1.0, seed=3)
    sym = symbolic(p.n, p.rowptr, p.colind, 32)
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0, Options(leaf_max=32))
    blocks = [(j, F.LO[j]) for j in range(sym.M) if sym.r(j)]
    assert _offdiag_worst(F, blocks, np.random.default_rng(0)) <= 1e-12


def test_offdiag_multiply_with_compressed_descendants_matches_dense_block():
    # With compressed descendants (eq. lowRankMult, U_prod = U_k^T U_k): Algorithm 2's
    # product equals the dense L^O_j that the explicit path forms from the same
    # low-rank updates, for every compressed supernode that has compressed descendants.
    p = grid_problem((16, 15, 14), sigma=1.0, seed=4)
    sym = symbolic(p.n, p.rowptr, p.colind, 32)
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-2, Options(leaf_max=32, tau_O=16, keep_lo=True))
    comp = {j for j in range(sym.M) if F.V[j] is not None}
    blocks = [(j, F.LO_dense[j]) for j in sorted(comp) if any(k in comp for (k, _, _) in sym.pairs[j])]
    assert len(blocks) >= 3
    assert _offdiag_worst(F, blocks, np.random.default_rng(1)) <= 1e-12


@pytest.mark.parametrize("power_iters", [0, 1])
def test_implicit_compression_reproduces_explicit_factor(power_iters):
    # Algorithm 3 through Algorithm 2 (L^O_j of compressed supernodes never formed)
    # against Algorithm 3 on the explicit block, same samples: identical ranks, V_j U_j^T
    # and preconditioner to rounding.
    p = grid_problem((16, 15, 14), sigma=1.0, seed=5)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    opts = dict(seed=7, power_iters=power_iters)
    Fe = factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-2, Options(**opts))
    Fi = factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-2, Options(implicit=True, **opts))
    assert Fe.ell == Fi.ell and Fe.q == Fi.q and sum(Fe.q) > 0
    for j in range(sym.M):
        if Fe.V[j] is not None:
            a, b = Fe.V[j] @ Fe.U[j].T, Fi.V[j] @ Fi.U[j].T
            assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
            assert Fi.LO[j] is None
    r = np.random.default_rng(2).standard_normal(p.n)
    ze, zi = apply_preconditioner(Fe, r), apply_preconditioner(Fi, r)
    assert np.linalg.norm(ze - zi) <= 1e-12 * np.linalg.norm(ze)
