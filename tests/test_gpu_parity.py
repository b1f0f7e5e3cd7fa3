"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from oracle.adjoint import dense_adjoint, grad_faces as o_grad_faces, grad_values as o_grad_values
from oracle.factor import NotSPDError, Options, compress as o_compress, factor as o_factor
from oracle.philox import gaussian_sample
from oracle.ordering import symbolic
from oracle.solve import apply_preconditioner as o_apply, solve as o_solve
from workloads import grid_problem
from workloads.grids import batched_problems

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _sol(p, **kw):
    from paper_1507_05593_amd import RSCSolver
    return RSCSolver(p.n, p.rowptr, p.colind, **kw)


def _vals(p):
    return torch.tensor(p.values, dtype=torch.float64, device=DEV)


def _vec(v):
    return torch.tensor(np.asarray(v), dtype=torch.float64, device=DEV)


def _check_blocks(sol, F, rel=1e-12):
    sym = F.sym
    scale = max(np.abs(F.LD[j]).max() for j in range(sym.M))
    worst = 0.0
    for j in range(sym.M):
        blk = sol.block(j)
        worst = max(worst, np.abs(blk["LD"] - F.LD[j]).max())
        if sym.r(j) and F.LO[j] is not None:
            worst = max(worst, np.abs(blk["LO"] - F.LO[j]).max())
    assert worst <= rel * scale, worst / scale


@pytest.mark.parametrize("dims,sigma,leaf", [((16, 16), 0.0, 64), ((8, 8, 8), 1.0, 8), ((12, 11, 10), 1.5, 64),
                                             ((20, 20, 20), 1.0, 64), ((64, 64), 0.0, 64)])
def test_exact_factor_blocks_match_oracle(dims, sigma, leaf):
    print("case", dims, sigma, leaf, flush=True)
    p = grid_problem(dims, sigma=sigma, seed=1, unit=(sigma == 0))
    sym = symbolic(p.n, p.rowptr, p.colind, leaf)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0, Options(leaf_max=leaf))
    sol = _sol(p, leaf_max=leaf)
    sol.factor(_vals(p), 0.0)
    torch.cuda.synchronize()
    _check_blocks(sol, F, 1e-12)


@pytest.mark.parametrize("tile", [64, 128])
def test_fixed_tile_sizes_match_oracle(tile):
    # every product launch cut to one tile edge: exact blocks to 1e-12 and the
    # compressed factor's PCG against the oracle's
    print("case tile", tile, flush=True)
    p = grid_problem((22, 20, 18), sigma=1.0, seed=6)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0, Options())
    sol = _sol(p, gemm_tile=tile)
    sol.factor(_vals(p), 0.0)
    torch.cuda.synchronize()
    _check_blocks(sol, F, 1e-12)
    Fc = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-2, Options(seed=3))
    sc = _sol(p, gemm_tile=tile, seed=3)
    sc.factor(_vals(p), 1e-2)
    x, info = sc.pcg(_vec(p.b), rtol=1e-8)
    res = o_solve(Fc, p.matrix(), p.b, rtol=1e-8)
    assert info["converged"] and abs(info["iters"] - res.iters) <= max(1, 0.1 * res.iters)


def test_exact_factor_residual_and_pcg():
    p = grid_problem((14, 13, 12), sigma=1.0, seed=3)
    sol = _sol(p)
    sol.factor(_vals(p), 0.0)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    L = np.zeros((p.n, p.n))
    for j in range(sym.M):
        blk = sol.block(j)
        lo, hi = sym.first[j], sym.first[j + 1]
        L[lo:hi, lo:hi] = blk["LD"]
        if sym.r(j):
            L[np.ix_(sym.rows[j], np.arange(lo, hi))] = blk["LO"]
    Ap = p.matrix()[sym.perm][:, sym.perm].toarray()
    assert np.linalg.norm(Ap - L @ L.T) / np.linalg.norm(Ap) <= 1e-11
    x, info = sol.pcg(_vec(p.b), rtol=1e-12)
    xs = np.linalg.solve(p.matrix().toarray(), p.b)
    assert info["iters"] <= 2 and info["true_residual"] <= 1e-12
    assert np.abs(x.cpu().numpy() - xs).max() <= 1e-10 * np.abs(xs).max()


def test_preconditioner_apply_matches_oracle_exact_and_compressed():
    p = grid_problem((16, 15, 14), sigma=1.0, seed=5)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    rng = np.random.default_rng(0)
    r = rng.standard_normal(p.n)
    for tol in (0.0, 1e-2):
        sol = _sol(p, seed=7)
        sol.factor(_vals(p), tol)
        z = sol.apply(_vec(r)).cpu().numpy()
        # compressed: the oracle also through Algorithm 2 (L^O_j of compressed supernodes
        # never formed on either side)
        F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, tol, Options(seed=7, implicit=tol > 0))
        zo = o_apply(F, r)
        # the compressed factors agree to the conditioning of the truncation only
        bound = 1e-11 if tol == 0 else 1e-6
        assert np.linalg.norm(z - zo) <= bound * np.linalg.norm(zo), (tol, np.linalg.norm(z - zo) / np.linalg.norm(zo))


@pytest.mark.parametrize("dims,sigma,tol", [((16, 16, 16), 1.0, 1e-2), ((24, 22, 20), 1.5, 1e-2),
                                            ((96, 96), 1.0, 1e-2), ((20, 20, 20), 1.0, 1e-1)])
def test_compressed_ranks_and_pcg_match_oracle(dims, sigma, tol):
    print("case", dims, sigma, tol, flush=True)
    p = grid_problem(dims, sigma=sigma, seed=2)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, tol, Options(seed=11))
    sol = _sol(p, seed=11, keep_lo=True)   # the dense L^O_j kept for the block comparison
    sol.factor(_vals(p), tol)
    ell, q = sol.ranks()
    assert np.array_equal(ell, np.array(F.ell))
    qo = np.array(F.q)
    assert np.abs(q - qo).max() <= 2 and np.mean(q != qo) <= 0.05, (q, qo)
    # Compression step on identical input: the dense L^O_j the device formed before
    # compressing is handed to the oracle's range finder (same seed, same sample).
    # Upstream drift (a descendant that kept one more near-threshold direction) is
    # thereby excluded; what remains is the device's orthonormalisation and
    # truncation against Householder QR + eigendecomposition.
    opts = Options(seed=11)
    for j in range(sym.M):
        if not ell[j]:
            continue
        blk = sol.block(j)
        U, V, LO = blk["U"], blk["V"], blk["LO"]
        assert np.abs(U.T @ U - np.eye(U.shape[1])).max() <= 1e-12
        assert np.linalg.norm(V - LO @ U) <= 1e-12 * max(np.linalg.norm(LO), 1e-300)
        Vo, Uo, ello, qj = o_compress(LO, j, opts, tol)
        assert ello == ell[j]
        # the device keeps a direction whose eigenvalue sits on the cut-off whole or
        # not at all, so its rank may differ by one there
        assert abs(q[j] - qj) <= 1, (j, q[j], qj)
        s1 = np.linalg.norm(LO, 2)
        e_dev = np.linalg.norm(LO - V @ U.T, 2)
        e_orc = np.linalg.norm(LO - Vo @ Uo.T, 2)
        # same sample span: the device error exceeds the oracle's by at most the one
        # near-threshold direction (sigma ~ tol sigma_1(V) <= tol ||L^O||)
        assert e_dev <= e_orc + 1.01 * tol * s1 + 1e-12 * s1, (j, e_dev / s1, e_orc / s1)
        if q[j] == qj and qj > 0:
            # Away from the cut-off the kept subspace is unique; the two sides' Gram
            # matrices differ by the rounding of the sample's orthonormalisation,
            # eps times the condition of Y (up to ~1e4-1e6 here), and that moves the
            # subspace by at most that over the eigenvalue gap.  A low-precision slip
            # (1e-3 and up) or a wrong direction fails this by orders of magnitude.
            Ys = np.linalg.qr(LO.T @ gaussian_sample(11, j, LO.shape[0], ello))[0]
            lam = np.linalg.svd(LO @ Ys, compute_uv=False) ** 2
            lam = lam / lam[0]
            near = [abs(lam[i] - tol ** 2) <= 1e-3 * tol ** 2 for i in (qj - 1, qj) if i < len(lam)]
            if not any(near):
                gap = lam[qj - 1] - (lam[qj] if qj < len(lam) else 0.0)
                bound = 1e-7 + 1e-10 / gap
                assert np.linalg.norm(V @ U.T - Vo @ Uo.T) <= bound * np.linalg.norm(Vo @ Uo.T), (j, gap)
    A = p.matrix()
    res = o_solve(F, A, p.b, rtol=1e-8)
    x, info = sol.pcg(_vec(p.b), rtol=1e-8)
    assert info["converged"] and info["true_residual"] <= 1e-8 * 1.5
    assert abs(info["iters"] - res.iters) <= max(1, 0.1 * res.iters), (info["iters"], res.iters)
    xs = res.x
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-6 * np.linalg.norm(xs)


@pytest.mark.parametrize("power_iters,tol", [(1, 1e-2), (2, 1e-1), (2, 1e-2)])
def test_power_iterations_ranks_compression_and_pcg(power_iters, tol):
    # Algorithm 3 with power iterations Y = (L^O)^T (L^O Y) on the device (FP64 form):
    # same sample counts as the oracle, ranks within the cut-off slack, each block's
    # compression of the device's own L^O_j within the oracle's error plus one
    # near-threshold direction, and PCG to the same iteration count.
    print("case power_iters", power_iters, "tol", tol, flush=True)
    dims, sigma = (16, 16, 16), 1.0
    p = grid_problem(dims, sigma=sigma, seed=2)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    opts = Options(seed=11, power_iters=power_iters)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, tol, opts)
    sol = _sol(p, seed=11, power_iters=power_iters, keep_lo=True)
    sol.factor(_vals(p), tol)
    ell, q = sol.ranks()
    assert np.array_equal(ell, np.array(F.ell))
    qo = np.array(F.q)
    assert np.abs(q - qo).max() <= 2 and np.mean(q != qo) <= 0.05, (q, qo)
    for j in range(sym.M):
        if not ell[j]:
            continue
        blk = sol.block(j)
        U, V, LO = blk["U"], blk["V"], blk["LO"]
        assert np.abs(U.T @ U - np.eye(U.shape[1])).max() <= 1e-10
        assert np.linalg.norm(V - LO @ U) <= 1e-10 * max(np.linalg.norm(LO), 1e-300)
        Vo, Uo, ello, qj = o_compress(LO, j, opts, tol)
        assert ello == ell[j] and abs(q[j] - qj) <= 1, (j, q[j], qj)
        s1 = np.linalg.norm(LO, 2)
        e_dev = np.linalg.norm(LO - V @ U.T, 2)
        e_orc = np.linalg.norm(LO - Vo @ Uo.T, 2)
        assert e_dev <= e_orc + 1.01 * tol * s1 + 1e-10 * s1, (j, e_dev / s1, e_orc / s1)
    res = o_solve(F, p.matrix(), p.b, rtol=1e-8)
    x, info = sol.pcg(_vec(p.b), rtol=1e-8)
    assert info["converged"] and info["true_residual"] <= 1e-8 * 1.5
    assert abs(info["iters"] - res.iters) <= max(1, 0.1 * res.iters), (info["iters"], res.iters)
    assert np.linalg.norm(x.cpu().numpy() - res.x) <= 1e-6 * np.linalg.norm(res.x)


def test_full_sampling_reproduces_exact_factor():
    # Full sampling (l_j = min(r_j, c_j)) with a cut-off below rounding keeps every
    # direction of L^O_j, so V_j U_j^T is the exact off-diagonal block: every block of
    # the device's compressed factor against the oracle's exact factor (the unique
    # Cholesky factor of the permuted matrix) to 1e-12, and the preconditioner against
    # the oracle's exact one.
    print("case full sampling (12, 12, 12)", flush=True)
    p = grid_problem((12, 12, 12), sigma=1.0, seed=4)
    sym = symbolic(p.n, p.rowptr, p.colind, 32)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0, Options(leaf_max=32, tau_O=8))
    fc = _sol(p, tau_O=8, leaf_max=32, alpha_O=1e9)
    fc.factor(_vals(p), 1e-13)
    ell, q = fc.ranks()
    comp = np.nonzero(ell)[0]
    assert comp.size > 0
    scale = max(np.abs(F.LD[j]).max() for j in range(sym.M))
    worst = 0.0
    for j in range(sym.M):
        blk = fc.block(j)
        worst = max(worst, np.abs(blk["LD"] - F.LD[j]).max())
        if not sym.r(j):
            continue
        if ell[j]:
            assert ell[j] == min(sym.r(j), sym.c(j)) and q[j] == ell[j], (j, ell[j], q[j])
            LO = blk["V"] @ blk["U"].T
        else:
            LO = blk["LO"]
        worst = max(worst, np.abs(LO - F.LO[j]).max())
    print("full sampling: largest block difference / scale", worst / scale, flush=True)
    assert worst <= 1e-12 * scale, worst / scale
    r = np.random.default_rng(1).standard_normal(p.n)
    z = fc.apply(_vec(r)).cpu().numpy()
    zo = o_apply(F, r)
    assert np.linalg.norm(z - zo) <= 1e-11 * np.linalg.norm(zo)


def test_not_spd_reports_supernode():
    p = grid_problem((8, 8, 8), sigma=1.0, seed=6)
    vals = p.values.copy()
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    d = np.nonzero(rows == p.colind)[0]
    vals[d[200]] = -vals[d[200]]
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    with pytest.raises(NotSPDError) as eo:
        o_factor(sym, p.n, p.rowptr, p.colind, vals, 0.0)
    from paper_1507_05593_amd import RSCError
    sol = _sol(p)
    with pytest.raises(RSCError) as eg:
        sol.factor(_vec(vals), 0.0)
    assert eg.value.code == 3
    assert sol.stats()["failed_supernode"] == eo.value.supernode
    # the handle recovers with valid values
    sol.factor(_vals(p), 0.0)
    x, info = sol.pcg(_vec(p.b), rtol=1e-10)
    assert info["converged"]


def test_mixed_retry_policy_and_recovery():
    # The restart policy: a mixed BF16 factorization that meets a non-positive pivot is
    # redone with FP32 products, then in FP64; an indefinite matrix fails all three and
    # reports the supernode.  The handle then factors valid values in BF16 again, twice
    # (FP32 sweep copy, solve graphs recaptured for the new plan), PCG converges each time,
    # and the solution agrees with an FP64 handle's.
    print("case retry policy", flush=True)
    p = grid_problem((10, 9, 8), sigma=1.0, seed=6)
    vals = p.values.copy()
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    d = np.nonzero(rows == p.colind)[0]
    vals[d[150]] = -vals[d[150]]
    from paper_1507_05593_amd import RSCError
    sol = _sol(p, precision="bf16", seed=1)
    with pytest.raises(RSCError) as eg:
        sol.factor(_vec(vals), 1e-2)
    assert eg.value.code == 3
    st = sol.stats()
    assert st["retries"] == 2 and st["failed_supernode"] >= 0
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-2, Options(seed=1))
    ref = o_solve(F, p.matrix(), p.b, rtol=1e-8)
    for _ in range(2):
        sol.factor(_vals(p), 1e-2)
        assert sol.stats()["precision_used"] == 1
        x, info = sol.pcg(_vec(p.b), rtol=1e-8)
        assert info["converged"] and info["true_residual"] <= 1.5e-8
        assert abs(info["iters"] - ref.iters) <= max(1, 0.1 * ref.iters), (info["iters"], ref.iters)
    s64 = _sol(p, seed=1)
    s64.factor(_vals(p), 1e-2)
    x64, i64 = s64.pcg(_vec(p.b), rtol=1e-8)
    assert np.linalg.norm(x.cpu().numpy() - x64.cpu().numpy()) <= 1e-6 * np.linalg.norm(x64.cpu().numpy())


def test_determinism_and_graph_replay():
    p = grid_problem((18, 17, 16), sigma=1.0, seed=8)
    b = _vec(p.b)
    runs = []
    for use_graph in (True, True, False):
        sol = _sol(p, use_graph=use_graph, seed=3)
        for _ in range(2):
            sol.factor(_vals(p), 1e-2)
            x, info = sol.pcg(b, rtol=1e-9)
            runs.append((x.cpu().numpy().copy(), info["iters"]))
    for x, it in runs[1:]:
        assert it == runs[0][1]
        assert np.array_equal(x, runs[0][0])


@pytest.mark.parametrize("precision,tol", [("fp64", 0.0), ("bf16", 1e-2)])
def test_wide_separator_graph_equals_eager_launch_order(precision, tol):
    # top separator of 867 columns, so its panel steps span several 256-column outer
    # blocks with end-of-block trailing products; the captured graph must give bit for
    # bit what the eager launches (one stream, list order) give
    print("case wide separator graph vs eager", precision, tol, flush=True)
    p = grid_problem((34, 34, 34), sigma=1.0, seed=5)
    b = _vec(p.b)
    out = []
    for use_graph in (True, False):
        sol = _sol(p, use_graph=use_graph, seed=3, precision=precision, gemm_tile=64)
        assert np.diff(sol.supernode_info()[0]).max() > 768
        sol.factor(_vals(p), tol)
        x, info = sol.pcg(b, rtol=1e-9)
        blocks = [sol.block(j)["LD"] for j in range(sol.supernodes)]
        out.append((x.cpu().numpy().copy(), info["iters"], blocks))
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])
    for u, v in zip(out[0][2], out[1][2]):
        assert np.array_equal(u, v)
    if tol == 0.0:
        sym = symbolic(p.n, p.rowptr, p.colind, 64)
        F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0, Options(leaf_max=64))
        _check_blocks(sol, F, 1e-12)


def test_adjoint_matches_dense_oracle_and_autograd():
    from paper_1507_05593_amd import grad_faces, solve
    p = grid_problem((5, 4, 3), sigma=1.0, seed=9)
    x_d, lam_d, _ = dense_adjoint(p.matrix().toarray(), p.b, p.x_target)
    sol = _sol(p)
    vals = _vals(p).requires_grad_(True)
    b = _vec(p.b).requires_grad_(True)
    x = solve(vals, b, sol, tol=0.0, rtol=1e-13)
    loss = 0.5 * ((x - _vec(p.x_target)) ** 2).sum()
    loss.backward()
    assert np.abs(x.detach().cpu().numpy() - x_d).max() <= 1e-11 * np.abs(x_d).max()
    assert np.abs(b.grad.cpu().numpy() - lam_d).max() <= 1e-10 * np.abs(lam_d).max()
    gv = o_grad_values(p.rowptr, p.colind, lam_d, x_d)
    assert np.abs(vals.grad.cpu().numpy() - gv).max() <= 1e-10 * np.abs(gv).max()
    gf = grad_faces(torch.tensor(p.face_i, device=DEV), torch.tensor(p.face_j, device=DEV),
                    b.grad, x.detach()).cpu().numpy()
    go = o_grad_faces(p.face_i, p.face_j, lam_d, x_d)
    assert np.abs(gf - go).max() <= 1e-10 * np.abs(go).max()


@pytest.mark.parametrize("lo,hi", [(12, 48), (60, 140)])
def test_batched_systems_equal_single_solves(lo, hi):
    # (60, 140): every system has compressed separators, so the per-system sample
    # keys are exercised too
    from paper_1507_05593_amd import RSCSolver
    probs = batched_problems(6, lo, hi, 1.0, seed=4)
    sol = RSCSolver.batch([q.n for q in probs], [q.rowptr for q in probs], [q.colind for q in probs])
    vals = torch.cat([_vals(q) for q in probs])
    b = torch.cat([_vec(q.b) for q in probs])
    sol.factor(vals, 1e-2)
    x, infos = sol.pcg(b, rtol=1e-10)
    off = 0
    for q, info in zip(probs, infos):
        s1 = _sol(q)
        s1.factor(_vals(q), 1e-2)
        x1, i1 = s1.pcg(_vec(q.b), rtol=1e-10)
        assert info["iters"] == i1["iters"]
        if hi > 100:
            assert s1.ranks()[1].sum() > 0
        assert np.abs(x[off:off + q.n].cpu().numpy() - x1.cpu().numpy()).max() <= 1e-12 * np.abs(x1.cpu().numpy()).max()
        off += q.n


def test_empty_rhs_and_tiny_system():
    p = grid_problem((3, 3), unit=True)
    sol = _sol(p)
    sol.factor(_vals(p), 0.0)
    x, info = sol.pcg(torch.zeros(p.n, dtype=torch.float64, device=DEV))
    assert info["iters"] == 0 and np.all(x.cpu().numpy() == 0)
    p1 = grid_problem((1, 1), unit=True)
    s1 = _sol(p1)
    s1.factor(_vals(p1), 0.0)
    x, info = s1.pcg(_vec(np.array([3.0])), rtol=1e-12)
    assert abs(x.item() - 3.0 / 4.0) < 1e-15


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("dims,sigma", [((20, 20, 20), 1.0), ((28, 26, 24), 1.5)])
def test_mixed_precision_forms_reach_rtol(precision, dims, sigma):
    # Mixed forms: parity with the FP64 oracle is unpinned bitwise; the stated bar is
    # convergence to rtol with a true residual <= 1e-8 and an iteration count within
    # 10 % of the FP64 oracle's (at least one; FP64 PCG recovers the accuracy).
    print("case", precision, dims, sigma, flush=True)
    p = grid_problem(dims, sigma=sigma, seed=12)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-2, Options(seed=0))
    ref = o_solve(F, p.matrix(), p.b, rtol=1e-8)
    sol = _sol(p, precision=precision, seed=0)
    sol.factor(_vals(p), 1e-2)
    st = sol.stats()
    x, info = sol.pcg(_vec(p.b), rtol=1e-8)
    assert info["converged"] and info["true_residual"] <= 1.5e-8
    print(precision, dims, "iters", info["iters"], "oracle", ref.iters, "precision used",
          st["precision_used"], flush=True)
    assert abs(info["iters"] - ref.iters) <= max(1, 0.1 * ref.iters), (info["iters"], ref.iters)
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_mixed_precision_exact_factor_error_is_small():
    # tol = 0 with low-precision Schur updates: the factor residual is at the level of
    # the operand rounding (FP32: ~1e-7, BF16 split: ~1e-5), not FP64's 1e-15.
    p = grid_problem((12, 12, 12), sigma=1.0, seed=3)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    Ap = p.matrix()[sym.perm][:, sym.perm].toarray()
    for precision, bound in (("fp32", 1e-5), ("bf16", 1e-3)):
        sol = _sol(p, precision=precision, retry=False)
        sol.factor(_vals(p), 0.0)
        L = np.zeros((p.n, p.n))
        for j in range(sym.M):
            blk = sol.block(j)
            lo, hi = sym.first[j], sym.first[j + 1]
            L[lo:hi, lo:hi] = blk["LD"]
            if sym.r(j):
                L[np.ix_(sym.rows[j], np.arange(lo, hi))] = blk["LO"]
        res = np.linalg.norm(Ap - L @ L.T) / np.linalg.norm(Ap)
        print(precision, "factor residual", res)
        assert res <= bound


def test_mixed_forms_sweeps_apply_the_fp32_rounded_factor():
    # After a mixed factorization the sweeps read an FP32 copy of the factor operands
    # with FP64 vectors and sums: the operator applied is F^T F for the rounded
    # sweep operators F, so it is symmetric to FP64 summation, and it stays within FP32
    # rounding (times the factor's conditioning) of the FP64 apply of the same factor.
    print("case fp32 sweeps (12, 11, 10)", flush=True)
    p = grid_problem((12, 11, 10), sigma=1.0, seed=4)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(p.n), rng.standard_normal(p.n)
    for precision in ("fp32", "bf16"):
        sol = _sol(p, precision=precision, retry=False)
        sol.factor(_vals(p), 0.0)
        L = np.zeros((p.n, p.n))
        for j in range(sym.M):
            blk = sol.block(j)
            lo, hi = sym.first[j], sym.first[j + 1]
            L[lo:hi, lo:hi] = blk["LD"]
            if sym.r(j):
                L[np.ix_(sym.rows[j], np.arange(lo, hi))] = blk["LO"]
        Mu = sol.apply(_vec(u)).cpu().numpy()
        Mv = sol.apply(_vec(v)).cpu().numpy()
        asym = abs(u @ Mv - v @ Mu) / (np.linalg.norm(u) * np.linalg.norm(Mv))
        zp = np.linalg.solve(L.T, np.linalg.solve(L, u[sym.perm]))
        z64 = np.empty(p.n)
        z64[sym.perm] = zp
        rel = np.linalg.norm(Mu - z64) / np.linalg.norm(z64)
        print(precision, "asymmetry", asym, "vs FP64 apply", rel, flush=True)
        assert asym <= 1e-12
        assert rel <= 1e-6


@pytest.mark.parametrize("precision,tol", [("fp64", 0.0), ("fp64", 1e-2), ("bf16", 1e-2)])
def test_small_level_sweeps_equal_per_operation_sweeps(precision, tol):
    # The lowest elimination-tree levels run each sweep step as one launch (one workgroup
    # per supernode, descendants' contributions pulled by the rows); the per-operation
    # launches compute the same products in another summation order.  Bounds on this grid
    # (level column maxima 63, 25, 40, 56, 96, 126, 216): none, four levels (64 threads per
    # supernode), five (the fifth with 256), and every level, the root's included.
    print("case small sweeps", precision, tol, flush=True)
    p = grid_problem((18, 17, 16), sigma=1.5, seed=8)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    rng = np.random.default_rng(4)
    r = _vec(rng.standard_normal(p.n))
    nlev = max(sym.level) + 1
    b = _vec(p.b)
    zs = {}
    for bound in (0, 64, 100, 1024):
        sol = _sol(p, seed=3, precision=precision, retry=False, sweep_small_c=bound)
        sol.factor(_vals(p), tol)
        zs[bound] = sol.apply(r).cpu().numpy()
        # launches per preconditioner apply, from a profiled PCG run
        sol.profile(True)
        _, res = sol.pcg(b, rtol=1e-6)
        prof = sol.kernel_profile()
        sol.profile(False)
        nfwd, nbwd = prof["sweep_fwd"]["launches"], prof["sweep_bwd"]["launches"]
        iters = res["iters"]
        small = 0
        while small < nlev and all(sym.c(j) <= bound and sym.r(j) <= 2048
                                   for j in range(sym.M) if sym.level[j] == small):
            small += 1
        assert small == {0: 0, 64: 4, 100: 5, 1024: nlev}[bound], (bound, small)
        print(bound, "small levels", small, "of", nlev, flush=True)
        # one apply before the loop and one per iteration that did not stop it
        assert nfwd == nbwd, (nfwd, nbwd)
        if small == 0:
            assert nfwd == 0
        else:
            assert nfwd % small == 0 and nfwd // small in (iters, iters + 1), (bound, nfwd, small, iters)
    ref = zs[0]
    for bound in (64, 100, 1024):
        rel = np.linalg.norm(zs[bound] - ref) / np.linalg.norm(ref)
        print(bound, "vs per-operation sweeps", rel, flush=True)
        assert rel <= 1e-13, (bound, rel)
    # and the default against the oracle
    if precision == "fp64":
        F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, tol, Options(seed=3, implicit=tol > 0))
        zo = o_apply(F, r.cpu().numpy())
        bound = 1e-11 if tol == 0 else 1e-6
        assert np.linalg.norm(zs[100] - zo) <= bound * np.linalg.norm(zo)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_projector_iteration_in_lds_ranks_and_pcg(precision):
    # Levels whose supernodes all have small sample counts run the projector iteration in
    # one workgroup per supernode (k_trunc_ns): check that it ran, that the ranks agree
    # with the FP64 oracle's to the bar of the product-launch path, and that PCG
    # converges within the stated iteration tolerance of the oracle's.
    print("case projector in LDS", precision, flush=True)
    p = grid_problem((18, 17, 16), sigma=1.0, seed=9)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-2, Options(seed=2))
    ref = o_solve(F, p.matrix(), p.b, rtol=1e-8)
    sol = _sol(p, precision=precision, seed=2, retry=False)
    sol.profile(True)
    sol.factor(_vals(p), 1e-2)
    kp = sol.kernel_profile()
    sol.profile(False)
    assert kp["trunc_ns"]["launches"] > 0, kp.get("trunc_ns")
    ell, q = sol.ranks()
    assert np.array_equal(ell, np.array(F.ell))
    qo = np.array(F.q)
    # the same bar as the product-launch path (upstream drift of near-threshold ranks)
    assert np.abs(q - qo).max() <= 2 and np.mean(q != qo) <= 0.05, (q, qo)
    x, info = sol.pcg(_vec(p.b), rtol=1e-8)
    assert info["converged"] and info["true_residual"] <= 1.5e-8
    assert abs(info["iters"] - ref.iters) <= max(1, 0.1 * ref.iters), (info["iters"], ref.iters)


def test_poisson2d_64_exact_then_compressed_pcg():
    # The 2D unit-coefficient 64 x 64 workload (4096 unknowns): the exact factor's
    # blocks against the oracle's, then the rank-structured factor at tol 1e-2 with
    # PCG to 1e-8 -- sample counts equal, kept ranks within one, iterations within
    # 10 % of the oracle's (at least one), and the solution element by element.
    from workloads import workload_config
    print("case poisson2d_64", flush=True)
    cfg = workload_config("poisson2d_64")
    p = grid_problem(cfg["dims"], sigma=cfg["sigma"], seed=cfg["seed"], unit=cfg["unit"])
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F0 = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0, Options())
    sol = _sol(p, seed=0)
    sol.factor(_vals(p), 0.0)
    _check_blocks(sol, F0, 1e-12)
    x0, i0 = sol.pcg(_vec(p.b), rtol=1e-12)
    assert i0["iters"] <= 2 and i0["true_residual"] <= 1e-12
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, cfg["tol"], Options(seed=0))
    ref = o_solve(F, p.matrix(), p.b, rtol=cfg["rtol"])
    sol.factor(_vals(p), cfg["tol"])
    ell, q = sol.ranks()
    assert np.array_equal(ell, np.array(F.ell)) and ell.sum() > 0
    assert np.abs(q - np.array(F.q)).max() <= 1, (q, F.q)
    x, info = sol.pcg(_vec(p.b), rtol=cfg["rtol"])
    print("poisson2d_64 iters", info["iters"], "oracle", ref.iters, flush=True)
    assert info["converged"] and info["true_residual"] <= cfg["rtol"]
    assert abs(info["iters"] - ref.iters) <= max(1, 0.1 * ref.iters), (info["iters"], ref.iters)
    err = np.abs(x.cpu().numpy() - ref.x).max() / np.abs(ref.x).max()
    print("poisson2d_64 max |x - x_oracle| / max |x_oracle|", err, flush=True)
    assert err <= 1e-6


def test_pcg_not_converged_reports_status_and_first_iterate():
    # max_iter = 1 with rtol out of reach: RSC_ERR_NOT_CONVERGED, and the iterate left
    # in x is the oracle's first CG iterate (x1 = alpha_0 z_0) for the exact factor.
    from paper_1507_05593_amd import RSCError
    print("case not converged", flush=True)
    p = grid_problem((12, 11, 10), sigma=1.0, seed=2)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-1, Options(seed=4))
    ref = o_solve(F, p.matrix(), p.b, rtol=1e-14, max_iter=1)
    sol = _sol(p, seed=4)
    sol.factor(_vals(p), 1e-1)
    with pytest.raises(RSCError) as e:
        sol.pcg(_vec(p.b), rtol=1e-14, max_iter=1)
    assert e.value.code == 4
    x, info = sol.pcg(_vec(p.b), rtol=1e-14, max_iter=1, raise_on_failure=False)
    assert not info["converged"] and info["iters"] == 1 and not ref.converged
    assert abs(info["rel_residual"] - ref.rel_residual) <= 1e-6 * ref.rel_residual
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_adjoint_after_the_solver_factored_other_values():
    # Backward through a solve after the same solver factored another matrix (a second
    # solve under no_grad): the adjoint must still be the first matrix's.
    from paper_1507_05593_amd import solve
    print("case stale factor adjoint", flush=True)
    p = grid_problem((5, 4, 3), sigma=1.0, seed=9)
    q = grid_problem((5, 4, 3), sigma=1.0, seed=10)
    assert np.array_equal(p.colind, q.colind) and not np.allclose(p.values, q.values)
    x_d, lam_d, _ = dense_adjoint(p.matrix().toarray(), p.b, p.x_target)
    sol = _sol(p)
    vals = _vals(p).requires_grad_(True)
    b = _vec(p.b).requires_grad_(True)
    x = solve(vals, b, sol, tol=0.0, rtol=1e-13)
    with torch.no_grad():
        solve(_vals(q), _vec(q.b), sol, tol=0.0, rtol=1e-13)
    loss = 0.5 * ((x - _vec(p.x_target)) ** 2).sum()
    loss.backward()
    assert np.abs(b.grad.cpu().numpy() - lam_d).max() <= 1e-10 * np.abs(lam_d).max()
    gv = o_grad_values(p.rowptr, p.colind, lam_d, x_d)
    assert np.abs(vals.grad.cpu().numpy() - gv).max() <= 1e-10 * np.abs(gv).max()


def test_compressed_lo_not_kept_by_default_and_same_factor():
    # Without keep_lo the dense L^O_j of a compressed supernode lives in the level pool
    # only while its level is factored: rsc_get_block refuses it, and the rank-structured
    # factor (ranks, V_j, U_j, the preconditioner) is identical to the one kept with it.
    from paper_1507_05593_amd import RSCError
    print("case keep_lo", flush=True)
    p = grid_problem((16, 15, 14), sigma=1.0, seed=5)
    a = _sol(p, seed=2)
    b = _sol(p, seed=2, keep_lo=True)
    for s in (a, b):
        s.factor(_vals(p), 1e-2)
    ell, q = a.ranks()
    assert np.array_equal((ell, q), b.ranks())
    j = int(np.nonzero(ell)[0][-1])
    from paper_1507_05593_amd import lib
    import ctypes as C
    lo = np.zeros(1 << 20)
    assert lib().rsc_get_block(a._h, j, None, lo.ctypes.data_as(C.c_void_p), None, None) == 8
    ba, bb = a.block(j), b.block(j)
    assert ba["LO"] is None and bb["LO"] is not None
    assert np.array_equal(ba["V"], bb["V"]) and np.array_equal(ba["U"], bb["U"])
    r = _vec(np.random.default_rng(0).standard_normal(p.n))
    assert np.array_equal(a.apply(r).cpu().numpy(), b.apply(r).cpu().numpy())
