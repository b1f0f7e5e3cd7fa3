"""GPU parity of the diagonal block trees (§4.1-4.2, Algorithms 4-6, §5.3) against the
FP64 oracle, through the C ABI: the written-out L^D_j of every tree supernode, the
preconditioner, full-rank sampling against the exact factor, and PCG."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.factor import Options, factor as o_factor
from oracle.ordering import symbolic
from oracle.solve import apply_preconditioner as o_apply, solve as o_solve
from workloads import grid_coordinates, grid_problem

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _sol(p, xyz, **kw):
    from paper_1507_05593_amd import RSCSolver
    return RSCSolver(p.n, p.rowptr, p.colind, coords=xyz, **kw)


def _vals(p):
    return torch.tensor(p.values, dtype=torch.float64, device=DEV)


# (dims, tau_D, oversample): sizes where some blocks are sampled below full rank
CASES = [((48, 48), 8, 2), ((14, 14, 14), 32, 10), ((18, 17, 16), 24, 4)]


@pytest.mark.parametrize("dims,tau,over", CASES)
def test_tree_blocks_and_preconditioner_match_oracle(dims, tau, over):
    """Off-diagonal blocks sampled at full rank (tol 1e-10), so that the trees are the
    only approximation: every tree's written-out L^D_j and the preconditioner agree with
    the oracle's Algorithms 4-6 on the same samples."""
    print("case", dims, tau, over, flush=True)
    p = grid_problem(dims, sigma=1.0, seed=5)
    xyz = grid_coordinates(dims)
    tol = 1e-10
    o = Options(tau_D=tau, oversample=over, alpha_O=1e6)
    sym = symbolic(p.n, p.rowptr, p.colind, 64, tau, xyz)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, tol, o)
    trees = [j for j in range(sym.M) if sym.depth[j] > 0]
    assert trees
    assert any(H.ell[s] < min(H.rows(s)[1] - H.rows(s)[0], H.cols(s)[1] - H.cols(s)[0])
               for H in (F.LD[j] for j in trees) for s in H.ell)
    sol = _sol(p, xyz, tau_D=tau, oversample=over, alpha_O=1e6)
    assert np.array_equal(sol.perm, sym.perm)
    sol.factor(_vals(p), tol)
    torch.cuda.synchronize()
    st = sol.stats()
    assert st["tree_supernodes"] == len(trees) and st["diag_restarts"] == 0 and st["alpha_D_used"] == 0.5
    want_blocks = sum(F.LD[j].nblocks // 2 for j in trees)
    assert st["tree_blocks"] == want_blocks
    assert st["tree_rank_sum"] == sum(sum(F.LD[j].ell.values()) for j in trees)
    worst = 0.0
    for j in trees:
        Ld = F.LD[j].dense()
        got = np.tril(sol.block(j)["LD"])
        worst = max(worst, np.abs(got - Ld).max() / np.abs(Ld).max())
    assert worst <= 1e-8, worst
    r = np.random.default_rng(3).standard_normal(p.n)
    z = sol.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    zo = o_apply(F, r)
    assert np.abs(z - zo).max() <= 1e-8 * np.abs(zo).max()


def test_full_rank_trees_give_the_exact_factor():
    dims, tau = (16, 15, 14), 24
    print("case", dims, tau, flush=True)
    p = grid_problem(dims, sigma=1.5, seed=6)
    xyz = grid_coordinates(dims)
    sym = symbolic(p.n, p.rowptr, p.colind, 64, tau, xyz)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 0.0, Options())
    sol = _sol(p, xyz, tau_D=tau, alpha_D=1e5, alpha_O=1e6)
    sol.factor(_vals(p), 1e-14)
    torch.cuda.synchronize()
    assert sol.stats()["tree_supernodes"] > 0
    worst, scale = 0.0, max(np.abs(F.LD[j]).max() for j in range(sym.M))
    for j in range(sym.M):
        if sym.depth[j]:
            worst = max(worst, np.abs(np.tril(sol.block(j)["LD"]) - F.LD[j]).max())
    assert worst <= 1e-10 * scale, worst / scale


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_tree_pcg_iterations_match_oracle(precision):
    """Default rank constants (alpha_O 1, alpha_D 0.5), tol 1e-2: PCG to 1e-8 within
    10 % (+1) of the oracle's iteration count with the same trees."""
    dims, tau = (24, 24, 24), 48
    print("case", dims, tau, precision, flush=True)
    p = grid_problem(dims, sigma=1.0, seed=7)
    xyz = grid_coordinates(dims)
    sym = symbolic(p.n, p.rowptr, p.colind, 64, tau, xyz)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-2, Options(tau_D=tau))
    ro = o_solve(F, p.matrix(), p.b, rtol=1e-8)
    sol = _sol(p, xyz, tau_D=tau, precision=precision)
    sol.factor(_vals(p), 1e-2)
    x, res = sol.pcg(torch.tensor(p.b, device=DEV), 1e-8)
    assert res["converged"] and res["true_residual"] < 1e-7
    assert abs(res["iters"] - ro.iters) <= max(1, int(0.1 * ro.iters) + 1), (res["iters"], ro.iters)
    assert sol.stats()["tree_supernodes"] == sum(1 for j in range(sym.M) if sym.depth[j])


def test_tree_without_positions_and_spectral_positions():
    """Block trees in the dissection's own order (no positions) and with positions from
    the device's spectral coordinates (§4.3): both factor and converge."""
    dims, tau = (20, 20, 20), 40
    print("case", dims, tau, flush=True)
    p = grid_problem(dims, sigma=1.0, seed=8)
    it = []
    for coords in (None, "spectral"):
        sol = _sol(p, coords, tau_D=tau)
        sol.factor(_vals(p), 1e-2)
        x, res = sol.pcg(torch.tensor(p.b, device=DEV), 1e-8)
        assert res["converged"] and res["true_residual"] < 1e-7
        assert sol.stats()["tree_supernodes"] > 0
        it.append(res["iters"])
    assert max(it) <= 30, it


def test_restart_matches_oracle():
    """The alpha_D restart (§5.3) on a separator whose rank-one blocks make a leaf
    indefinite: the device restarts as often as the oracle, ends at the same alpha_D,
    and its block tree and preconditioner then agree with the oracle's."""
    from paper_1507_05593_amd import RSCSolver
    from workloads import clique_separator
    print("case clique separator", flush=True)
    n, rp, ci, v = clique_separator(8, 8, 32, 1e-3, 0)
    sym = symbolic(n, rp, ci, 8, 4)
    o = Options(tau_D=4, alpha_D=0.05, oversample=0, leaf_max=8)
    F = o_factor(sym, n, rp, ci, v, 1e-2, o)
    assert F.restarts > 0
    sol = RSCSolver(n, rp, ci, leaf_max=8, tau_D=4, alpha_D=0.05, oversample=0)
    sol.factor(torch.tensor(v, device=DEV), 1e-2)
    st = sol.stats()
    assert st["diag_restarts"] == F.restarts and st["alpha_D_used"] == pytest.approx(F.alpha_D)
    j = sym.M - 1
    Ld = F.LD[j].dense()
    assert np.abs(np.tril(sol.block(j)["LD"]) - Ld).max() <= 1e-8 * np.abs(Ld).max()
    r = np.random.default_rng(1).standard_normal(n)
    z = sol.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    zo = o_apply(F, r)
    assert np.abs(z - zo).max() <= 1e-6 * np.abs(zo).max()
