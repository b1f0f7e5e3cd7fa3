"""GPU parity of the interior blocks (§5.1) through the C ABI: the factor keeps only the
rows of each interior supernode's L^O_j inside its block, and the preconditioner reaches
the rest through A's entries and solves with the block's own factor -- the same
preconditioner as with every block stored, against the oracle's closed form."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.factor import Options, factor as o_factor
from oracle.ordering import symbolic
from oracle.solve import apply_preconditioner as o_apply, interior_blocks
from workloads import grid_problem

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _sol(p, **kw):
    from paper_1507_05593_amd import RSCSolver
    return RSCSolver(p.n, p.rowptr, p.colind, **kw)


@pytest.mark.parametrize("dims,precision", [((64, 64), "fp64"), ((16, 15, 14), "fp64"), ((24, 24, 24), "fp64"),
                                            ((24, 24, 24), "bf16"), ((20, 19, 18), "fp32")])
def test_interior_apply_equals_stored_apply(dims, precision):
    print("case", dims, precision, flush=True)
    p = grid_problem(dims, sigma=1.0, seed=9)
    vals = torch.tensor(p.values, device=DEV)
    b = torch.tensor(p.b, device=DEV)
    r = torch.tensor(np.random.default_rng(4).standard_normal(p.n), device=DEV)
    out = {}
    for inter in (False, True):
        sol = _sol(p, interior=inter, precision=precision)
        sol.factor(vals, 1e-2)
        z = sol.apply(r).cpu().numpy()
        x, info = sol.pcg(b, rtol=1e-8)
        out[inter] = (z, info, sol.stats(), sol)
    z0, i0, st0, _ = out[False]
    z1, i1, st1, sol1 = out[True]
    # mixed forms: the sweeps read the factor rounded to FP32; the stored-block apply rounds
    # L(R^B, C^B) itself, the closed form applies FP32 solves with L^B to A's exact entries
    # (two symmetric positive definite operators ~1e-5 apart), so PCG must agree instead
    tol = 1e-11 if precision == "fp64" else 1e-4
    assert np.abs(z1 - z0).max() <= tol * np.abs(z0).max()
    assert i1["converged"] and i1["iters"] == i0["iters"] and i1["true_residual"] < 1e-7
    assert st1["interior_blocks"] > 0 and st1["interior_dropped"] > 0
    assert st1["factor_entries"] == st0["factor_entries"] - st1["interior_dropped"]
    # against the oracle: blocks, dropped entries, and the apply through the closed form
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-2, Options())
    blocks = interior_blocks(F)
    assert st1["interior_blocks"] == sum(1 for s0, s1 in blocks if sym.rows[s1].size)
    dropped = 0
    for s0, s1 in blocks:
        end = int(sym.first[s1 + 1])
        for k in range(s0, s1 + 1):
            dropped += sym.c(k) * int(np.count_nonzero(sym.rows[k] >= end))
    assert st1["interior_dropped"] == dropped
    # an interior supernode's block: its rows inside the block, zero beyond
    j = next(k for s0, s1 in blocks for k in range(s0, s1 + 1) if sym.rows[k].size and
             np.count_nonzero(sym.rows[k] < int(sym.first[s1 + 1])) and
             np.count_nonzero(sym.rows[k] >= int(sym.first[s1 + 1])))
    s1 = next(b1 for b0, b1 in blocks if b0 <= j <= b1)
    inside = sym.rows[j] < int(sym.first[s1 + 1])
    LO1 = sol1.block(j)["LO"]
    LO0 = out[False][3].block(j)["LO"]
    assert np.array_equal(LO1[inside], LO0[inside]) and not LO1[~inside].any()


def test_interior_exact_matches_oracle_closed_form():
    """tol 1e-12 with full-rank sampling: ranks are unambiguous, so the interior apply
    matches the oracle's closed-form apply to rounding."""
    dims = (14, 13, 12)
    print("case", dims, flush=True)
    p = grid_problem(dims, sigma=1.0, seed=10)
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    F = o_factor(sym, p.n, p.rowptr, p.colind, p.values, 1e-12, Options(alpha_O=1e6))
    sol = _sol(p, interior=True, alpha_O=1e6)
    sol.factor(torch.tensor(p.values, device=DEV), 1e-12)
    r = np.random.default_rng(5).standard_normal(p.n)
    z = sol.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    zo = o_apply(F, r, interior=True)
    assert np.abs(z - zo).max() <= 1e-9 * np.abs(zo).max()
