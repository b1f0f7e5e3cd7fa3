"""The kept basis of a compressed supernode (Algorithm 3's U_j, V_j with L^O_j ~ V_j U_j^T,
Sec. 3.2): the factor stores U_j as W_j = (L^D_j)^{-T} U_j for its sweeps, and
rsc_get_block rebuilds U_j = (L^D_j)^T W_j on the host.  In every precision form the
rebuilt U_j is orthonormal and V_j = L^O_j U_j, to the rounding of that form's basis
products, and the device's apply of the rank-structured factor agrees with the oracle's
preconditioner built from the device's own blocks (L^D_j, V_j, U_j)."""
import numpy as np
import pytest
import scipy.linalg as sla

torch = pytest.importorskip("torch")

from workloads import grid_problem

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _apply_from_blocks(sol, p, r):
    """z = L^{-T} L^{-1} r (permuted order) from the device's blocks, off-diagonal blocks
    V_j U_j^T for compressed supernodes and L^O_j otherwise: the definition of the
    preconditioner applied to the factor the device holds."""
    first, _, _, _ = sol.supernode_info()
    rp, rows = sol.rowsets()
    ell, q = sol.ranks()
    perm = sol.perm
    y = r[perm].copy()
    blocks = [sol.block(j, (ell, q)) for j in range(len(first) - 1)]
    for j, b in enumerate(blocks):                   # forward: L y = r, columns in order
        c0, c1 = first[j], first[j + 1]
        y[c0:c1] = sla.solve_triangular(b["LD"], y[c0:c1], lower=True)
        R = rows[rp[j]:rp[j + 1]]
        if len(R):
            LO = b["V"] @ b["U"].T if b["compressed"] else b["LO"]
            y[R] -= LO @ y[c0:c1]
    for j in range(len(first) - 2, -1, -1):          # backward: L^T z = y
        b = blocks[j]
        c0, c1 = first[j], first[j + 1]
        R = rows[rp[j]:rp[j + 1]]
        if len(R):
            LO = b["V"] @ b["U"].T if b["compressed"] else b["LO"]
            y[c0:c1] -= LO.T @ y[R]
        y[c0:c1] = sla.solve_triangular(b["LD"].T, y[c0:c1], lower=False)
    z = np.empty_like(y)
    z[perm] = y
    return z


@pytest.mark.parametrize("precision,orth_tol,apply_tol", [("fp64", 1e-12, 1e-10), ("fp32", 1e-5, 1e-5),
                                                          ("bf16", 1e-5, 1e-5)])
def test_rebuilt_basis_and_apply(precision, orth_tol, apply_tol):
    from paper_1507_05593_amd import RSCSolver
    dims = (18, 17, 16)
    print("case kept basis", dims, precision, flush=True)
    p = grid_problem(dims, sigma=1.0, seed=9)
    sol = RSCSolver(p.n, p.rowptr, p.colind, precision=precision, seed=2, keep_lo=True)
    sol.factor(torch.tensor(p.values, dtype=torch.float64, device=DEV), 1e-2)
    ell, q = sol.ranks()
    comp = np.nonzero(q)[0]
    assert comp.size > 0
    for j in comp:
        b = sol.block(j, (ell, q))
        U, V, LO = b["U"], b["V"], b["LO"]
        assert U.shape[1] == q[j]
        assert np.abs(U.T @ U - np.eye(q[j])).max() <= orth_tol, (j, np.abs(U.T @ U - np.eye(q[j])).max())
        assert np.linalg.norm(V - LO @ U) <= orth_tol * max(np.linalg.norm(LO), 1e-300)
    r = np.random.default_rng(4).standard_normal(p.n)
    z = sol.apply(torch.tensor(r, dtype=torch.float64, device=DEV)).cpu().numpy()
    zb = _apply_from_blocks(sol, p, r)
    assert np.abs(z - zb).max() <= apply_tol * np.abs(zb).max(), np.abs(z - zb).max() / np.abs(zb).max()
