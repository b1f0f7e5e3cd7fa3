"""GPU parity of the spectral coordinates (§4.3) against the oracle's block Lanczos."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.spectral import spectral_coordinates as o_spectral
from workloads import grid_problem
from workloads.grids import batched_problems

pytestmark = pytest.mark.gpu


def _sol(p, **kw):
    from paper_1507_05593_amd import RSCSolver
    return RSCSolver(p.n, p.rowptr, p.colind, **kw)


def _angles(A, B):
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    return np.linalg.svd(qa.T @ qb, compute_uv=False)


@pytest.mark.parametrize("dims,steps,seed", [((12, 7, 5), 30, 1), ((40, 30), 25, 2), ((8, 8, 8), 20, 3),
                                             ((20, 17, 15), 12, 4)])
def test_spectral_coordinates_match_oracle(dims, steps, seed):
    print("case spectral", dims, steps, seed, flush=True)
    p = grid_problem(dims, sigma=1.0, seed=0)
    sol = _sol(p)
    xyz, ritz = sol.spectral_coordinates(steps=steps, seed=seed)
    Y = xyz.cpu().numpy()
    Yo, to = o_spectral(p.n, p.rowptr, p.colind, steps=steps, seed=seed)
    print("ritz", ritz, "oracle", to, flush=True)
    assert np.allclose(ritz, to, rtol=1e-9, atol=1e-12), (ritz, to)
    # the three-dimensional subspace always; single vectors where the Ritz values are apart
    assert _angles(Y, Yo).min() > 1 - 1e-8
    gaps = np.diff(np.concatenate([[-np.inf], to, [np.inf]]))
    for c in range(3):
        if min(gaps[c], gaps[c + 1]) > 1e-6 * abs(to).max():
            assert abs(Y[:, c] @ Yo[:, c]) > 1 - 1e-8, (c, Y[:, c] @ Yo[:, c])
            assert np.allclose(Y[:, c], Yo[:, c], atol=1e-6), c     # the same sign convention
    assert np.allclose(Y.T @ Y, np.eye(3), atol=1e-10)
    assert np.abs(Y.sum(axis=0)).max() < 1e-8


def test_spectral_coordinates_argument_errors():
    from paper_1507_05593_amd._lib import RSC_ERR_INVALID_ARG, RSCError
    p = grid_problem((6, 5), sigma=0.0, seed=0)
    sol = _sol(p)
    for steps in (0, 31, 10):                 # 10: 1 + 30 > 30 indices
        with pytest.raises(RSCError) as e:
            sol.spectral_coordinates(steps=steps)
        assert e.value.code == RSC_ERR_INVALID_ARG
    from paper_1507_05593_amd import RSCSolver
    ps = batched_problems(2, 8, 10, 1.0, 0)
    b = RSCSolver.batch([q.n for q in ps], [q.rowptr for q in ps], [q.colind for q in ps])
    with pytest.raises(RSCError) as e:
        b.spectral_coordinates(steps=3)
    assert e.value.code == RSC_ERR_INVALID_ARG
