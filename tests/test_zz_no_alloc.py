"""The allocation-free preconditioner apply (rsc_apply_preconditioner_noalloc) against
rsc_apply_preconditioner, through the C ABI: the same kernels on the same factor, so
the results are identical bit for bit; two calls in a row, the second on a smaller
system, each in the FP64 form, after a mixed-precision factorization (FP32 sweep
operands) and with interior blocks (their solves in the same apply)."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import grid_problem

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _apply_both(sol, r):
    from paper_1507_05593_amd import lib
    z_ref = sol.apply(r)
    z = torch.full_like(r, float("nan"))
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = lib().rsc_apply_preconditioner_noalloc(sol._h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()),
                                                  stream)
    assert code == 0, lib().rsc_last_error()
    torch.cuda.synchronize()
    return z_ref.cpu().numpy(), z.cpu().numpy()


@pytest.mark.parametrize("precision,interior", [("fp64", False), ("bf16", False), ("fp64", True)])
def test_noalloc_apply_equals_apply_two_calls_smaller_second(precision, interior):
    from paper_1507_05593_amd import RSCSolver
    print("case noalloc apply", precision, interior, flush=True)
    rng = np.random.default_rng(5)
    for dims in ((22, 21, 20), (9, 8, 7)):          # the second call's system is smaller
        p = grid_problem(dims, sigma=1.0, seed=3)
        sol = RSCSolver(p.n, p.rowptr, p.colind, precision=precision, seed=1, interior=interior)
        sol.factor(torch.tensor(p.values, dtype=torch.float64, device=DEV), 1e-2)
        r = torch.tensor(rng.standard_normal(p.n), dtype=torch.float64, device=DEV)
        z_ref, z = _apply_both(sol, r)
        assert np.all(np.isfinite(z))
        assert np.array_equal(z, z_ref), np.abs(z - z_ref).max()


def test_noalloc_apply_needs_a_factor():
    from paper_1507_05593_amd import RSCSolver, lib
    p = grid_problem((6, 5, 4), sigma=1.0, seed=3)
    sol = RSCSolver(p.n, p.rowptr, p.colind)
    r = torch.zeros(p.n, dtype=torch.float64, device=DEV)
    z = torch.zeros_like(r)
    code = lib().rsc_apply_preconditioner_noalloc(sol._h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()),
                                                  None)
    assert code == 8   # RSC_ERR_STATE
