"""Device memory through the caller's allocator (rsc_set_allocator, here torch's caching
allocator): the factor and PCG give the same bits as with hipMalloc, the memory shows up
in torch's accounting, and it goes back when the solver is destroyed."""
import gc

import pytest

from workloads import grid_problem


@pytest.mark.gpu
def test_torch_allocator_same_result_and_accounting():
    torch = pytest.importorskip("torch")
    from paper_1507_05593_amd import RSCSolver, use_torch_allocator
    print("case torch allocator, grid 20x18x16", flush=True)
    p = grid_problem((20, 18, 16), sigma=1.0, seed=1)
    vals = torch.tensor(p.values, dtype=torch.float64, device="cuda:0")
    b = torch.tensor(p.b, dtype=torch.float64, device="cuda:0")

    def run():
        sol = RSCSolver(p.n, p.rowptr, p.colind, seed=3)
        sol.factor(vals, 1e-2)
        x, info = sol.pcg(b, rtol=1e-10)
        torch.cuda.synchronize()
        return sol, x.clone(), info

    sol0, x0, info0 = run()
    del sol0
    gc.collect()
    use_torch_allocator(True)
    try:
        before = torch.cuda.memory_allocated()
        sol1, x1, info1 = run()
        grown = torch.cuda.memory_allocated() - before
        arena = 8.0 * sol1.stats()["n"]          # at least the solution-sized work vectors
        assert grown > arena, (grown, arena)
        assert info1["iters"] == info0["iters"]
        assert torch.equal(x1, x0)
        del sol1
        gc.collect()
        assert torch.cuda.memory_allocated() - before < 1 << 20
    finally:
        gc.collect()
        use_torch_allocator(False)
