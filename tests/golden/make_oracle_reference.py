"""Writes oracle reference results for a full-size workload (CPU, oracle only).

Usage: python tests/golden/make_oracle_reference.py diffusion3d_96
Output: tests/golden/oracle_<workload>.json with the symbolic sizes, the kept rank of
every compressed supernode, and the PCG iteration count and residuals of the
oracle's rank-structured factor (seed 0, the benchmark's settings).  Takes a long
time at full size; the GPU tests compare against the stored file.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.factor import Options, factor  # noqa: E402
from oracle.ordering import symbolic  # noqa: E402
from oracle.solve import solve  # noqa: E402
from workloads import grid_problem, workload_config  # noqa: E402


def main(name):
    cfg = workload_config(name)
    p = grid_problem(cfg["dims"], sigma=cfg["sigma"], seed=cfg["seed"], unit=cfg["unit"])
    t0 = time.time()
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    t1 = time.time()
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, cfg["tol"], Options(seed=0))
    t2 = time.time()
    res = solve(F, p.matrix(), p.b, rtol=cfg["rtol"])
    t3 = time.time()
    comp = [j for j in range(sym.M) if F.ell[j]]
    out = dict(workload=name, n=p.n, nnz=p.nnz, supernodes=int(sym.M), levels=int(sym.level.max() + 1),
               tol=cfg["tol"], rtol=cfg["rtol"], seed=0,
               compressed=[int(j) for j in comp], ell=[int(F.ell[j]) for j in comp],
               q=[int(F.q[j]) for j in comp],
               pcg_iters=int(res.iters), rel_residual=res.rel_residual, true_residual=res.true_residual,
               x_norm=float((res.x @ res.x) ** 0.5), x_sum=float(res.x.sum()),
               seconds=dict(symbolic=t1 - t0, factor=t2 - t1, pcg=t3 - t2),
               written_by="tests/golden/make_oracle_reference.py (oracle only)")
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(out, f)
    print(json.dumps({k: out[k] for k in ("pcg_iters", "true_residual", "seconds")}))


if __name__ == "__main__":
    main(sys.argv[1])
