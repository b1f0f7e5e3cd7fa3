"""Writes oracle reference results for a full-size workload (CPU, oracle only).

Usage: python tests/golden/make_oracle_reference.py diffusion3d_96 [--symbolic-only]
Output: tests/golden/oracle_<workload>.json with the symbolic sizes and SHA-256
digests of the ordering and supernode structure, the kept rank of every compressed
supernode, and the PCG iteration count and residuals of the oracle's
rank-structured factor (seed 0, the benchmark's settings), the oracle's solution at
4096 indices drawn from numpy.random.default_rng(20151) (for element-wise comparison),
and the host it ran on (cores, BLAS threads, per-phase seconds).  The full run takes
minutes at full size; ``--symbolic-only`` refreshes the structure digests of an
existing file.  The tests compare against the stored file.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.factor import Options, factor  # noqa: E402
from oracle.ordering import symbolic  # noqa: E402
from oracle.solve import solve  # noqa: E402
from workloads import batched_problems, grid_problem, workload_config  # noqa: E402


def structure_digests(sym):
    """SHA-256 of the permutation (int64 new -> old), the supernode boundaries
    (int64), parent / level / kind (int32) and the concatenated row sets (int64)."""
    def h(a, dt):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=dt).tobytes()).hexdigest()
    rows = np.concatenate([np.asarray(r, dtype=np.int64) for r in sym.rows]) if sym.M else np.zeros(0)
    return dict(perm=h(sym.perm, "<i8"), first=h(sym.first, "<i8"), parent=h(sym.parent, "<i4"),
                level=h(sym.level, "<i4"), kind=h(sym.kind, "<i4"), rows=h(rows, "<i8"))


def host_info():
    """Cores and BLAS threads of the host the oracle ran on."""
    info = dict(cpu_count=os.cpu_count())
    try:
        from threadpoolctl import threadpool_info
        info["blas"] = [dict(api=d.get("internal_api"), threads=d.get("num_threads")) for d in threadpool_info()]
    except Exception:  # pragma: no cover - threadpoolctl is optional
        pass
    try:
        with open("/proc/cpuinfo") as f:
            info["cpu"] = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except Exception:  # pragma: no cover
        pass
    return info


def solution_sample(x, k=4096):
    """x at k distinct indices from a fixed generator, sorted."""
    idx = np.sort(np.random.default_rng(20151).choice(x.size, size=min(k, x.size), replace=False))
    return dict(idx=[int(i) for i in idx], x=[float(v) for v in x[idx]])


def main_batched(name):
    """Independent systems: each one alone through the oracle (its own dissection,
    supernodes numbered within the system, sample seed 0)."""
    cfg = workload_config(name)
    probs = batched_problems(cfg["count"], cfg["side_lo"], cfg["side_hi"], cfg["sigma"], cfg["seed"])
    systems = []
    t0 = time.time()
    for i, p in enumerate(probs):
        sym = symbolic(p.n, p.rowptr, p.colind, 64)
        F = factor(sym, p.n, p.rowptr, p.colind, p.values, cfg["tol"], Options(seed=0))
        res = solve(F, p.matrix(), p.b, rtol=cfg["rtol"])
        systems.append(dict(side=int(p.dims[0]), n=p.n, supernodes=int(sym.M), q_sum=int(sum(F.q)),
                            compressed=int(sum(1 for e in F.ell if e)), pcg_iters=int(res.iters),
                            true_residual=res.true_residual, x_norm=float((res.x @ res.x) ** 0.5),
                            structure_sha256=structure_digests(sym)))
        print(i, systems[-1]["side"], systems[-1]["pcg_iters"], round(time.time() - t0, 1), flush=True)
    out = dict(workload=name, count=len(probs), tol=cfg["tol"], rtol=cfg["rtol"], seed=0, systems=systems,
               seconds=time.time() - t0, written_by="tests/golden/make_oracle_reference.py (oracle only)")
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(out, f)


def main(name, symbolic_only=False):
    cfg = workload_config(name)
    if "count" in cfg:
        return main_batched(name)
    p = grid_problem(cfg["dims"], sigma=cfg["sigma"], seed=cfg["seed"], unit=cfg["unit"])
    t0 = time.time()
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    t1 = time.time()
    path = os.path.join(HERE, f"oracle_{name}.json")
    if symbolic_only:
        with open(path) as f:
            out = json.load(f)
        out["structure_sha256"] = structure_digests(sym)
        with open(path, "w") as f:
            json.dump(out, f)
        print(json.dumps(out["structure_sha256"]))
        return
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
               x_sample=solution_sample(res.x),
               seconds=dict(symbolic=t1 - t0, factor=t2 - t1, pcg=t3 - t2), host=host_info(),
               structure_sha256=structure_digests(sym),
               written_by="tests/golden/make_oracle_reference.py (oracle only)")
    with open(path, "w") as f:
        json.dump(out, f)
    print(json.dumps({k: out[k] for k in ("pcg_iters", "true_residual", "seconds")}))


if __name__ == "__main__":
    main(sys.argv[1], "--symbolic-only" in sys.argv[2:])
