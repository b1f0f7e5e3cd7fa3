#!/usr/bin/env python
"""Benchmark: rank-structured supernodal Cholesky factor + PCG on one MI355X.

One step = rsc_factor (assembly, Schur updates, POTRF, TRSM, randomized
compression with truncation) followed by rsc_pcg from x0 = 0 to relative residual
1e-8 -- for the adjoint workload also the adjoint PCG and the face gradients -- on
seeded synthetic diffusion matrices whose values and right-hand sides are already
resident in HBM.  The default is the 96^3 variable-coefficient problem in the mixed
BF16/FP32/FP64 form, with the plain FP64 form timed beside it on the same GPU.

Prints one JSON line.  Fields beyond the common ones:
  fp64_form      the FP64 form's timings (mixed-precision default only)
  roofline       the kernel with the largest event-timed share of a profiled pass
                 of the same steps: algorithmic flops per launch (the method's own
                 work, counted per supernode from the symbolic plan and credited to the
                 launches that carry it) / mean launch time, against the MI355X peak of
                 its arithmetic; the executed tile flops beside them; the rocprofv3 mean
                 launch time from the committed kernel-time summary of the same build;
                 traffic from the stored rocprofv3 counter summary if the kernel source
                 is unchanged
  mfma_util      the time-weighted MFMA utilisation of the factorization:
                 (F_bf16 / P_bf16 + F_f32 / P_f32 + F_f64 / P_f64) / T_factor over
                 the algorithmic flops F of each arithmetic; also split into the
                 diagonal factorizations (panel classes) and the rest of each supernode
                 (updates, off-diagonal solve, compression), each over its own time
  pcg_hbm        PCG algorithmic bytes (SpMV, two factor sweeps, vector updates)
                 per second against 8 TB/s
  cpu_baseline   the FP64 CPU oracle on a bounded sample (see cpu_baseline())

  --calibrate-copy   only time a plain device copy of 1 GiB (the reference kernel
                     for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE) and exit
  --summarize-pmc FETCH WRITE COPYFETCH COPYWRITE --pmc-kernel NAME --pmc-last N
                     turn four rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE of the
                     bench, then of --calibrate-copy) into the kernel's HBM bytes per
                     launch over its last N dispatches (one factorization), each counter
                     scaled by what it reads for the plain copy of known size (JSON)
  --summarize-trace DIR [--trace-last-from LINE.json]
                     turn a rocprofv3 --kernel-trace --stats CSV directory into the
                     kernel-time summary (JSON on stdout): per kernel over all
                     dispatches, and over the last dispatches of the profiled pass
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense, no sparsity)
PEAK_FLOPS = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15}
PEAK_HBM = 8.0e12
KERNEL_PREC = {"gemm_staged_f64": "f64", "gemm_staged_f32": "f32", "gemm_staged_bf16x3": "bf16",
               "gemm_staged_bf16": "bf16", "gemm_staged128_f64": "f64", "gemm_staged128_f32": "f32",
               "gemm_staged128_bf16x3": "bf16", "gemm_staged128_bf16": "bf16",
               "update_waves_f64": "f64", "update_waves_f32": "f32",
               "update_waves_bf16x3": "bf16", "update_waves_bf16": "bf16", "potrf_f64": "f64",
               "gemm_potrf_f64": "f64"}
# kernel name prefix -> the source files its code lives in (digest of their concatenation)
KERNEL_SOURCE = {"gemm_staged": ("kernels_gemm.hip",), "update_waves": ("kernels_gemm.hip",),
                 "gemm_potrf": ("kernels_gemm.hip", "potrf_block.h"),
                 "potrf_f64": ("kernels_dense.hip", "potrf_block.h")}
DEFAULT_PRECISION = {"diffusion3d_96": "bf16", "batched2d_64": "fp32"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diffusion3d_96")
    ap.add_argument("--precision", default="", choices=["", "fp64", "fp32", "bf16"])
    ap.add_argument("--compare", default="auto", help="second precision timed beside (none to skip)")
    ap.add_argument("--cpu-sample-side", type=int, default=46)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-spectral", action="store_true", help="skip the spectral-coordinates timing")
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying hipGraphs")
    ap.add_argument("--no-interior", action="store_true", help="skip the interior-block run")
    ap.add_argument("--tree-tau", type=int, default=512,
                    help="tau_D of the diagonal block-tree run timed beside (0 to skip)")
    ap.add_argument("--gemm-tile", type=int, default=0, choices=[0, 64, 128],
                    help="output tile edge of the product launches (0: autotuned)")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--summarize-trace", default="", help="rocprofv3 kernel-trace CSV directory")
    ap.add_argument("--trace-last-from", default="", help="bench output whose profiled pass the trace ends with")
    ap.add_argument("--summarize-pmc", nargs=4, default=None)
    ap.add_argument("--pmc-kernel", default="gemm_staged_f64")
    ap.add_argument("--pmc-last", type=int, default=0)
    ap.add_argument("--cpu-record", action="store_true",
                    help="time the oracle on the full workload and on the bench's sample (no GPU)")
    return ap.parse_args()


# ------------------------------------------------------------------ inputs

def make_inputs(name):
    import numpy as np
    import torch

    from workloads import batched_problems, grid_problem, workload_config

    cfg = workload_config(name)
    dev = torch.device("cuda:0")
    if "count" in cfg:
        probs = batched_problems(cfg["count"], cfg["side_lo"], cfg["side_hi"], cfg["sigma"], cfg["seed"])
        pattern = ([q.n for q in probs], [q.rowptr for q in probs], [q.colind for q in probs])
        vals = torch.tensor(np.concatenate([q.values for q in probs]), device=dev)
        b = torch.tensor(np.concatenate([q.b for q in probs]), device=dev)
        desc = dict(workload=name, systems=len(probs), sides=[int(q.dims[0]) for q in probs],
                    n=int(sum(q.n for q in probs)), nnz=int(sum(q.nnz for q in probs)), sigma=cfg["sigma"])
        return cfg, None, pattern, vals, b, None, desc
    p = grid_problem(cfg["dims"], sigma=cfg["sigma"], seed=cfg["seed"], unit=cfg["unit"])
    vals = torch.tensor(p.values, device=dev)
    b = torch.tensor(p.b, device=dev)
    extra = None
    if name.startswith("adjoint"):
        extra = dict(x_target=torch.tensor(p.x_target, device=dev),
                     face_i=torch.tensor(p.face_i, device=dev), face_j=torch.tensor(p.face_j, device=dev),
                     value_map=p)
    desc = dict(workload=name, dims=list(p.dims), n=p.n, nnz=p.nnz, sigma=cfg["sigma"])
    return cfg, p, (p.n, p.rowptr, p.colind), vals, b, extra, desc


def make_solver(pattern, precision, batched, use_graph=True, gemm_tile=0):
    from paper_1507_05593_amd import RSCSolver
    kw = dict(precision=precision, seed=0, use_graph=use_graph, gemm_tile=gemm_tile)
    if batched:
        return RSCSolver.batch(*pattern, **kw)
    return RSCSolver(*pattern, **kw)


def spectral_bytes(n, nnz, m):
    """Algorithmic HBM bytes of one rsc_spectral_coordinates call (FP64, m blocks of three):
    per block the Laplacian product (pattern and 3 vectors in, 3 out), the diagonal block's
    inner products, the copy of L X, two orthogonalisation passes against the c0 earlier
    basis vectors (inner products: c0 + 3 columns read; update: c0 + 3 read, 3 written)
    and two Cholesky-QR passes (Gram: 3 columns; scaling: 3 read, 3 written); then the Ritz
    vectors (3 m columns read, 3 written) and the sign (3 read, 3 + 3 read/written)."""
    col = 8.0 * n
    total = 2 * (2 * (1 + 3) + 3) * col + 2 * 9 * col          # start block
    for k in range(m):
        c0 = 1 + 3 * (k + 1)
        total += 12.0 * nnz + 8.0 * n + 6 * col + 6 * col      # Laplacian product, A_k
        if k + 1 == m:
            break
        total += 6 * col + 2 * ((c0 + 3) + (c0 + 6)) * col + 2 * 9 * col
    return total + (3 * m + 3) * col + 9 * col


def spectral_line(pattern, m=20, reps=3):
    """Timed spectral coordinates (paper Sec. 4.3) on the workload's pattern."""
    import torch
    from paper_1507_05593_amd import RSCSolver
    sol = RSCSolver(*pattern)
    sol.spectral_coordinates(steps=m, seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, ritz = sol.spectral_coordinates(steps=m, seed=0)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    n, nnz = sol.n, sol.nnz
    byt = spectral_bytes(n, nnz, m)
    del sol
    gbs = byt / (ms * 1e-3) / 1e9
    return {"steps": m, "ms": round(ms, 3), "ritz": [float(x) for x in ritz],
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                         "frac": round(gbs / 8000.0, 4), "bytes": byt}}


def variant_run(cfg, p, vals, b, precision, steps=2, warmup=1, **opts):
    """Factor + PCG on the workload with extra solver options, timed like the headline."""
    import torch
    from paper_1507_05593_amd import RSCSolver
    t0 = time.perf_counter()
    sol = RSCSolver(p.n, p.rowptr, p.colind, precision=precision, seed=0, **opts)
    t_an = time.perf_counter() - t0
    info = None
    for _ in range(warmup):
        info = step(sol, vals, b, cfg, None)
    torch.cuda.synchronize()
    fms = pms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        info = step(sol, vals, b, cfg, None)
        fms += sol.stats()["t_factor_ms"]
        pms += info["t_pcg_ms"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st = sol.stats()
    out = {"precision": precision, "ms_per_step": round(1e3 * dt, 3), "factor_ms": round(fms / steps, 3),
           "pcg_ms": round(pms / steps, 3), "pcg_iters": info["iters"], "true_residual": info["true_residual"],
           "analyze_s": round(t_an, 3), "factor_entries": st["factor_entries"],
           "device_gb": round(st["device_bytes"] / 1e9, 2),
           "apply_gb": round(st["bytes_factor"] / 1e9, 3)}
    return sol, st, out


def tree_line(cfg, p, vals, b, precision, tau):
    """Diagonal block trees (paper Sec. 4.1-4.2, 5.3): separators of more than tau columns
    store L^D_j as a block tree, ordered by the grid positions."""
    import numpy as np
    from workloads import grid_coordinates
    sol, st, out = variant_run(cfg, p, vals, b, precision, coords=grid_coordinates(p.dims), tau_D=tau)
    first, _, _, _ = sol.supernode_info()
    c = np.diff(first)[sol.tree_depths > 0].astype(np.int64)
    out.update({"tau_D": tau, "positions": "grid", "tree_supernodes": st["tree_supernodes"],
                "tree_blocks": st["tree_blocks"], "tree_rank_sum": st["tree_rank_sum"],
                "tree_entries": st["tree_entries"], "dense_diag_entries": int(np.sum(c * (c + 1) // 2)),
                "alpha_D": st["alpha_D_used"], "restarts": st["diag_restarts"]})
    del sol
    return out


def interior_line(cfg, p, vals, b, precision):
    """Interior blocks (paper Sec. 5.1): the factor keeps only the rows of each interior
    supernode's L^O_j inside its block; the sweeps reach the rest through A."""
    sol, st, out = variant_run(cfg, p, vals, b, precision, interior=True)
    out.update({"interior_blocks": st["interior_blocks"], "dropped_entries": st["interior_dropped"]})
    del sol
    return out


# ------------------------------------------------------------------ one step

def step(sol, vals, b, cfg, extra):
    from paper_1507_05593_amd import grad_faces
    sol.factor(vals, cfg["tol"])
    x, info = sol.pcg(b, rtol=cfg["rtol"])
    out = dict(iters=info["iters"] if isinstance(info, dict) else [i["iters"] for i in info],
               true_residual=(info["true_residual"] if isinstance(info, dict)
                              else max(i["true_residual"] for i in info)))
    t_pcg = sol.stats()["t_pcg_ms"]
    if extra is not None:
        # adjoint of L = 0.5 ||x - x_t||^2: lambda = A^{-1} (x - x_t), dL/dk_f on every face
        lam, ainfo = sol.pcg(x - extra["x_target"], rtol=cfg["rtol"])
        t_pcg += sol.stats()["t_pcg_ms"]
        g = grad_faces(extra["face_i"], extra["face_j"], lam, x)
        out["adjoint_iters"] = ainfo["iters"]
        out["grad_norm"] = float(g.norm())
    out["t_pcg_ms"] = t_pcg
    return out


def run_form(pattern, vals, b, cfg, extra, precision, steps, warmup, profile, batched, use_graph=True,
             gemm_tile=0):
    import torch
    t0 = time.perf_counter()
    sol = make_solver(pattern, precision, batched, use_graph, gemm_tile)
    t_an = time.perf_counter() - t0
    info = None
    for _ in range(warmup):
        info = step(sol, vals, b, cfg, extra)
    torch.cuda.synchronize()
    fms = pms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        info = step(sol, vals, b, cfg, extra)
        fms += sol.stats()["t_factor_ms"]
        pms += info["t_pcg_ms"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    out = dict(sec_per_step=dt, analyze_s=t_an, factor_ms=fms / max(steps, 1), pcg_ms=pms / max(steps, 1),
               info=info, stats=sol.stats())
    if profile:
        # the same steps once more with an event pair around every launch
        sol.profile(True)
        pinfo = step(sol, vals, b, cfg, extra)
        torch.cuda.synchronize()
        out["kernels"] = sol.kernel_profile()
        out["classes"] = sol.profile_result()
        out["profiled_factor_ms"] = sol.stats()["t_factor_ms"]
        out["profiled_iters"] = pinfo["iters"]
        sol.profile(False)
    del sol
    torch.cuda.synchronize()
    return out


# ------------------------------------------------------------------ measurement helpers

def source_digest(kernel):
    for prefix, srcs in KERNEL_SOURCE.items():
        if kernel.startswith(prefix):
            h = hashlib.sha256()
            for src in srcs:
                with open(os.path.join(ROOT, "paper_1507_05593_amd", "csrc", src), "rb") as f:
                    h.update(f.read())
            return "+".join(srcs), h.hexdigest()[:16]
    return None, None


def stored_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current source of the kernel (else None)."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    src, dig = source_digest(kernel)
    if d.get("source") != src or d.get("source_sha256_16") != dig:
        return None
    return d.get("hbm_bytes_per_launch")


def stored_kernel_time(kernel, workload, precision):
    """Mean launch time (ms) of the kernel over the profiled pass in the committed
    rocprofv3 kernel-time summary, if it was taken on the current source (else None)."""
    path = os.path.join(ROOT, "profiles", f"kernels_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    src, dig = source_digest(kernel)
    if src is None or d.get("sources", {}).get(src) != dig:
        return None
    k = d.get("pass", {}).get(kernel)
    return k["avg_us"] * 1e-3 if k else None


def roofline(kernels, workload, precision):
    name = max((k for k in kernels if k in KERNEL_PREC), key=lambda k: kernels[k]["ms"])
    d = kernels[name]
    n = max(d["launches"], 1)
    avg_s = d["ms"] / n * 1e-3
    achieved = d["flops"] / n / avg_s if avg_s > 0 else 0.0
    tile = d["tile_flops"] / n / avg_s if avg_s > 0 else 0.0
    peak = PEAK_FLOPS[KERNEL_PREC[name]]
    out = {"kernel": name, "bound": "mfma", "achieved": round(achieved / 1e12, 3),
           "peak": round(peak / 1e12, 1), "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
           "traffic": stored_traffic(name, workload), "launches": d["launches"],
           "avg_launch_ms": round(d["ms"] / n, 5), "flops_per_launch": d["flops"] / n,
           "tile_flops_per_launch": d["tile_flops"] / n, "tile_achieved": round(tile / 1e12, 3),
           "arith": KERNEL_PREC[name]}
    rp = stored_kernel_time(name, workload, precision)
    if rp:
        out["rocprof_avg_launch_ms"] = round(rp, 5)
        out["achieved_rocprof"] = round(d["flops"] / n / rp / 1e9, 3) if rp > 0 else None
    return out


PANEL_CLASSES = ("panel_potrf", "panel_trsm", "panel_trailing")
ARITH_PEAK = {"f64": PEAK_FLOPS["f64"], "f32": PEAK_FLOPS["f32"], "bf16": PEAK_FLOPS["bf16"]}


def mfma_util(classes, factor_ms):
    """Time-weighted MFMA utilisation of the factorization and of its two parts."""
    def ideal(names):
        return sum(classes[c]["flops_arith"][a] / ARITH_PEAK[a] for c in names for a in ARITH_PEAK)
    fact = [c for c in classes if c != "pcg"]
    rest = [c for c in fact if c not in PANEL_CLASSES]
    t_diag = sum(classes[c]["ms"] for c in PANEL_CLASSES) * 1e-3
    t_rest = sum(classes[c]["ms"] for c in rest) * 1e-3
    out = {"factor": round(ideal(fact) / (factor_ms * 1e-3), 4) if factor_ms > 0 else None,
           "diag_factor": round(ideal(PANEL_CLASSES) / t_diag, 4) if t_diag > 0 else None,
           "supernode_rest": round(ideal(rest) / t_rest, 4) if t_rest > 0 else None,
           "flops_by_arith": {a: sum(classes[c]["flops_arith"][a] for c in fact) for a in ARITH_PEAK}}
    return out


def pcg_hbm(desc, stats, iters, pcg_ms):
    it = iters if isinstance(iters, int) else max(iters)
    n, nnz = desc["n"], desc["nnz"]
    # SpMV, one preconditioner apply (both sweeps: bytes_factor), ten vector passes
    per_iter = 12.0 * nnz + 24.0 * n + stats["bytes_factor"] + 10.0 * 8.0 * n
    total = (it + 1) * per_iter
    gbs = total / (pcg_ms * 1e-3) if pcg_ms > 0 else 0.0
    return {"bytes_per_iter": per_iter, "achieved": round(gbs / 1e9, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM, 4)}


def _host_info():
    info = {"cpu_count": os.cpu_count()}
    try:
        from threadpoolctl import threadpool_info
        import numpy  # noqa: F401  (loads the BLAS threadpoolctl reports)
        info["blas"] = [{"api": d.get("internal_api"), "threads": d.get("num_threads")}
                        for d in threadpool_info()]
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as f:
            info["cpu"] = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except Exception:
        pass
    return info


def _oracle_run(cfg, dims, report=False):
    """The oracle's full pipeline (symbolic, factor, PCG to rtol) on a grid of the
    workload's law: seconds per phase, iterations.  report: a line on stderr after each
    phase and after each supernode that ends 30 s of factor work."""
    from oracle.factor import Options, factor
    from oracle.ordering import symbolic
    from oracle.solve import solve
    from workloads import grid_problem

    p = grid_problem(dims, sigma=cfg["sigma"], seed=cfg["seed"], unit=cfg.get("unit", False))
    last = [time.perf_counter()]

    def say(msg):
        if report:
            print(f"oracle {'x'.join(map(str, dims))}: {msg}", file=sys.stderr, flush=True)

    def progress(j, M):
        if report and time.perf_counter() - last[0] >= 30.0:
            last[0] = time.perf_counter()
            say(f"factor: supernode {j + 1} of {M}, {last[0] - t1:.0f} s")

    t0 = time.perf_counter()
    sym = symbolic(p.n, p.rowptr, p.colind, 64)
    t1 = time.perf_counter()
    say(f"symbolic {t1 - t0:.1f} s")
    last[0] = t1
    F = factor(sym, p.n, p.rowptr, p.colind, p.values, cfg["tol"], Options(seed=0), progress=progress)
    t2 = time.perf_counter()
    say(f"factor {t2 - t1:.1f} s")
    r = solve(F, p.matrix(), p.b, rtol=cfg["rtol"])
    t3 = time.perf_counter()
    say(f"pcg {t3 - t2:.1f} s, {r.iters} iterations")
    return {"dims": list(dims), "n": p.n, "seconds": t3 - t0, "symbolic_s": t1 - t0, "factor_s": t2 - t1,
            "pcg_s": t3 - t2, "iters": int(r.iters), "true_residual": r.true_residual}


def _sample_dims(cfg, side):
    d = 2 if ("count" in cfg or len(cfg["dims"]) == 2) else 3
    return (side,) * d


def cpu_record(name, cfg, side):
    """The oracle timed on this host on the whole workload and on the bench's bounded
    sample (JSON on stdout; kept under profiles/ as cpu_oracle_<workload>.json)."""
    full = _oracle_run(cfg, tuple(cfg["dims"]), report=True)
    sample = _oracle_run(cfg, _sample_dims(cfg, side), report=True)
    print(json.dumps({"workload": name, "host": _host_info(), "full": full, "sample": sample,
                      "command": f"python bench.py --workload {name} --cpu-record --cpu-sample-side {side}"}),
          flush=True)


def cpu_baseline(name, cfg, side, gpu_desc):
    """The oracle as it stands (plain NumPy/SciPy FP64) on a bounded sample: the full
    pipeline -- symbolic analysis, factor, PCG to the same rtol -- on a grid of side
    `side` with the workload's own coefficient law, seed, tol and rtol, timed here.
    The value is the oracle's time on the whole workload as measured on a host of this
    kind (profiles/cpu_oracle_<workload>.json, written by --cpu-record), corrected by how
    this run's sample time compares with that record's; without the record, the sample
    time alone, scaled by nothing, with value null."""
    dims = _sample_dims(cfg, side)
    live = _oracle_run(cfg, dims)
    host = _host_info()
    threads = max([b.get("threads") or 1 for b in host.get("blas", [])] or [os.cpu_count() or 1])
    out = dict(value=None, unit="s", cores=int(threads), kind="oracle",
               sample=(f"oracle symbolic+factor+PCG(rtol {cfg['rtol']}) on the workload's law at "
                       f"{'x'.join(map(str, dims))} (n={live['n']}): {live['seconds']:.2f} s, "
                       f"{live['iters']} iterations"),
               sample_s=round(live["seconds"], 3))
    path = os.path.join(ROOT, "profiles", f"cpu_oracle_{name}.json")
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        if rec["sample"]["dims"] == list(dims) and rec["sample"]["seconds"] > 0:
            scale = live["seconds"] / rec["sample"]["seconds"]
            out["value"] = round(rec["full"]["seconds"] * scale, 2)
            out["measured_full_s"] = round(rec["full"]["seconds"], 2)
            out["measured_full_phases_s"] = {k: round(rec["full"][k], 1) for k in ("symbolic_s", "factor_s", "pcg_s")}
            out["host_speed_vs_record"] = round(scale, 3)
            out["sample"] += (f"; value = the oracle's measured time on the whole workload "
                              f"({rec['full']['seconds']:.1f} s, profiles/cpu_oracle_{name}.json) x this "
                              f"run's sample time / the record's ({rec['sample']['seconds']:.2f} s)")
    return out


def calibrate_copy():
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    c = torch.empty_like(a)
    for _ in range(5):
        c.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        c.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "sec": dt,
                      "GBps": round(2 * nbytes / dt / 1e9, 1)}), flush=True)


_MODE_NAMES = {0: "f64", 1: "f32", 2: "bf16x3", 3: "bf16"}


def profile_name(rocprof_name):
    """Kernel name of the library's profile for a rocprofv3 kernel name (or None)."""
    import re
    if re.search(r"k_gemm_staged<0, 64, true>", rocprof_name):
        return "gemm_potrf_f64"
    m = re.search(r"k_gemm_staged<(\d), (\d+)", rocprof_name)
    if m:
        return f"gemm_staged{'128' if m.group(2) == '128' else ''}_{_MODE_NAMES[int(m.group(1))]}"
    m = re.search(r"k_update_waves<(\d)>", rocprof_name)
    if m:
        return f"update_waves_{_MODE_NAMES[int(m.group(1))]}"
    m = re.search(r"rsc::k_(\w+)", rocprof_name)
    return m.group(1) if m else None


def summarize_trace(d, last_from):
    """Per-kernel dispatch counts and durations of a rocprofv3 kernel trace: over all
    dispatches, and over the last N dispatches of each kernel, N = its launch count in
    the profiled pass of the bench line in `last_from` (that pass is the run's last)."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                             r["Kernel_Name"]))
    rows.sort()
    per = {}
    for _, dur, nm in rows:
        per.setdefault(nm, []).append(dur)
    allk = {nm: {"calls": len(v), "total_ms": sum(v) * 1e-6, "avg_us": sum(v) / len(v) * 1e-3}
            for nm, v in per.items()}
    out = {"all": dict(sorted(allk.items(), key=lambda kv: -kv[1]["total_ms"])),
           "sources": {"+".join(src): source_digest(k)[1] for k, src in KERNEL_SOURCE.items()}}
    if last_from:
        with open(last_from) as fh:
            line = json.loads(next(l for l in reversed(fh.read().splitlines()) if l.startswith('{"metric"')))
        out["bench_line"] = line
        pas = {}
        for k, v in line.get("kernels", {}).items():
            durs = [x for nm, xs in per.items() if profile_name(nm) == k for x in xs]
            n = v["launches"]
            if len(durs) < n:
                continue
            # last n dispatches of this kernel (trace order)
            seq = sorted((t, dur) for t, dur, nm in rows if profile_name(nm) == k)[-n:]
            pas[k] = {"launches": n, "avg_us": sum(x for _, x in seq) / n * 1e-3,
                      "bench_event_avg_us": v["ms"] / n * 1e3}
        out["pass"] = pas
    print(json.dumps(out, indent=1), flush=True)


def _pmc_rows(d, counter):
    """(dispatch id, kernel name, value) of one counter in a rocprofv3 --pmc CSV directory."""
    import csv
    import glob
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    return sorted(out)


def summarize_pmc(dirs, kernel, last, workload):
    fetch_d, write_d, cfetch_d, cwrite_d = dirs
    def per_dispatch(d, counter, pick):
        rows = [x for x in _pmc_rows(d, counter) if pick(x[1])]
        return rows
    mine = lambda nm: profile_name(nm) == kernel
    fr = per_dispatch(fetch_d, "FETCH_SIZE", mine)[-last:]
    wr = per_dispatch(write_d, "WRITE_SIZE", mine)[-last:]
    copy = lambda nm: "copy" in nm.lower() or "elementwise" in nm.lower() or "direct_copy" in nm.lower()
    cf = per_dispatch(cfetch_d, "FETCH_SIZE", copy)
    cw = per_dispatch(cwrite_d, "WRITE_SIZE", copy)
    nbytes = 1 << 30
    # the copy's last dispatch moves exactly nbytes each way
    fkib, wkib = cf[-1][2], cw[-1][2]
    ff, wf = nbytes / 1024.0 / fkib, nbytes / 1024.0 / wkib
    f_avg = sum(x[2] for x in fr) / len(fr)
    w_avg = sum(x[2] for x in wr) / len(wr)
    src, dig = source_digest(kernel)
    out = {"kernel": kernel, "workload": workload, "source": src, "source_sha256_16": dig,
           "dispatches_used": len(fr), "fetch_kib_per_dispatch": f_avg, "write_kib_per_dispatch": w_avg,
           "copy_calibration": {"bytes": nbytes, "fetch_kib": fkib, "write_kib": wkib, "fetch_factor": ff,
                                "write_factor": wf},
           "hbm_bytes_per_launch": 1024.0 * (f_avg * ff + w_avg * wf),
           "commands": [
               "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch -o run -- python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-profile --compare none --no-graph --no-spectral --tree-tau 0 --no-interior",
               "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write -o run -- python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-profile --compare none --no-graph --no-spectral --tree-tau 0 --no-interior",
               "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/copyfetch -o run -- python3 bench.py --calibrate-copy",
               "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/copywrite -o run -- python3 bench.py --calibrate-copy",
               f"python bench.py --summarize-pmc OUT/fetch OUT/write OUT/copyfetch OUT/copywrite --pmc-kernel {kernel} --pmc-last {last}"],
           "note": "last N dispatches of the kernel in each counter run = one factorization; FETCH_SIZE and "
                   "WRITE_SIZE scaled by what they read for a plain 1 GiB device copy"}
    print(json.dumps(out, indent=1), flush=True)


# ------------------------------------------------------------------ main

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this path runs on one GPU (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design only and is not implemented", file=sys.stderr)
        sys.exit(2)
    name = args.workload
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.trace_last_from)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.pmc_kernel, args.pmc_last, name)
        return
    if args.cpu_record:
        from workloads import workload_config
        cpu_record(name, workload_config(name), args.cpu_sample_side)
        return
    import torch
    if args.calibrate_copy:
        calibrate_copy()
        return
    precision = args.precision or DEFAULT_PRECISION.get(name, "fp64")
    compare = args.compare
    if compare == "auto":
        compare = "fp64" if precision != "fp64" and name == "diffusion3d_96" else "none"
    cfg, p, pattern, vals, b, extra, desc = make_inputs(name)
    batched = "count" in cfg
    res = run_form(pattern, vals, b, cfg, extra, precision, args.steps, args.warmup, not args.no_profile, batched,
                   not args.no_graph, args.gemm_tile)
    cmp = None
    if compare != "none":
        cmp = run_form(pattern, vals, b, cfg, extra, compare, args.steps, args.warmup, False, batched,
                       not args.no_graph, args.gemm_tile)
    info, st = res["info"], res["stats"]
    line = {
        "metric": "factor+PCG s to rel.res 1e-8, MFMA util; mixed-prec vs FP64 form, same GPU",
        "value": round(res["sec_per_step"], 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * res["sec_per_step"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16+f32+f64"}[precision],
        "data": "synthetic",
        "config": dict(desc, tol=cfg["tol"], rtol=cfg["rtol"], precision=precision,
                       gemm_tile=args.gemm_tile or "autotuned"),
        "factor_ms": round(res["factor_ms"], 3),
        "pcg_ms": round(res["pcg_ms"], 3),
        "pcg_iters": info["iters"],
        "true_residual": info["true_residual"],
        "analyze_s": round(res["analyze_s"], 3),
    }
    if "adjoint_iters" in info:
        line["adjoint_iters"] = info["adjoint_iters"]
    fl = sum(st[k] for k in ("flops_potrf", "flops_trsm", "flops_update", "flops_sample", "flops_orth",
                             "flops_trunc"))
    line["factor_tflop"] = round(fl / 1e12, 4)
    line["factor_tflop_per_s"] = round(fl / (res["factor_ms"] * 1e-3) / 1e12, 3)
    line["device_gb"] = round(st["device_bytes"] / 1e9, 2)
    line["factor_entries"] = st["factor_entries"]
    line["tile_tuner"] = {"launches_tuned": st["gemm_tuned"], "launches_128": st["gemm_tile128"]}
    if cmp:
        line["fp64_form" if compare == "fp64" else "compare_form"] = {
            "precision": compare, "ms_per_step": round(1e3 * cmp["sec_per_step"], 3),
            "factor_ms": round(cmp["factor_ms"], 3), "pcg_ms": round(cmp["pcg_ms"], 3),
            "pcg_iters": cmp["info"]["iters"], "true_residual": cmp["info"]["true_residual"]}
        line["speedup_vs_" + compare] = round(cmp["sec_per_step"] / res["sec_per_step"], 3)
    if "kernels" in res:
        ks = res["kernels"]
        line["roofline"] = roofline(ks, name, precision)
        mu = mfma_util(res["classes"], res["profiled_factor_ms"])
        line["mfma_util"] = mu["factor"]
        line["mfma_util_parts"] = {k: mu[k] for k in ("diag_factor", "supernode_rest")}
        top = sorted(ks.items(), key=lambda kv: -kv[1]["ms"])[:8]
        line["kernels"] = {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                               "tflop_s": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2) if v["ms"] > 0 else 0.0,
                               "tile_tflop_s": round(v["tile_flops"] / (v["ms"] * 1e-3) / 1e12, 2)
                               if v["ms"] > 0 else 0.0}
                           for k, v in top}
        line["classes_ms"] = {k: round(v["ms"], 3) for k, v in res["classes"].items() if v["launches"]}
    line["pcg_hbm"] = pcg_hbm(desc, st, info["iters"], res["pcg_ms"])
    if not batched and not args.no_spectral:
        line["spectral_coordinates"] = spectral_line(pattern)
    if not batched and args.tree_tau > 0 and len(p.dims) == 3 and extra is None:
        line["diag_trees"] = tree_line(cfg, p, vals, b, precision, args.tree_tau)
    if not batched and not args.no_interior and extra is None and cfg["tol"] > 0:
        line["interior_blocks"] = interior_line(cfg, p, vals, b, precision)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(name, cfg, args.cpu_sample_side, desc)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
