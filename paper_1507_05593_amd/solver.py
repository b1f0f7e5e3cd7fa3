"""Python face of the solver: argument marshalling around the C ABI (include/rsc.h).

Every numeric step runs in the HIP library; torch supplies device memory and the
current stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import (RSC_ERR_NOT_CONVERGED, Options, PcgResult, Profile, RSCError, Stats, check, lib)

PRECISIONS = {"fp64": _lib.RSC_FP64, "bf16": _lib.RSC_MIXED_BF16, "fp32": _lib.RSC_MIXED_FP32}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def _dev_f64(t, n, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with {n} entries")
    return t


_allocator_refs = None   # the ctypes callbacks must outlive their use by the library


def use_torch_allocator(on: bool = True) -> None:
    """Route the library's device memory (rsc_set_allocator) through torch's caching
    allocator, or back to hipMalloc with on=False.  Only while no solver exists."""
    global _allocator_refs
    L = lib()
    if not on:
        check(L.rsc_set_allocator(None, None, None), "rsc_set_allocator")
        _allocator_refs = None
        return

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except RuntimeError:        # out of memory: the library reports RSC_ERR_OUT_OF_MEMORY
            return None

    def _release(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    refs = (_lib.ALLOC_FN(_alloc), _lib.RELEASE_FN(_release))
    check(L.rsc_set_allocator(_lib.fnptr(refs[0]), _lib.fnptr(refs[1]), None), "rsc_set_allocator")
    _allocator_refs = refs


def make_options(leaf_max=64, tau_O=32, oversample=10, power_iters=0, alpha_O=1.0, seed=0,
                 precision="fp64", use_graph=True, retry=True, gemm_tile=0, keep_lo=False,
                 sweep_small_c=64, tau_D=0, alpha_D=0.5, interior=False) -> Options:
    o = Options()
    lib().rsc_default_options(C.byref(o))
    o.leaf_max, o.tau_O, o.oversample, o.power_iters = leaf_max, tau_O, oversample, power_iters
    o.alpha_O, o.seed = float(alpha_O), int(seed)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.use_graph, o.retry = int(bool(use_graph)), int(bool(retry))
    o.gemm_tile = int(gemm_tile)
    o.keep_lo = int(bool(keep_lo))
    o.sweep_small_c = int(sweep_small_c)
    o.tau_D, o.alpha_D = int(tau_D), float(alpha_D)
    o.interior = int(bool(interior))
    return o


class RSCSolver:
    """Rank-structured supernodal Cholesky + PCG on one GPU.

    ``RSCSolver(n, rowptr, colind, **options)`` runs the symbolic phase on the host
    (no GPU needed); ``factor(values, tol)`` and ``pcg(b, rtol)`` run on the device.
    For several independent systems pass lists to ``RSCSolver.batch``.
    """

    def __init__(self, n=None, rowptr=None, colind=None, _handle=None, _systems=1, coords=None, **opts):
        """``coords``: positions of the indices (``n x 3`` host array, or ``"spectral"``
        for the three spectral coordinates computed on the device first); with
        ``tau_D > 0`` they order the columns of the block-tree separators."""
        L = lib()
        self._opts = make_options(**opts)
        if _handle is None:
            rp = np.ascontiguousarray(rowptr, dtype=np.int64)
            ci = np.ascontiguousarray(colind, dtype=np.int32)
            if isinstance(coords, str):
                if coords != "spectral":
                    raise ValueError("coords must be an n x 3 array or 'spectral'")
                pre = RSCSolver(n, rowptr, colind, **{k: v for k, v in opts.items() if k != "tau_D"})
                xyz, _ = pre.spectral_coordinates()
                coords = xyz.cpu().numpy()
                del pre
            h = C.c_void_p()
            if coords is None:
                check(L.rsc_analyze(int(n), rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
                                    C.byref(self._opts), C.byref(h)), "rsc_analyze")
            else:
                xyz = np.ascontiguousarray(coords, dtype=np.float64)
                if xyz.shape != (int(n), 3):
                    raise ValueError("coords must have shape (n, 3)")
                check(L.rsc_analyze_coords(int(n), rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
                                           xyz.ctypes.data_as(C.c_void_p), C.byref(self._opts), C.byref(h)),
                      "rsc_analyze_coords")
            _handle = h
        self._h = _handle
        n_, nnz, M, lev, sysn = (C.c_int64() for _ in range(5))
        check(L.rsc_get_sizes(self._h, C.byref(n_), C.byref(nnz), C.byref(M), C.byref(lev), C.byref(sysn)))
        self.n, self.nnz, self.supernodes, self.levels, self.systems = (
            n_.value, nnz.value, M.value, lev.value, sysn.value)
        self._keep = []
        self._struct = None   # (first, rowptr of R_j): fixed by the symbolic phase
        self.generation = 0   # successful factorizations so far

    @classmethod
    def batch(cls, ns, rowptrs, colinds, **opts):
        L = lib()
        o = make_options(**opts)
        rps = [np.ascontiguousarray(r, dtype=np.int64) for r in rowptrs]
        cis = [np.ascontiguousarray(c, dtype=np.int32) for c in colinds]
        cnt = len(rps)
        n_arr = (C.c_int64 * cnt)(*[int(x) for x in ns])
        rp_arr = (C.c_void_p * cnt)(*[r.ctypes.data for r in rps])
        ci_arr = (C.c_void_p * cnt)(*[c.ctypes.data for c in cis])
        h = C.c_void_p()
        check(L.rsc_analyze_batch(cnt, n_arr, rp_arr, ci_arr, C.byref(o), C.byref(h)), "rsc_analyze_batch")
        return cls(_handle=h, **opts)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().rsc_destroy(h)   # synchronises the handle's device itself
            except Exception:
                pass
            self._h = None

    # ---------------------------------------------------------------- numeric
    def factor(self, values: torch.Tensor, tol: float = 0.0):
        v = _dev_f64(values, self.nnz, "values")
        check(lib().rsc_factor(self._h, _ptr(v), float(tol), _stream()), "rsc_factor")
        self.generation += 1
        return self

    def pcg(self, b: torch.Tensor, rtol: float = 1e-8, max_iter: int = 1000, x: torch.Tensor = None,
            raise_on_failure: bool = True):
        b = _dev_f64(b, self.n, "b")
        if x is None:
            x = torch.empty_like(b)
        res = (PcgResult * self.systems)()
        code = lib().rsc_pcg(self._h, _ptr(b), _ptr(x), float(rtol), int(max_iter), _stream(), res)
        out = [dict(iters=r.iters, converged=bool(r.converged), rel_residual=r.rel_residual,
                    true_residual=r.true_residual) for r in res]
        if code != 0 and (raise_on_failure or code != RSC_ERR_NOT_CONVERGED):
            raise RSCError(code, "rsc_pcg")
        return x, (out[0] if self.systems == 1 else out)

    def apply(self, r: torch.Tensor) -> torch.Tensor:
        r = _dev_f64(r, self.n, "r")
        z = torch.empty_like(r)
        check(lib().rsc_apply_preconditioner(self._h, _ptr(r), _ptr(z), _stream()), "rsc_apply_preconditioner")
        return z

    def apply_noalloc(self, r: torch.Tensor, z: torch.Tensor) -> torch.Tensor:
        """z = M^{-1} r into the caller's z through rsc_apply_preconditioner_noalloc (no
        device allocation by the library; see include/rsc.h for the shared buffer)."""
        r = _dev_f64(r, self.n, "r")
        z = _dev_f64(z, self.n, "z")
        check(lib().rsc_apply_preconditioner_noalloc(self._h, _ptr(r), _ptr(z), _stream()),
              "rsc_apply_preconditioner_noalloc")
        return z

    def grad_values(self, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
        lam = _dev_f64(lam, self.n, "lambda")
        x = _dev_f64(x, self.n, "x")
        g = torch.empty(self.nnz, dtype=torch.float64, device=lam.device)
        check(lib().rsc_grad_values(self._h, _ptr(lam), _ptr(x), _ptr(g), _stream()), "rsc_grad_values")
        return g

    # ---------------------------------------------------------------- inspection
    def spectral_coordinates(self, steps: int = 20, seed: int = 0):
        """Positions (n, 3) of the indices from the graph Laplacian of the pattern (§4.3)
        and the three Ritz values (rsc_spectral_coordinates)."""
        xyz = torch.empty(3 * self.n, dtype=torch.float64, device="cuda")
        ritz = (C.c_double * 3)()
        check(lib().rsc_spectral_coordinates(self._h, int(steps), int(seed), _ptr(xyz), ritz, _stream()))
        return xyz.view(3, self.n).t(), np.array(ritz[:])

    @property
    def tree_depths(self) -> np.ndarray:
        """Depth of each supernode's diagonal block tree (0: dense L^D_j)."""
        d = np.empty(self.supernodes, dtype=np.int32)
        check(lib().rsc_get_tree_depths(self._h, d.ctypes.data_as(C.c_void_p)))
        return d

    @property
    def perm(self) -> np.ndarray:
        p = np.empty(self.n, dtype=np.int64)
        check(lib().rsc_get_permutation(self._h, p.ctypes.data_as(C.c_void_p)))
        return p

    def supernode_info(self):
        M = self.supernodes
        first = np.empty(M + 1, dtype=np.int64)
        parent, level, kind = (np.empty(M, dtype=np.int32) for _ in range(3))
        check(lib().rsc_get_supernodes(self._h, *(a.ctypes.data_as(C.c_void_p) for a in (first, parent, level, kind))))
        return first, parent, level, kind

    def rowsets(self):
        rp = np.empty(self.supernodes + 1, dtype=np.int64)
        check(lib().rsc_get_rowsets(self._h, rp.ctypes.data_as(C.c_void_p), None))
        rows = np.empty(int(rp[-1]), dtype=np.int64)
        check(lib().rsc_get_rowsets(self._h, rp.ctypes.data_as(C.c_void_p), rows.ctypes.data_as(C.c_void_p)))
        return rp, rows

    def ranks(self):
        ell = np.empty(self.supernodes, dtype=np.int32)
        q = np.empty(self.supernodes, dtype=np.int32)
        check(lib().rsc_get_ranks(self._h, ell.ctypes.data_as(C.c_void_p), q.ctypes.data_as(C.c_void_p)))
        return ell, q

    def block(self, j, ranks=None):
        """Host copies of supernode j's blocks (rsc_get_block).  ranks: the (ell, q)
        pair of ranks() when the caller already holds it (they change with each factor)."""
        if self._struct is None:
            first, _, _, _ = self.supernode_info()
            rp, _ = self.rowsets()
            self._struct = (first, rp)
        first, rp = self._struct
        c = int(first[j + 1] - first[j]); r = int(rp[j + 1] - rp[j])
        ell, q = self.ranks() if ranks is None else ranks
        qj = int(q[j])
        LD = np.zeros((c, c), order="F"); LO = np.zeros((r, c), order="F")
        V = np.zeros((r, qj), order="F"); U = np.zeros((c, qj), order="F")
        # the dense L^O_j of a compressed supernode exists only with keep_lo
        want_lo = not (ell[j] > 0 and not self._opts.keep_lo)
        check(lib().rsc_get_block(self._h, int(j), LD.ctypes.data_as(C.c_void_p),
                                  LO.ctypes.data_as(C.c_void_p) if want_lo else None,
                                  V.ctypes.data_as(C.c_void_p), U.ctypes.data_as(C.c_void_p)), "rsc_get_block")
        return dict(LD=np.tril(LD), LO=LO if want_lo else None, V=V, U=U, compressed=bool(ell[j] > 0))

    def stats(self) -> dict:
        s = Stats()
        check(lib().rsc_get_stats(self._h, C.byref(s)))
        return {name: getattr(s, name) for name, _ in Stats._fields_}

    def profile(self, on: bool = True):
        check(lib().rsc_profile_enable(self._h, int(on)))

    def profile_result(self) -> dict:
        p = Profile()
        check(lib().rsc_get_profile(self._h, C.byref(p)))
        return {k: dict(launches=p.launches[i], ms=p.ms[i], flops=p.flops[i], tile_flops=p.tile_flops[i],
                        flops_arith={a: p.flops_arith[i][q] for q, a in enumerate(_lib.ARITHS)})
                for i, k in enumerate(_lib.K_CLASSES)}

    def kernel_profile(self) -> dict:
        """Per-kernel launches, hipEvent ms, algorithmic and executed tile flops while profiling."""
        out = {}
        for k in range(_lib.RSC_KERNELS):
            name, n, ms, fl, tf = C.c_char_p(), C.c_int64(), C.c_double(), C.c_double(), C.c_double()
            check(lib().rsc_get_kernel_profile(self._h, k, C.byref(name), C.byref(n), C.byref(ms), C.byref(fl),
                                               C.byref(tf)))
            out[name.value.decode()] = dict(launches=n.value, ms=ms.value, flops=fl.value, tile_flops=tf.value)
        return out


def grad_faces(face_i: torch.Tensor, face_j: torch.Tensor, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Face-coefficient gradient of a two-point-flux operator (see include/rsc.h)."""
    g = torch.empty(face_i.numel(), dtype=torch.float64, device=lam.device)
    check(lib().rsc_grad_faces(face_i.numel(), _ptr(face_i), _ptr(face_j), _ptr(lam), _ptr(x), _ptr(g),
                               _stream()), "rsc_grad_faces")
    return g


class RSCSolve(torch.autograd.Function):
    """``x = A(values)^{-1} b`` by factor + PCG; backward by the adjoint solve that
    reuses the factor: ``dL/db = lambda = A^{-1} g`` and
    ``dL/dvalues[p] = -lambda_row(p) x_col(p)`` on A's pattern."""

    @staticmethod
    def forward(ctx, values, b, solver: RSCSolver, tol: float, rtol: float, max_iter: int):
        v = values.detach()
        solver.factor(v, tol)
        x, info = solver.pcg(b.detach(), rtol=rtol, max_iter=max_iter)
        ctx.solver, ctx.tol, ctx.rtol, ctx.max_iter = solver, tol, rtol, max_iter
        ctx.generation = solver.generation
        ctx.save_for_backward(x, v)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, g):
        x, v = ctx.saved_tensors
        solver = ctx.solver
        # The adjoint solve must use this forward's matrix: the handle's SpMV and factor
        # are those of its latest rsc_factor, so if the solver factored other values
        # since, it is refactored from the values saved here first.
        if solver.generation != ctx.generation:
            solver.factor(v, ctx.tol)
            ctx.generation = solver.generation
        lam, _ = solver.pcg(g.detach().contiguous(), rtol=ctx.rtol, max_iter=ctx.max_iter)
        gv = solver.grad_values(lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gv, gb, None, None, None, None


def solve(values, b, solver: RSCSolver, tol=0.0, rtol=1e-8, max_iter=1000):
    return RSCSolve.apply(values, b, solver, tol, rtol, max_iter)
