"""Host side of the C library (no GPU): exported symbols, the symbolic phase bit for
bit against the oracle, and argument/pattern validation."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

from conftest import ROOT, golden_path
from oracle.ordering import symbolic
from workloads import grid_coordinates, grid_problem
from workloads.grids import batched_problems

from paper_1507_05593_amd import RSCSolver, lib
from paper_1507_05593_amd._lib import RSC_ERR_INVALID_ARG, RSC_ERR_PATTERN, Options, RSCError


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "rsc.h")).read()
    names = set(re.findall(r"\b(rsc_[a-z_]+)\s*\(", hdr))
    names -= {"rsc_handle"}
    assert len(names) >= 20
    L = lib()
    for n in sorted(names):
        assert hasattr(L, n), n


def _compare(sol: RSCSolver, sym, n):
    assert np.array_equal(sol.perm, sym.perm)
    first, parent, level, kind = sol.supernode_info()
    assert np.array_equal(first, sym.first)
    assert np.array_equal(parent, sym.parent)
    assert np.array_equal(level, sym.level)
    assert np.array_equal(kind, sym.kind)
    rp, rows = sol.rowsets()
    for j in range(sym.M):
        assert np.array_equal(rows[rp[j]:rp[j + 1]], sym.rows[j])


@pytest.mark.parametrize("dims,sigma,leaf", [((64, 64), 0.0, 64), ((31, 17), 1.0, 16), ((12, 12, 12), 1.0, 64),
                                             ((16, 16, 16), 1.0, 64), ((9, 10, 11), 1.5, 8),
                                             ((24, 24, 24), 1.0, 64)])
def test_symbolic_bit_exact_with_oracle(dims, sigma, leaf):
    p = grid_problem(dims, sigma=sigma, seed=2, unit=(sigma == 0))
    sym = symbolic(p.n, p.rowptr, p.colind, leaf)
    sol = RSCSolver(p.n, p.rowptr, p.colind, leaf_max=leaf)
    _compare(sol, sym, p.n)


@pytest.mark.parametrize("dims,tau,scramble", [((12, 12, 12), 16, False), ((40, 40), 8, False),
                                               ((20, 18, 16), 24, False), ((24, 24, 24), 40, False),
                                               ((14, 14, 14), 20, True)])
def test_coordinate_order_bit_exact_with_oracle(dims, tau, scramble):
    """The block trees' column order inside large separators (§4.1) and their depths;
    scrambled positions exercise the stable sort's ties and the longest-side choice."""
    p = grid_problem(dims, sigma=1.0, seed=2)
    xyz = grid_coordinates(dims)
    if scramble:
        rng = np.random.default_rng(7)
        xyz = xyz[:, rng.permutation(3)] * rng.choice([1.0, 2.0], size=3) + rng.integers(0, 3, size=(p.n, 3))
    sym = symbolic(p.n, p.rowptr, p.colind, 64, tau, xyz)
    sol = RSCSolver(p.n, p.rowptr, p.colind, coords=xyz, tau_D=tau)
    _compare(sol, sym, p.n)
    assert np.array_equal(sol.tree_depths, sym.depth)
    assert sym.depth.max() >= 1
    # without positions the columns keep the dissection order; the depths are the same
    sym0 = symbolic(p.n, p.rowptr, p.colind, 64, tau)
    sol0 = RSCSolver(p.n, p.rowptr, p.colind, tau_D=tau)
    _compare(sol0, sym0, p.n)
    assert np.array_equal(sol0.tree_depths, sym.depth)


def test_batched_symbolic_is_per_system_dissection():
    probs = batched_problems(5, 8, 40, 1.0, seed=4)
    sol = RSCSolver.batch([q.n for q in probs], [q.rowptr for q in probs], [q.colind for q in probs])
    assert sol.systems == 5
    perm = sol.perm
    first, parent, level, kind = sol.supernode_info()
    off = 0
    sn = 0
    for q in probs:
        sym = symbolic(q.n, q.rowptr, q.colind, 64)
        assert np.array_equal(perm[off:off + q.n], sym.perm + off)
        assert np.array_equal(first[sn:sn + sym.M + 1], sym.first + off)
        assert np.array_equal(level[sn:sn + sym.M], sym.level)
        off += q.n
        sn += sym.M
    assert sn == sol.supernodes


def test_path_graph_structure_hand_worked():
    # the library's dissection, row sets, parents and levels of the path graph 0-...-199
    # against the structure worked by hand in the fixture (same as the oracle's test)
    g = json.load(open(golden_path("nd_path200.json")))
    n = g["n"]
    rows_ = []
    for i in range(n):
        rows_.append([v for v in (i - 1, i, i + 1) if 0 <= v < n])
    rp = np.cumsum([0] + [len(r) for r in rows_]).astype(np.int64)
    ci = np.concatenate(rows_).astype(np.int32)
    sol = RSCSolver(n, rp, ci, leaf_max=g["leaf_max"])
    first, parent, level, kind = sol.supernode_info()
    perm = sol.perm
    got = [[int(perm[first[j]]), int(perm[first[j + 1] - 1]), "leaf" if kind[j] == 0 else "separator"]
           for j in range(sol.supernodes)]
    assert got == g["supernodes"]
    rptr, rows = sol.rowsets()
    assert [rows[rptr[j]:rptr[j + 1]].tolist() for j in range(sol.supernodes)] == g["rows"]
    assert parent.tolist() == g["parent"]
    assert level.tolist() == g["level"]


def test_pattern_and_argument_errors():
    p = grid_problem((5, 5), unit=True)
    bad = p.colind.copy()
    bad[1], bad[2] = bad[2], bad[1]            # unsorted row
    with pytest.raises(RSCError) as e:
        RSCSolver(p.n, p.rowptr, bad)
    assert e.value.code == RSC_ERR_PATTERN
    # asymmetric pattern: drop one off-diagonal entry of row 0 (and shift the row pointer)
    rp = p.rowptr.copy(); ci = p.colind.copy()
    ci2 = np.delete(ci, 1); rp2 = rp.copy(); rp2[1:] -= 1
    with pytest.raises(RSCError) as e:
        RSCSolver(p.n, rp2, ci2)
    assert e.value.code == RSC_ERR_PATTERN
    for bad_opt in (dict(leaf_max=0), dict(sweep_small_c=-1), dict(sweep_small_c=1025), dict(gemm_tile=32),
                    dict(tau_D=-1), dict(tau_D=1), dict(alpha_D=0.0)):
        with pytest.raises(RSCError) as e:
            RSCSolver(p.n, p.rowptr, p.colind, **bad_opt)
        assert e.value.code == RSC_ERR_INVALID_ARG, bad_opt
    h = C.c_void_p()
    assert lib().rsc_analyze(-1, None, None, None, C.byref(h)) == RSC_ERR_INVALID_ARG
    # positions: null, wrong shape, non-finite
    assert lib().rsc_analyze_coords(p.n, p.rowptr.ctypes.data, p.colind.ctypes.data, None, None,
                                    C.byref(h)) == RSC_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        RSCSolver(p.n, p.rowptr, p.colind, coords=np.zeros((p.n, 2)))
    xyz = grid_coordinates((5, 5))
    xyz[3, 1] = np.nan
    with pytest.raises(RSCError) as e:
        RSCSolver(p.n, p.rowptr, p.colind, coords=xyz, tau_D=4)
    assert e.value.code == RSC_ERR_INVALID_ARG


def test_stats_before_factor():
    p = grid_problem((20, 20), unit=True)
    sol = RSCSolver(p.n, p.rowptr, p.colind)
    s = sol.stats()
    assert s["n"] == p.n and s["nnz"] == p.nnz and s["supernodes"] == sol.supernodes
    assert s["flops_potrf"] == 0.0 and s["t_analyze_ms"] > 0
    o = Options()
    lib().rsc_default_options(C.byref(o))
    assert (o.leaf_max, o.tau_O, o.oversample, o.power_iters, o.alpha_O) == (64, 32, 10, 0, 1.0)


def test_set_allocator_arguments_and_state():
    """rsc_set_allocator: both callbacks or neither; no change while a handle exists
    (analysis needs no device, so a handle can be made here)."""
    import gc

    from paper_1507_05593_amd import _lib
    from paper_1507_05593_amd._lib import RSC_ERR_STATE, RSC_OK
    L = lib()
    assert L.rsc_set_allocator(None, None, None) == RSC_OK          # already the default
    alloc_cb = _lib.ALLOC_FN(lambda n, s, c: None)
    release_cb = _lib.RELEASE_FN(lambda p, s, c: None)
    alloc, release = _lib.fnptr(alloc_cb), _lib.fnptr(release_cb)
    assert L.rsc_set_allocator(alloc, None, None) == RSC_ERR_INVALID_ARG
    assert L.rsc_set_allocator(None, release, None) == RSC_ERR_INVALID_ARG
    p = grid_problem((6, 6), sigma=0.0, seed=1)
    sol = RSCSolver(p.n, p.rowptr, p.colind)
    assert L.rsc_set_allocator(alloc, release, None) == RSC_ERR_STATE
    assert L.rsc_set_allocator(None, None, None) == RSC_OK          # no change: allowed
    del sol
    gc.collect()
