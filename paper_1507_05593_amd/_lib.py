"""ctypes declarations of the C ABI in include/rsc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsc.so")

RSC_OK = 0
RSC_ERR_INVALID_ARG = 1
RSC_ERR_PATTERN = 2
RSC_ERR_NOT_SPD = 3
RSC_ERR_NOT_CONVERGED = 4
RSC_ERR_BREAKDOWN = 5
RSC_ERR_OUT_OF_MEMORY = 6
RSC_ERR_DEVICE = 7
RSC_ERR_STATE = 8

RSC_FP64 = 0
RSC_MIXED_BF16 = 1
RSC_MIXED_FP32 = 2

K_CLASSES = ["update", "panel_potrf", "panel_trsm", "panel_trailing", "truncation", "pcg", "other", "lo_product",
             "sample", "orthonormalise", "basis"]
RSC_KERNELS = 42


class Options(C.Structure):
    _fields_ = [("leaf_max", C.c_int32), ("tau_O", C.c_int32), ("oversample", C.c_int32),
                ("power_iters", C.c_int32), ("alpha_O", C.c_double), ("seed", C.c_uint64),
                ("precision", C.c_int32), ("use_graph", C.c_int32), ("retry", C.c_int32),
                ("gemm_tile", C.c_int32), ("keep_lo", C.c_int32),
                ("sweep_small_c", C.c_int32), ("tau_D", C.c_int32), ("reserved0", C.c_int32),
                ("alpha_D", C.c_double), ("interior", C.c_int32), ("reserved2", C.c_int32)]


class PcgResult(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("rel_residual", C.c_double),
                ("true_residual", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("supernodes", C.c_int64), ("levels", C.c_int64),
                ("systems", C.c_int64), ("factor_entries", C.c_int64), ("compressed", C.c_int64),
                ("rank_sum", C.c_int64), ("sample_sum", C.c_int64), ("rank_saturated", C.c_int64),
                ("failed_supernode", C.c_int32), ("precision_used", C.c_int32), ("retries", C.c_int32),
                ("reserved", C.c_int32), ("flops_potrf", C.c_double), ("flops_trsm", C.c_double),
                ("flops_update", C.c_double), ("flops_sample", C.c_double), ("flops_orth", C.c_double),
                ("flops_trunc", C.c_double), ("bytes_factor", C.c_double), ("t_analyze_ms", C.c_double),
                ("t_factor_ms", C.c_double), ("t_pcg_ms", C.c_double), ("device_bytes", C.c_double),
                ("gemm_tuned", C.c_int64), ("gemm_tile128", C.c_int64), ("tree_supernodes", C.c_int64),
                ("tree_blocks", C.c_int64), ("tree_rank_sum", C.c_int64), ("tree_entries", C.c_int64),
                ("alpha_D_used", C.c_double), ("diag_restarts", C.c_int32), ("reserved1", C.c_int32),
                ("interior_blocks", C.c_int64), ("interior_dropped", C.c_int64)]


ARITHS = ("f64", "f32", "bf16")


class Profile(C.Structure):
    _fields_ = [("launches", C.c_int64 * len(K_CLASSES)), ("ms", C.c_double * len(K_CLASSES)),
                ("flops", C.c_double * len(K_CLASSES)), ("tile_flops", C.c_double * len(K_CLASSES)),
                ("flops_arith", (C.c_double * len(ARITHS)) * len(K_CLASSES))]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def fnptr(f):
    """A ctypes callback as the plain pointer rsc_set_allocator takes (None: NULL)."""
    return None if f is None else C.cast(f, C.c_void_p)

_lib = None

SYMBOLS = {
    "rsc_default_options": (None, [C.POINTER(Options)]),
    "rsc_analyze": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "rsc_get_tree_depths": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rsc_analyze_coords": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Options),
                                     C.POINTER(C.c_void_p)]),
    "rsc_analyze_batch": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Options),
                                    C.POINTER(C.c_void_p)]),
    "rsc_factor": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "rsc_pcg": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p,
                          C.POINTER(PcgResult)]),
    "rsc_apply_preconditioner": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rsc_apply_preconditioner_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rsc_grad_values": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rsc_spectral_coordinates": (C.c_int, [C.c_void_p, C.c_int32, C.c_uint64, C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "rsc_grad_faces": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "rsc_get_sizes": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_int64)] * 5),
    "rsc_get_permutation": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rsc_get_supernodes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rsc_get_rowsets": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "rsc_get_ranks": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "rsc_get_block": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rsc_get_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "rsc_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "rsc_get_profile": (C.c_int, [C.c_void_p, C.POINTER(Profile)]),
    "rsc_get_kernel_profile": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_char_p), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "rsc_set_allocator": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),   # ALLOC_FN, RELEASE_FN or NULL
    "rsc_status_string": (C.c_char_p, [C.c_int]),
    "rsc_last_error": (C.c_char_p, []),
    "rsc_destroy": (None, [C.c_void_p]),
}


def lib():
    """The loaded C library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1507_05593_amd.build` (there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class RSCError(RuntimeError):
    def __init__(self, code, where=""):
        L = lib()
        self.code = code
        msg = L.rsc_status_string(code).decode()
        detail = L.rsc_last_error().decode()
        super().__init__(f"{where}: {msg}: {detail}" if where else f"{msg}: {detail}")


def check(code, where=""):
    if code != RSC_OK:
        raise RSCError(code, where)
