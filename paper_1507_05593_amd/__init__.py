"""Rank-structured supernodal Cholesky preconditioned CG on MI355X (gfx950).

Symbolic analysis on the host, numeric factorization and PCG in hand-written HIP
kernels, exposed through the C ABI of include/rsc.h; this package is the thin
Python binding (ctypes) plus a torch.autograd.Function for the solve adjoint.
"""
from ._lib import RSCError, lib  # noqa: F401
from .solver import RSCSolve, RSCSolver, grad_faces, make_options, solve, use_torch_allocator  # noqa: F401
