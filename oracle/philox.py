"""Oracle: counter-based Gaussian generator for the range finder (test infrastructure).

The paper draws the sampling matrix from a Gaussian distribution with mean 0
and unit variance (Algorithm 3, ``randomMatrix``) and names no generator.  Both
this oracle and the device library implement, each on its own, the published
Philox4x32-10 generator (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC 2011): a 10-round bijection of a 128-bit counter under a
64-bit key, each round two 32x32->64-bit multiplies by fixed odd multipliers and
a Weyl-sequence key schedule.  Gaussians come from the Box-Muller transform.

Stream layout (shared definition, no shared code): the sample for supernode
``j`` under seed ``s`` is keyed ``(s mod 2^32, j XOR (s >> 32))``; entry
``(row, col)`` of the ``r_j x l_j`` matrix comes from the counter
``(row, col // 4, 0, 0)``: its four output words ``w0..w3`` give two Box-Muller
pairs, ``u1 = (w + 1) 2^-32`` in ``(0, 1]`` and ``u2 = w' 2^-32`` in ``[0, 1)``,
``g = sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2)``; column ``4t + i`` takes the
``i``-th of ``(g0 from w0/w1 cos, g1 from w0/w1 sin, g2 from w2/w3 cos, g3 from
w2/w3 sin)``.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint32 arrays; returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32); c1 = np.asarray(c1, dtype=np.uint32)
    c2 = np.asarray(c2, dtype=np.uint32); c3 = np.asarray(c3, dtype=np.uint32)
    k0 = np.asarray(k0, dtype=np.uint32).copy(); k1 = np.asarray(k1, dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd:
                k0 = k0 + W0
                k1 = k1 + W1
            p0 = M0 * c0.astype(np.uint64)
            p1 = M1 * c2.astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32); lo0 = (p0 & MASK).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32); lo1 = (p1 & MASK).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def gaussian_sample(seed: int, j: int, rows: int, cols: int, c2: int = 0) -> np.ndarray:
    """The ``rows x cols`` FP64 Gaussian sample of supernode ``j`` (third counter word
    ``c2``: 0 for the range finder's sample, 2 for the spectral start block)."""
    seed = int(seed)
    k0 = np.uint32(seed & 0xFFFFFFFF)
    k1 = np.uint32(((seed >> 32) & 0xFFFFFFFF) ^ (j & 0xFFFFFFFF))
    ngrp = (cols + 3) // 4
    r = np.repeat(np.arange(rows, dtype=np.uint32), ngrp)
    t = np.tile(np.arange(ngrp, dtype=np.uint32), rows)
    z = np.zeros_like(r)
    w0, w1, w2, w3 = philox4x32_10(r, t, np.full_like(r, c2), z, np.full_like(r, k0), np.full_like(r, k1))
    two32 = 2.0 ** -32
    out = np.empty((rows, ngrp, 4))
    for a, b, i in ((w0, w1, 0), (w2, w3, 2)):
        u1 = (a.astype(np.float64) + 1.0) * two32
        u2 = b.astype(np.float64) * two32
        rad = np.sqrt(-2.0 * np.log(u1))
        th = 2.0 * np.pi * u2
        out[:, :, i] = (rad * np.cos(th)).reshape(rows, ngrp)
        out[:, :, i + 1] = (rad * np.sin(th)).reshape(rows, ngrp)
    return out.reshape(rows, ngrp * 4)[:, :cols].copy()
