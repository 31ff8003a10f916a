"""Philox4x32-10 and the library's built-in draws of D and Omega (oracle side).

Test infrastructure only.  The solver accepts D and Omega from the caller; when
they are not given it draws them from a counter-based generator, Philox4x32-10
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11), with the counter/key layout and the conversion to doubles stated in the
library's C header.  This module implements the same generator from its
published definition (ten rounds of the 4x32 Philox round: two 32 x 32 -> 64
multiplications with the constants 0xD2511F53 and 0xCD9E8D57, the key bumped
by the Weyl constants 0x9E3779B9 and 0xBB67AE85), so that a run with
built-in draws can be compared with the oracle.  It is pinned by the
generator's published known-answer vectors.
"""
from __future__ import annotations

import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_LO = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox4x32 rounds on counter arrays (uint32 values) with key (k0, k1)."""
    c = [np.asarray(x, dtype=np.uint64) & _LO for x in (c0, c1, c2, c3)]
    k0, k1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [((p1 >> _S32) ^ c[1] ^ np.uint64(k0)) & _LO, p1 & _LO,
             ((p0 >> _S32) ^ c[3] ^ np.uint64(k1)) & _LO, p0 & _LO]
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return c


def u53(a, b) -> np.ndarray:
    """A double in [0, 1) from 53 bits: 27 of a and 26 of b (exact in FP64)."""
    hi = (np.asarray(a, dtype=np.uint64) >> np.uint64(5)).astype(np.float64)
    lo = (np.asarray(b, dtype=np.uint64) >> np.uint64(6)).astype(np.float64)
    return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0)


def _words(n: int, stream: int, seed: int):
    i = np.arange(n, dtype=np.uint64)
    z = np.zeros(n, dtype=np.uint64)
    return philox4x32_10(i, z + np.uint64(stream), z, z, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def perturbation_diagonal(n: int, seed: int) -> np.ndarray:
    """D_i = u53(x0, x1) of counter (i, 0, 0, 0)."""
    x = _words(n, 0, seed)
    return u53(x[0], x[1])


def start_block(n: int, d: int, seed: int) -> np.ndarray:
    """Omega (n x d, column-major): Box-Muller on counter (i, j + 1, 0, 0) for column j."""
    om = np.empty((n, d), order="F")
    for j in range(d):
        x = _words(n, j + 1, seed)
        u1 = 1.0 - u53(x[0], x[1])
        u2 = u53(x[2], x[3])
        om[:, j] = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return om
