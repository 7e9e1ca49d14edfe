"""Philox-4x32-10 counter-based generator and Box-Muller normals.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Philox-4x32 as defined by Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC 2011): a 128-bit counter (4 x 32-bit words)
and a 64-bit key (2 x 32-bit words); each round multiplies words 0 and 2 by
fixed odd constants, keeping the high and low halves of the 64-bit products,
and mixes the high halves with words 1 and 3 and the round key; the key is
bumped by two Weyl constants between rounds; 10 rounds.  The multipliers and
Weyl constants are the published ones.  Pinned by the authors' known-answer
vectors in the test suite.

Box-Muller: with u = (x + 0.5) / 2^32 in (0, 1) for a 32-bit word x,
    n0 = sqrt(-2 ln u0) cos(2 pi u1),  n1 = sqrt(-2 ln u0) sin(2 pi u1).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_SH = np.uint64(32)


def philox4x32(ctr, key, rounds: int = 10):
    """Vectorised Philox-4x32-R.  ctr: 4 arrays (or ints), key: 2 arrays (or ints).

    Returns four uint32 arrays.
    """
    c = [np.asarray(x, dtype=np.uint64) & _MASK for x in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & _MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & _MASK
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> _SH, p0 & _MASK
        hi1, lo1 = p1 >> _SH, p1 & _MASK
        c = [(hi1 ^ c[1] ^ k0) & _MASK, lo1, (hi0 ^ c[3] ^ k1) & _MASK, lo0]
    return [x.astype(np.uint32) for x in c]


def u01(x) -> np.ndarray:
    """32-bit word -> uniform in (0, 1): (x + 1/2) / 2^32, exact in FP64."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)


def box_muller(x0, x1):
    """Two 32-bit words -> two independent N(0,1) values."""
    u0 = u01(x0)
    u1 = u01(x1)
    r = np.sqrt(-2.0 * np.log(u0))
    t = 2.0 * np.pi * u1
    return r * np.cos(t), r * np.sin(t)


def split_seed(seed: int):
    """64-bit seed -> Philox key words (low, high)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


# Streams used by conditional simulation (word 2 of the counter selects the stream).
STREAM_CE = 0      # complex white noise of the circulant-embedding sampler
STREAM_NUGGET = 1  # N(0, tau^2) measurement noise at the observation sites


def ce_noise(seed: int, pair: int, F1: int, F2: int):
    """Complex white noise xi1 + i xi2 on the F1 x F2 embedding for one realisation pair.

    Bin e = k1*F2 + k2 uses counter (e, pair, STREAM_CE, 0); its words 0 and 1
    give (xi1, xi2) by Box-Muller.
    """
    e = np.arange(F1 * F2, dtype=np.uint64)
    k0, k1 = split_seed(seed)
    w = philox4x32((e, np.uint64(pair), np.uint64(STREAM_CE), np.uint64(0)), (k0, k1))
    a, b = box_muller(w[0], w[1])
    return (a + 1j * b).reshape(F1, F2)


def nugget_noise(seed: int, real: int, n: int) -> np.ndarray:
    """N(0,1) values for realisation `real` at the n sites: counter (i, real, STREAM_NUGGET, 0)."""
    i = np.arange(n, dtype=np.uint64)
    k0, k1 = split_seed(seed)
    w = philox4x32((i, np.uint64(real), np.uint64(STREAM_NUGGET), np.uint64(0)), (k0, k1))
    a, _ = box_muller(w[0], w[1])
    return a
