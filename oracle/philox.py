"""Philox4x32-10 counter-based generator and Box-Muller Gaussians.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Written from the published definition (J. K. Salmon, M. A. Moraes,
R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11): a 4x32-bit counter and a 2x32-bit key, ten rounds of two 32x32->64
multiplications whose high halves are xor-ed with the other counter words
and the key, the key advancing by a Weyl sequence between rounds.  The ARA
step draws its Gaussian test matrices ("randn" in Algorithm "Adaptive
Randomized Approximation") from this stream; the oracle itself never needs
them, they exist here only to check the device generator bit for bit.

Stream layout used by the library: element e of the m x bs test matrix of
(seed, column k, iteration t, stream s) takes Gaussian number e % 2 of
counter (e // 2, t, k, s) under key (seed & 0xffffffff, seed >> 32).
"""
from __future__ import annotations

import math
from typing import Tuple

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def _mulhilo(a: int, b: int) -> Tuple[int, int]:
    p = (a * b) & 0xFFFFFFFFFFFFFFFF
    return p >> 32, p & MASK


def philox4x32_10(ctr: Tuple[int, int, int, int], key: Tuple[int, int]) -> Tuple[int, int, int, int]:
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        hi0, lo0 = _mulhilo(M0, c0)
        hi1, lo1 = _mulhilo(M1, c2)
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def uniform53(hi: int, lo: int) -> float:
    """[0, 1) double with 53 random bits from two 32-bit words."""
    return ((hi >> 5) * 67108864 + (lo >> 6)) * (1.0 / 9007199254740992.0)


def gaussian_pair(words: Tuple[int, int, int, int]) -> Tuple[float, float]:
    """Box-Muller: radius from u1 in (0, 1], angle from u2 in [0, 1)."""
    u1 = 1.0 - uniform53(words[0], words[1])
    u2 = uniform53(words[2], words[3])
    rad = math.sqrt(-2.0 * math.log(u1))
    ang = 2.0 * math.pi * u2
    return rad * math.cos(ang), rad * math.sin(ang)


def test_matrix(seed: int, k: int, t: int, s: int, rows: int, cols: int):
    """The column-major rows x cols Gaussian matrix of the stream above."""
    import numpy as np
    n = rows * cols
    out = np.empty(n)
    key = (seed & MASK, (seed >> 32) & MASK)
    for c in range((n + 1) // 2):
        z = gaussian_pair(philox4x32_10((c, t & MASK, k & MASK, s & MASK), key))
        out[2 * c] = z[0]
        if 2 * c + 1 < n:
            out[2 * c + 1] = z[1]
    return out.reshape(cols, rows).T
