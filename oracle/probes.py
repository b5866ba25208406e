"""Counter-based Rademacher probes from SplitMix64 (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

LightGP Sec. 4.3 uses independent Rademacher probes (+-1, probability 1/2
each) for its Hutchinson estimator.  For a seeded run both sides draw the
same probes from one published counter-based generator, implemented
independently on each side: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  With the golden gamma
G = 0x9E3779B97F4A7C15, the k-th output (k = 1, 2, ...) of the stream seeded
with s is mix(s + k G) where

    mix(z):  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
             z = (z ^ (z >> 27)) * 0x94D049BB133111EB
             return z ^ (z >> 31)          (all arithmetic mod 2^64)

Entry (j, c) of an n x p probe matrix uses counter k = c n + j + 1, and takes
the sign from the top bit of the output: bit 63 clear gives +1, set gives -1.
"""

from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def stream(seed: int, count: int) -> list:
    """The first ``count`` outputs of SplitMix64 seeded with ``seed``."""
    out, s = [], seed & _M64
    for _ in range(count):
        s = (s + GAMMA) & _M64
        out.append(mix64(s))
    return out


def rademacher(seed: int, n: int, p: int) -> np.ndarray:
    """n x p matrix of +-1 (float64): entry (j, c) from counter c n + j + 1."""
    k = np.arange(1, n * p + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + k * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    sign = np.where((z >> np.uint64(63)) == 0, 1.0, -1.0)
    return sign.reshape(p, n).T.copy()
