"""bfloat16 rounding and the BF16 tile-product models (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

bfloat16 keeps the sign, the 8-bit exponent and the top 7 stored mantissa
bits of an IEEE binary32 value.  Rounding binary32 -> bfloat16 is
round-to-nearest, ties-to-even on the 16 dropped bits (NaN and infinity are not
produced by the inputs used here).  The models below state what a K-tile
product computes when the kernel entries and the right-hand sides are rounded
to bfloat16 and the products are accumulated exactly:

    x1 :  sum_j bf(k_ij) bf(v_j)
    x2 :  sum_j [bf(k_ij) bf(v_j) + bf(k_ij) bf(v_j - bf(v_j)) + bf(k_ij - bf(k_ij)) bf(v_j)]

(hi/lo split: a = hi + lo with hi = bf(a), lo = bf(a - hi); the lo*lo term is
dropped), and with a three-way split a = h + m + l (h = bf(a), m = bf(a - h),
l = bf(a - h - m); each difference is exact in binary32, and h + m + l equals
a exactly for normal binary32 values, since each bfloat16 piece with its sign
carries 8 significant bits of the 24):

    x3 :  sum_j [hh + hm + mh + hl + lh + mm]   (products of the pieces of k and v)

The three dropped products (ml, lm, ll) are below 2^-23 of |k v|, so x3 is as
accurate as a binary32 product.  LightGP itself is float32 only (Sec. 5, "Limitations"); these forms
are the precision extension and are judged by the end-to-end residual.
"""

from __future__ import annotations

import numpy as np


def round_bf16(a) -> np.ndarray:
    """float32 -> bfloat16 (RNE) returned as float32 values."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)


def split_bf16(a):
    """hi = bf(a), lo = bf(a - hi) computed in float32."""
    a = np.asarray(a, dtype=np.float32)
    hi = round_bf16(a)
    lo = round_bf16((a - hi).astype(np.float32))
    return hi, lo


def tile_product_x1(K32: np.ndarray, V32: np.ndarray) -> np.ndarray:
    return round_bf16(K32).astype(np.float64) @ round_bf16(V32).astype(np.float64)


def tile_product_x2(K32: np.ndarray, V32: np.ndarray) -> np.ndarray:
    kh, kl = split_bf16(K32)
    vh, vl = split_bf16(V32)
    kh, kl, vh, vl = (x.astype(np.float64) for x in (kh, kl, vh, vl))
    return kh @ vh + kh @ vl + kl @ vh


def split3_bf16(a):
    """h = bf(a), m = bf(a - h), l = bf(a - h - m), differences in float32."""
    a = np.asarray(a, dtype=np.float32)
    h = round_bf16(a)
    r = (a - h).astype(np.float32)
    m = round_bf16(r)
    l = round_bf16((r - m).astype(np.float32))
    return h, m, l


def tile_product_x3(K32: np.ndarray, V32: np.ndarray) -> np.ndarray:
    kh, km, kl = (x.astype(np.float64) for x in split3_bf16(K32))
    vh, vm, vl = (x.astype(np.float64) for x in split3_bf16(V32))
    return kh @ vh + kh @ vm + km @ vh + kh @ vl + kl @ vh + km @ vm
