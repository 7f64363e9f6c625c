"""Storage formats of the reduced vectors, as exact value-level converters.

The paper stores reduced vectors with scalar quantization but leaves the format
open (Section 2.1).  The formats used here are public definitions:

* FP16  -- IEEE 754 binary16: 1 sign, 5 exponent (bias 15), 10 fraction bits,
           subnormals, max finite 65504.
* BF16  -- 1 sign, 8 exponent (bias 127), 7 fraction bits, max finite
           (2 - 2^-7) * 2^127.
* FP8   -- OCP 8-bit E4M3 ("e4m3fn"): 1 sign, 4 exponent (bias 7), 3 fraction
           bits, subnormals, no infinities, S.1111.111 is NaN, max finite 448.

Rounding is round-to-nearest, ties-to-even, and saturating: magnitudes above
the largest finite value become that value.  Everything is done on float64
values, whose exact scaling by powers of two makes the rounding exact:
``rint(x / quantum) * quantum`` with ``numpy.rint`` (ties to even).

This is oracle code (test infrastructure); it shares nothing with the HIP path.
"""
from __future__ import annotations

import numpy as np

# name -> (exponent bits, fraction bits, bias, max finite)
SPECS = {
    "fp16": (5, 10, 15, 65504.0),
    "bf16": (8, 7, 127, (2.0 - 2.0 ** -7) * 2.0 ** 127),
    "fp8": (4, 3, 7, 448.0),
}

# scale targets: the per-cluster / per-(query, cluster) power-of-two scale maps
# the block's largest magnitude into (T/2, T]
SCALE_TARGET = {"fp32": None, "fp16": 65504.0, "bf16": 1.0, "fp8": 448.0}


def round_to(fmt: str, x) -> np.ndarray:
    """Round float64 values to the nearest value of ``fmt`` (RNE, saturating)."""
    x = np.asarray(x, dtype=np.float64)
    if fmt == "fp32":
        return x.astype(np.float32).astype(np.float64)
    E, M, bias, vmax = SPECS[fmt]
    emin = 1 - bias                      # exponent of the smallest normal
    ax = np.abs(x)
    with np.errstate(divide="ignore"):
        _, ex = np.frexp(ax)             # ax = f * 2^ex, f in [0.5, 1)
    e = np.maximum(ex - 1, emin)         # unbiased exponent of the binade (subnormals share emin)
    quantum = np.ldexp(1.0, e - M)
    y = np.rint(ax / quantum) * quantum
    y = np.minimum(y, vmax)
    return np.where(np.signbit(x), -y, y)


def decode(fmt: str, codes) -> np.ndarray:
    """Value of each bit pattern (uint16 for fp16/bf16, uint8 for fp8); NaN codes give NaN."""
    E, M, bias, _ = SPECS[fmt]
    c = np.asarray(codes).astype(np.int64)
    sign = (c >> (E + M)) & 1
    ef = (c >> M) & ((1 << E) - 1)
    mf = c & ((1 << M) - 1)
    normal = ef > 0
    mag = np.where(normal,
                   np.ldexp(1.0 + mf / float(1 << M), ef - bias),
                   np.ldexp(mf / float(1 << M), 1 - bias))
    emax_field = (1 << E) - 1
    if fmt == "fp8":
        nan = (ef == emax_field) & (mf == (1 << M) - 1)
        inf = np.zeros_like(nan)
    else:
        nan = (ef == emax_field) & (mf != 0)
        inf = (ef == emax_field) & (mf == 0)
    mag = np.where(inf, np.inf, mag)
    mag = np.where(nan, np.nan, mag)
    return np.where(sign == 1, -mag, mag)


def pow2_scale(fmt: str, amax) -> np.ndarray:
    """Power-of-two scale s with amax / s in (T/2, T]; 1 where amax == 0 or fmt is fp32."""
    amax = np.asarray(amax, dtype=np.float64)
    T = SCALE_TARGET[fmt]
    if T is None:
        return np.ones_like(amax)
    with np.errstate(divide="ignore"):
        f, ex = np.frexp(amax / T)       # amax/T = f * 2^ex, f in [0.5, 1)
    # smallest e with amax/T <= 2^e: e = ex, except when amax/T is exactly 2^(ex-1)
    e = np.where(f == 0.5, ex - 1, ex)
    s = np.ldexp(1.0, e)
    return np.where(amax > 0, s, 1.0)
