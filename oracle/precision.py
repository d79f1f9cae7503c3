"""Storage precisions of the block inverses and their exact rounding.

Test infrastructure only (see the package docstring).

The paper uses one low format (fp32) for the whole preconditioner (Sec. 4.2);
reduced 16-bit formats with a per-block scale follow Anzt et al.'s adaptive
block-Jacobi storage (cited in Sec. 2). Readings fixed here:
  * every conversion is round-to-nearest, ties-to-even, directly from the FP64
    value (no double rounding), with gradual underflow (subnormals kept) and
    overflow to infinity;
  * FP16 and BF16 blocks carry a power-of-two scale s chosen so that the
    largest |entry|/s lies in (2^14, 2^15]; FP32 and FP64 blocks use s = 1.
    A power-of-two scale is exact, so it adds no rounding of its own.
"""
from __future__ import annotations

import numpy as np

FP64, FP32, BF16, FP16 = 0, 1, 2, 3
NAMES = {FP64: "fp64", FP32: "fp32", BF16: "bf16", FP16: "fp16"}
BYTES = {FP64: 8, FP32: 4, BF16: 2, FP16: 2}
# (significand bits incl. the hidden bit, minimum normal exponent, largest finite)
_FORMAT = {
    FP32: (24, -126, float(np.finfo(np.float32).max)),
    BF16: (8, -126, float.fromhex("0x1.fep127")),
    FP16: (11, -14, 65504.0),
}
SCALE_TOP_EXP = 15   # 16-bit blocks are scaled so that max|H|/s is in (2^14, 2^15]


def round_to_format(x, prec: int) -> np.ndarray:
    """Round float64 values to the nearest value of a binary floating-point
    format (ties to even, gradual underflow, overflow to +-inf), returned as
    float64. The quantum of x is 2^(max(e, emin) - (p-1)) where 2^e <= |x| <
    2^(e+1); dividing by a power of two and ``np.rint`` (ties-to-even) are
    exact, so the result is the correctly rounded value."""
    x = np.asarray(x, dtype=np.float64)
    if prec == FP64:
        return x.copy()
    p, emin, fmax = _FORMAT[prec]
    out = np.zeros_like(x)
    nz = (x != 0) & np.isfinite(x)
    m, e = np.frexp(x[nz])            # x = m 2^e, 0.5 <= |m| < 1  -> leading bit 2^(e-1)
    lead = e.astype(np.int64) - 1
    qexp = np.maximum(lead, emin) - (p - 1)
    y = np.ldexp(np.rint(np.ldexp(x[nz], -qexp)), qexp)
    y = np.where(np.abs(y) > fmax, np.copysign(np.inf, y), y)
    out[nz] = y
    out[~nz] = x[~nz]                 # zeros (with sign), inf, nan pass through
    return out


def ceil_log2(v: float) -> int:
    """Smallest integer c with v <= 2^c, for v > 0 (exact, via frexp)."""
    m, e = np.frexp(float(v))
    return int(e) - 1 if m == 0.5 else int(e)


def block_scale(maxabs: float, prec: int) -> float:
    """Per-block power-of-two scale s: max|H|/s in (2^14, 2^15] for 16-bit
    formats, s = 1 otherwise."""
    if prec in (FP16, BF16):
        return float(np.ldexp(1.0, ceil_log2(maxabs) - SCALE_TOP_EXP))
    return 1.0


def store_block(H: np.ndarray, prec: int):
    """Emulated storage of one FP64 block inverse: returns (Hhat, s) with the
    stored values Hhat (as float64) so that the represented matrix is s*Hhat."""
    if prec == FP64:
        return np.array(H, dtype=np.float64), 1.0
    s = block_scale(float(np.max(np.abs(H))), prec)
    return round_to_format(np.asarray(H) / s, prec), s


def rhat(r: np.ndarray) -> np.ndarray:
    """FP32 copy of the working-precision residual fed to a reduced-precision
    block (the first ConvertPrecision step of Algorithm 3.1)."""
    return round_to_format(r, FP32)
