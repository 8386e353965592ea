"""Rounding to 16-bit floating-point formats, written from the IEEE-754 /
bfloat16 definitions (round to nearest, ties to even).  TEST INFRASTRUCTURE:
used to hand the oracle the same BF16-valued weights the GPU path uses."""
from __future__ import annotations

import numpy as np


def round_bf16(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32.
    bfloat16 keeps the upper 16 bits of the float32 pattern; rounding adds
    0x7FFF plus the lowest kept bit before truncating.  NaN/inf pass through."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).copy()
    bad = ~np.isfinite(a)
    out[bad] = a[bad]
    return out


def split_bf16(x):
    """(hi, lo) with hi = bf16(x), lo = bf16(x - hi)."""
    x = np.asarray(x, dtype=np.float32)
    hi = round_bf16(x)
    lo = round_bf16(x - hi)
    return hi, lo
