"""Rounding of float32 values to bfloat16 / float16 (round to nearest, ties to even).

Diagnostic only: lets a test form the low-precision normal matrix the way a
BF16/FP16 matrix-core kernel sees its inputs, to tell rounding apart from
kernel mistakes.  Test infrastructure only (see the package header).
"""
import numpy as np


def round_bf16(x):
    """float -> nearest bfloat16 value (returned as float64); NaN/Inf pass through."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    rounded = ((b + 0x7FFF + lsb) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    return np.where(np.isfinite(f), out, f).astype(np.float64)


def round_fp16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)
