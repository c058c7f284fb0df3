"""Rounding of the centered matrix to the library's storage precisions,
written from the formats' definitions (FP32: IEEE single, round to nearest
even; BF16: the upper 16 bits of the FP32 value after round to nearest
even), so that the oracle can run on the exact problem a stored matrix
defines."""

import numpy as np


def round_storage(A, precision):
    if precision == "fp64":
        return np.array(A, dtype=np.float64)
    f32 = np.asarray(A, dtype=np.float64).astype(np.float32)
    if precision == "fp32":
        return f32.astype(np.float64)
    if precision != "bf16":
        raise ValueError(precision)
    bits = f32.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)
