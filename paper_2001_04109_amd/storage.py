"""Host-side conversion of residues into the caller-side operand storages
accepted by fsyrk_modp (FFP_I8_CENTERED and FFP_I8_LIMB2).

These produce the representations the C ABI documents for its int8 inputs;
the library itself packs FFP_U32 operands on the device.
"""
from __future__ import annotations

import numpy as np


def centred_i8(A: np.ndarray, p: int) -> np.ndarray:
    """Residues in [0, p) (p <= 251) as centred int8 in [-(p-1)/2, (p-1)/2]."""
    return np.where(A > (p - 1) // 2, A.astype(np.int64) - p, A).astype(np.int8)


def limbs(A: np.ndarray, p: int) -> np.ndarray:
    """Residues in [0, p) (p <= 65521) as the two int8 planes (hi, lo) of a
    representative 256*hi + lo in [-32896, 32639]."""
    x = np.where(A <= 32639, A.astype(np.int64), A.astype(np.int64) - p)
    lo = ((x + 128) & 255) - 128
    hi = (x - lo) >> 8
    return np.stack([hi.astype(np.int8), lo.astype(np.int8)])
