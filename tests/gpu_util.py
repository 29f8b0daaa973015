"""Helpers shared by the GPU tests: device upload and the C-ABI calls with
torch tensors (marshalling only)."""
import ctypes

import numpy as np

from paper_2001_04109_amd import ffp


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev_u32(A: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(A).view(np.int32)).to(dev())


def from_dev_u32(T) -> np.ndarray:
    return T.cpu().numpy().view(np.uint32)


def centred_i8(A: np.ndarray, p: int) -> np.ndarray:
    return np.where(A > (p - 1) // 2, A.astype(np.int64) - p, A).astype(np.int8)


def limbs(A: np.ndarray, p: int) -> np.ndarray:
    x = np.where(A <= 32639, A.astype(np.int64), A.astype(np.int64) - p)
    lo = ((x + 128) & 255) - 128
    hi = (x - lo) >> 8
    return np.stack([hi.astype(np.int8), lo.astype(np.int8)])


def set_kblk(k: int):
    f = ffp.lib().ffp_debug_set_kblk
    f.argtypes = [ctypes.c_int64]
    f.restype = None
    f(k)


def lower_mask(n):
    return np.tril(np.ones((n, n), dtype=bool))


def set_knob(key: str, value: int):
    f = ffp.lib().ffp_debug_set
    f.argtypes = [ctypes.c_char_p, ctypes.c_int64]
    f.restype = ctypes.c_int
    assert f(key.encode(), value) == 0
