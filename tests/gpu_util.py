"""Helpers shared by the GPU tests: device upload and the C-ABI calls with
torch tensors (marshalling only)."""
import ctypes

import numpy as np

from paper_2001_04109_amd import ffp
from paper_2001_04109_amd.storage import centred_i8, limbs  # noqa: F401 (re-exported for the tests)


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev_u32(A: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(A).view(np.int32)).to(dev())


def from_dev_u32(T) -> np.ndarray:
    return T.cpu().numpy().view(np.uint32)


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
