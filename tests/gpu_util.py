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


def _profile_lib():
    L = ffp.lib()
    L.ffp_debug_profile.argtypes = [ctypes.c_int]
    L.ffp_debug_profile.restype = None
    for f in (L.ffp_debug_profile_read, L.ffp_debug_profile_read_variant):
        f.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                      ctypes.POINTER(ctypes.c_int64)]
        f.restype = ctypes.c_int
    return L


def product_launches(fn, cls=-1, variant=None) -> int:
    """Runs fn with the library's product-launch profiling on and returns
    the number of product launches of base class cls (-1: all), or of
    product-kernel variant `variant`; the other records are dropped."""
    L = _profile_lib()
    ms, fl, n, rest = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
    L.ffp_debug_profile(1)
    try:
        fn()
        if variant is None:
            assert L.ffp_debug_profile_read(cls, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(n)) == 0
        else:
            assert L.ffp_debug_profile_read_variant(variant, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(n)) == 0
        L.ffp_debug_profile_read(-1, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(rest))
    finally:
        L.ffp_debug_profile(0)
    return n.value
