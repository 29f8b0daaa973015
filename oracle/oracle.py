"""ctypes binding of the C oracle (ffp_oracle.c).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain definition of each
operation of Dumas, Pernet and Sedoglavic, "On Fast Multiplication of a
Matrix by its Transpose" (arXiv:2001.04109), computed on the CPU with exact
128-bit integer accumulation.  It shares no code with the HIP library.

Arrays are numpy uint32 in [0, p), row-major.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ffp_oracle.c")
_LIB = os.path.join(_HERE, "libffp_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP) into oracle/libffp_oracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-Wextra", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u64, i64, c_int = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
        P = ctypes.c_void_p
        sigs = {
            "oracle_powmod": (u64, [u64, u64, u64]),
            "oracle_is_prime": (c_int, [u64]),
            "oracle_legendre": (c_int, [u64, u64]),
            "oracle_inv": (u64, [u64, u64]),
            "oracle_sqrt_mod": (u64, [u64, u64]),
            "oracle_sos": (c_int, [u64, u64, P, P]),
            "oracle_nrsyf": (c_int, [u64, u64, u64, P]),
            "oracle_syrk": (c_int, [i64, i64, u64, P, i64, P, i64]),
            "oracle_syrk_rows": (c_int, [i64, i64, u64, P, i64, i64, i64, P, i64]),
            "oracle_syrk_entries": (c_int, [i64, i64, u64, P, i64, i64, P, P, P]),
            "oracle_gemm": (c_int, [i64, i64, i64, u64, P, i64, P, i64, u64, u64, P, i64]),
            "oracle_syrk_ab": (c_int, [i64, i64, u64, P, i64, u64, u64, P, i64]),
            "oracle_syrkd": (c_int, [i64, i64, u64, P, i64, P, P, i64]),
            "oracle_ldlt": (c_int, [i64, u64, P, i64, P]),
            "oracle_syrkbd": (c_int, [i64, i64, u64, P, i64, P, P, u64, u64, P, i64]),
            "oracle_herk": (c_int, [i64, i64, u64, P, i64, i64, P, i64, i64]),
            "oracle_zsyrk": (c_int, [i64, i64, u64, P, i64, i64, P, i64, i64]),
            "oracle_num_threads": (c_int, []),
            "oracle_set_num_threads": (None, [c_int]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _u32(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != np.uint32:
        raise TypeError(f"oracle expects uint32 residues, got {a.dtype}")
    return a


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid argument (rc={rc})")


def is_prime(p: int) -> bool:
    return bool(load().oracle_is_prime(p))


def legendre(a: int, p: int) -> int:
    return int(load().oracle_legendre(a, p))


def inv_mod(a: int, p: int) -> int:
    return int(load().oracle_inv(a, p))


def sqrt_mod(a: int, p: int):
    """Canonical square root min(r, p-r) of a mod p, or None if a is not a square."""
    r = int(load().oracle_sqrt_mod(a, p))
    return None if r == 2**64 - 1 else r


def sos(p: int, k: int):
    """Algorithm 3: (a, b) with a^2 + b^2 = k mod p."""
    a = ctypes.c_uint64()
    b = ctypes.c_uint64()
    _check(load().oracle_sos(p, k, ctypes.byref(a), ctypes.byref(b)), "sos")
    return int(a.value), int(b.value)


def nrsyf(p: int, alpha: int, beta: int) -> np.ndarray:
    """Algorithm 4: 2x2 Y with Y Y^T = diag(alpha, beta) for non-residues alpha, beta."""
    y = np.zeros(4, dtype=np.uint64)
    _check(load().oracle_nrsyf(p, alpha, beta, _ptr(y)), "nrsyf")
    return y.reshape(2, 2)


def syrk(A, p: int) -> np.ndarray:
    """Full symmetric C = A A^T mod p."""
    A = _u32(A)
    n, k = A.shape
    C = np.zeros((n, n), dtype=np.uint32)
    _check(load().oracle_syrk(n, k, p, _ptr(A), max(k, 1), _ptr(C), max(n, 1)), "syrk")
    return C


def syrk_rows(A, p: int, i0: int, i1: int) -> np.ndarray:
    """Rows [i0, i1) of lower(A A^T mod p); entries above the diagonal are 0."""
    A = _u32(A)
    n, k = A.shape
    out = np.zeros((i1 - i0, max(i1, 1)), dtype=np.uint32)
    _check(load().oracle_syrk_rows(n, k, p, _ptr(A), max(k, 1), i0, i1, _ptr(out),
                                   max(i1, 1)), "syrk_rows")
    return out


def syrk_entries(A, p: int, rows, cols) -> np.ndarray:
    """Entries (rows[t], cols[t]) of A A^T mod p."""
    A = _u32(A)
    n, k = A.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if rows.shape != cols.shape:
        raise ValueError("rows/cols shape mismatch")
    if rows.size and (rows.min() < 0 or rows.max() >= n or cols.min() < 0 or cols.max() >= n):
        raise ValueError("sample index out of range")
    out = np.zeros(rows.shape, dtype=np.uint32)
    _check(load().oracle_syrk_entries(n, k, p, _ptr(A), max(k, 1), rows.size, _ptr(rows),
                                      _ptr(cols), _ptr(out)), "syrk_entries")
    return out


def gemm(A, B, p: int, alpha: int = 1, beta: int = 0, C=None) -> np.ndarray:
    """C <- alpha A B^T + beta C mod p (a new array is returned)."""
    A = _u32(A)
    B = _u32(B)
    m, k = A.shape
    n, k2 = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    C = np.zeros((m, n), dtype=np.uint32) if C is None else _u32(C).copy()
    _check(load().oracle_gemm(m, n, k, p, _ptr(A), max(k, 1), _ptr(B), max(k, 1),
                              alpha, beta, _ptr(C), max(n, 1)), "gemm")
    return C


def syrk_ab(A, p: int, alpha: int, beta: int, C) -> np.ndarray:
    """lower(C) <- alpha A A^T + beta lower(C) mod p; the strict upper part is copied unchanged."""
    A = _u32(A)
    n, k = A.shape
    C = _u32(C).copy()
    _check(load().oracle_syrk_ab(n, k, p, _ptr(A), max(k, 1), alpha, beta, _ptr(C),
                                 max(n, 1)), "syrk_ab")
    return C


def syrkd(A, d, p: int) -> np.ndarray:
    """Full symmetric A diag(d) A^T mod p."""
    A = _u32(A)
    d = _u32(d)
    m, n = A.shape
    C = np.zeros((m, m), dtype=np.uint32)
    _check(load().oracle_syrkd(m, n, p, _ptr(A), max(n, 1), _ptr(d), _ptr(C), max(m, 1)),
           "syrkd")
    return C


def ldlt(S, p: int):
    """Crout LDL^T of the lower triangle of S mod p.

    Returns (L, D, info): L unit lower triangular (n x n), D the diagonal
    (length n), info = 0 or the 1-based index of the first zero pivot.
    """
    S = _u32(S).copy()
    n = S.shape[0]
    info = ctypes.c_int64(0)
    _check(load().oracle_ldlt(n, p, _ptr(S), max(n, 1), ctypes.byref(info)), "ldlt")
    L = np.tril(S, -1)
    L[np.arange(n), np.arange(n)] = 1
    D = S[np.arange(n), np.arange(n)].copy()
    return L, D, int(info.value)


def ldlt_packed(S, p: int):
    """Crout LDL^T returning the packed in-place form (strict lower = L, diag = D)."""
    S = _u32(S).copy()
    n = S.shape[0]
    info = ctypes.c_int64(0)
    _check(load().oracle_ldlt(n, p, _ptr(S), max(n, 1), ctypes.byref(info)), "ldlt")
    return S, int(info.value)


def syrkbd(A, bdiag, boff, p: int, alpha: int = 1, beta: int = 0, C=None) -> np.ndarray:
    """alpha A B A^T + beta C mod p (full m x m) with B the symmetric
    tridiagonal matrix of diagonal bdiag (n) and off-diagonal boff (n - 1)."""
    A = _u32(A)
    m, n = A.shape
    bdiag = _u32(np.asarray(bdiag, dtype=np.uint32).reshape(n))
    boff = _u32(np.zeros(1, dtype=np.uint32) if n <= 1 else np.asarray(boff, dtype=np.uint32).reshape(n - 1))
    C = np.zeros((m, m), dtype=np.uint32) if C is None else _u32(C).copy()
    _check(load().oracle_syrkbd(m, n, p, _ptr(A), max(n, 1), _ptr(bdiag), _ptr(boff), alpha, beta,
                                _ptr(C), max(m, 1)), "syrkbd")
    return C


def _cplx(re, im):
    re, im = _u32(re), _u32(im)
    if re.shape != im.shape:
        raise ValueError("real and imaginary planes differ in shape")
    return np.ascontiguousarray(np.stack([re, im]))


def herk(re, im, p: int):
    """(Re, Im) of A A^H over F_p[i] (conj(a + ib) = a - ib), full n x n."""
    A = _cplx(re, im)
    _, n, k = A.shape
    C = np.zeros((2, n, n), dtype=np.uint32)
    _check(load().oracle_herk(n, k, p, _ptr(A), max(k, 1), n * k, _ptr(C), max(n, 1), n * n), "herk")
    return C[0], C[1]


def zsyrk(re, im, p: int):
    """(Re, Im) of A A^T over F_p[i] (no conjugation), full n x n."""
    A = _cplx(re, im)
    _, n, k = A.shape
    C = np.zeros((2, n, n), dtype=np.uint32)
    _check(load().oracle_zsyrk(n, k, p, _ptr(A), max(k, 1), n * k, _ptr(C), max(n, 1), n * n), "zsyrk")
    return C[0], C[1]


def num_threads() -> int:
    return int(load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only)."""
    load().oracle_set_num_threads(int(n))
