"""Python binding of libffp.so (include/ffp.h, include/ffp_debug.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device memory and streams come from PyTorch; matrices of residues
are int32 tensors (values in [0, p), p <= 94906249), int8 tensors for the
int8 storages.  The functions raise FfpError on a negative status and
ImportError/OSError when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# FFP_LIBRARY: another build of the library to load instead (the host
# AddressSanitizer build of paper_2001_04109_amd.build, for host tests)
LIB_PATH = os.environ.get("FFP_LIBRARY") or os.path.join(HERE, "libffp.so")

FFP_OK = 0
FFP_EINVAL = -1
FFP_EPRIME = -2
FFP_EDTYPE = -3
FFP_ENOMEM = -4
FFP_EDEVICE = -5
FFP_EUNSUPPORTED = -6
FFP_ECANCELED = -7
FFP_ETIMEDOUT = -8

FFP_U32 = 0
FFP_I8_CENTERED = 1
FFP_I8_LIMB2 = 2

FFP_FILL_UPPER = 0x1
FFP_BASE_F64 = 0x100
FFP_LOW_MEMORY = 0x200
FFP_BASE_LIMB3 = 0x400
FFP_WS_BETA = 0x80000000


def FFP_DEPTH(d: int) -> int:
    return ((d & 0x7) + 1) << 4


class FfpError(RuntimeError):
    def __init__(self, status: int, what: str):
        detail = ""
        if status in (FFP_ENOMEM, FFP_EDEVICE):
            try:
                d = lib().ffp_last_error_detail().decode()
                detail = f" [{d}]" if d else ""
            except Exception:  # library missing: the status alone
                pass
        super().__init__(f"{what}: {strerror(status)} (status {status}){detail}")
        self.status = status


class ffp_job(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("k", ctypes.c_int64), ("p", ctypes.c_uint32),
                ("alpha", ctypes.c_uint32), ("beta", ctypes.c_uint32), ("a_dtype", ctypes.c_int32),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("C", ctypes.c_void_p),
                ("ldc", ctypes.c_int64)]


class ffp_ldlt_job(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("p", ctypes.c_uint32), ("S", ctypes.c_void_p),
                ("lds", ctypes.c_int64), ("info", ctypes.c_void_p)]


class ffp_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("p", ctypes.c_uint32), ("alpha", ctypes.c_uint32), ("A", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("timeout_s", ctypes.c_double)]


class ffp_result(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64),
                ("info", ctypes.c_void_p), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ffp_tune_result(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("tile", ctypes.c_int32), ("wide", ctypes.c_int32),
                ("base", ctypes.c_int32), ("candidates", ctypes.c_int32), ("ms", ctypes.c_double),
                ("rule_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ffp_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("units", ctypes.c_int64), ("batched_jobs", ctypes.c_int64),
                ("max_batch", ctypes.c_int64), ("peak_inflight", ctypes.c_int64),
                ("overlapped_units", ctypes.c_int64), ("peak_bytes", ctypes.c_size_t)]


FFP_REQ_SYRK = 0
FFP_REQ_LDLT = 1
FFP_STATE_QUEUED = 0
FFP_STATE_RUNNING = 1
FFP_STATE_DONE = 2

_lib = None


def lib():
    """Load libffp.so (built by paper_2001_04109_amd.build); raises if missing."""
    global _lib
    if _lib is None:
        # torch first: the library must bind to the HIP runtime torch loads
        # (the one that owns the device memory and streams passed in);
        # loading the system runtime before torch's gives a second runtime
        # in the process that sees no device.
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover - host-only use without torch
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2001_04109_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i64, u32, P, c_int, c_uint = (ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p,
                                      ctypes.c_int, ctypes.c_uint)
        sigs = {
            "fsyrk_modp": (c_int, [i64, i64, u32, P, i64, c_int, u32, u32, P, i64, c_uint, P]),
            "fsyrk_modp_noalloc": (c_int, [i64, i64, u32, P, i64, c_int, u32, u32, P, i64, c_uint, P]),
            "ffp_noalloc_scratch_bytes": (ctypes.c_size_t, []),
            "fgemm_modp": (c_int, [i64, i64, i64, u32, P, i64, P, i64, u32, u32, P, i64, P]),
            "fldlt_modp": (c_int, [i64, u32, P, i64, P, P]),
            "fsyrkbd_modp": (c_int, [i64, i64, u32, P, i64, P, P, u32, u32, P, i64, P, c_uint, P]),
            "fzsyrk_modp": (c_int, [i64, i64, u32, P, i64, i64, P, i64, i64, c_uint, P]),
            "fherk_modp": (c_int, [i64, i64, u32, P, i64, i64, P, i64, i64, c_uint, P]),
            "ffp_workspace_bytes": (ctypes.c_size_t, [i64, i64, u32, c_int, c_uint]),
            "fsyrk_modp_batched": (c_int, [c_int, P, c_uint, P]),
            "ffp_strerror": (ctypes.c_char_p, [c_int]),
            "ffp_version": (ctypes.c_char_p, []),
            "ffp_last_error_detail": (ctypes.c_char_p, []),
            "ffp_field_info": (c_int, [u32, P, P, P]),
            "ffp_host_sqrt": (c_int, [u32, u32, P]),
            "ffp_host_sos": (c_int, [u32, u32, P, P]),
            "ffp_host_nrsyf": (c_int, [u32, u32, u32, P]),
            "ffp_plan_describe": (c_int, [i64, i64, u32, c_int, i64, i64, u32, u32, c_uint,
                                          ctypes.c_char_p, ctypes.c_size_t]),
            "ffp_ldlt_workspace_bytes": (ctypes.c_size_t, [i64, u32]),
            "ffp_complex_plan_describe": (c_int, [i64, i64, u32, c_int, i64, i64, i64, i64, c_uint,
                                                  ctypes.c_char_p, ctypes.c_size_t]),
            "ffp_complex_plan_levels": (c_int, [i64, i64, u32, c_int, i64, i64, i64, i64, c_uint, P,
                                                ctypes.c_size_t]),
            "ffp_plan_levels": (c_int, [i64, i64, u32, c_int, i64, i64, u32, u32, c_uint, P,
                                        ctypes.c_size_t]),
            "fldlt_modp_batched": (c_int, [c_int, P, P]),
            "ffp_server_create": (c_int, [ctypes.c_size_t, c_int, c_int, P]),
            "ffp_server_create_simulated": (c_int, [ctypes.c_size_t, c_int, c_int, ctypes.c_double,
                                                    ctypes.c_double, P]),
            "ffp_server_submit": (c_int, [P, P, P]),
            "ffp_server_status": (c_int, [P, ctypes.c_uint64, P]),
            "ffp_server_release": (c_int, [P, ctypes.c_uint64]),
            "ffp_server_drain": (c_int, [P, ctypes.c_double]),
            "ffp_server_stats": (c_int, [P, P]),
            "ffp_server_poll": (c_int, [P, P, c_int, ctypes.c_double, P]),
            "ffp_server_fetch": (c_int, [P, ctypes.c_uint64, P, i64, P, P]),
            "ffp_server_cancel": (c_int, [P, ctypes.c_uint64]),
            "ffp_server_destroy": (c_int, [P]),
            "ffp_graph_syrk_batched": (c_int, [c_int, P, c_uint, P, P]),
            "ffp_graph_ldlt_batched": (c_int, [c_int, P, P, P]),
            "ffp_graph_launch": (c_int, [P, P]),
            "ffp_graph_device_bytes": (ctypes.c_size_t, [P]),
            "ffp_graph_nodes": (ctypes.c_size_t, [P]),
            "ffp_graph_destroy": (None, [P]),
            "ffp_autotune": (c_int, [i64, i64, u32, c_int, u32, u32, c_uint, P, P]),
            "ffp_tune_lookup": (c_int, [i64, i64, u32, c_int, u32, u32, c_uint, P]),
            "ffp_tune_save": (c_int, [ctypes.c_char_p]),
            "ffp_tune_load": (c_int, [ctypes.c_char_p]),
            "ffp_tune_clear": (None, []),
            "ffp_tune_entries": (c_int, []),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(status: int) -> str:
    try:
        return lib().ffp_strerror(status).decode()
    except Exception:  # library missing: still give a readable message
        return f"status {status}"


def _check(st: int, what: str):
    if st < 0:
        raise FfpError(st, what)
    return st


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- C-ABI entry points (same names and argument order) ------------------

def fsyrk_modp(n, k, p, A, lda, a_dtype, alpha, beta, C, ldc, flags=0, stream=None):
    return _check(lib().fsyrk_modp(n, k, p, _ptr(A), lda, a_dtype, alpha, beta, _ptr(C), ldc,
                                   flags, _stream(stream)), "fsyrk_modp")


def fsyrk_modp_noalloc(n, k, p, A, lda, a_dtype, alpha, beta, C, ldc, flags=0, stream=None):
    return _check(lib().fsyrk_modp_noalloc(n, k, p, _ptr(A), lda, a_dtype, alpha, beta, _ptr(C), ldc,
                                           flags, _stream(stream)), "fsyrk_modp_noalloc")


def ffp_noalloc_scratch_bytes() -> int:
    return lib().ffp_noalloc_scratch_bytes()


def fgemm_modp(m, n, k, p, A, lda, B, ldb, alpha, beta, C, ldc, stream=None):
    return _check(lib().fgemm_modp(m, n, k, p, _ptr(A), lda, _ptr(B), ldb, alpha, beta, _ptr(C),
                                   ldc, _stream(stream)), "fgemm_modp")


def fldlt_modp(n, p, S, lds, info, stream=None):
    return _check(lib().fldlt_modp(n, p, _ptr(S), lds, _ptr(info), _stream(stream)), "fldlt_modp")


def fsyrkbd_modp(m, n, p, A, lda, bdiag, boff, alpha, beta, C, ldc, info=None, flags=0, stream=None):
    return _check(lib().fsyrkbd_modp(m, n, p, _ptr(A), lda, _ptr(bdiag), _ptr(boff), alpha, beta, _ptr(C),
                                     ldc, _ptr(info), flags, _stream(stream)), "fsyrkbd_modp")


def fzsyrk_modp(n, k, p, A, lda, a_plane, C, ldc, c_plane, flags=0, stream=None):
    return _check(lib().fzsyrk_modp(n, k, p, _ptr(A), lda, a_plane, _ptr(C), ldc, c_plane, flags,
                                    _stream(stream)), "fzsyrk_modp")


def fherk_modp(n, k, p, A, lda, a_plane, C, ldc, c_plane, flags=0, stream=None):
    return _check(lib().fherk_modp(n, k, p, _ptr(A), lda, a_plane, _ptr(C), ldc, c_plane, flags,
                                   _stream(stream)), "fherk_modp")


def ffp_workspace_bytes(n, k, p, a_dtype=FFP_U32, flags=0) -> int:
    return int(lib().ffp_workspace_bytes(n, k, p, a_dtype, flags))


def ffp_ldlt_workspace_bytes(n, p) -> int:
    return int(lib().ffp_ldlt_workspace_bytes(n, p))


def fsyrk_modp_batched(jobs, flags=0, stream=None):
    arr = (ffp_job * len(jobs))(*jobs)
    return _check(lib().fsyrk_modp_batched(len(jobs), ctypes.cast(arr, ctypes.c_void_p), flags,
                                           _stream(stream)), "fsyrk_modp_batched")


def ffp_graph_syrk_batched(jobs, flags=0, stream=None) -> int:
    arr = (ffp_job * len(jobs))(*jobs)
    g = ctypes.c_void_p()
    _check(lib().ffp_graph_syrk_batched(len(jobs), ctypes.cast(arr, ctypes.c_void_p), flags,
                                        _stream(stream), ctypes.byref(g)), "ffp_graph_syrk_batched")
    return g.value or 0


def ffp_graph_ldlt_batched(jobs, stream=None) -> int:
    arr = (ffp_ldlt_job * len(jobs))(*jobs)
    g = ctypes.c_void_p()
    _check(lib().ffp_graph_ldlt_batched(len(jobs), ctypes.cast(arr, ctypes.c_void_p),
                                        _stream(stream), ctypes.byref(g)), "ffp_graph_ldlt_batched")
    return g.value or 0


def ffp_graph_launch(g: int, stream=None):
    return _check(lib().ffp_graph_launch(g, _stream(stream)), "ffp_graph_launch")


def ffp_graph_device_bytes(g: int) -> int:
    return int(lib().ffp_graph_device_bytes(g))


def ffp_graph_nodes(g: int) -> int:
    return int(lib().ffp_graph_nodes(g))


def ffp_graph_destroy(g: int):
    if g:
        lib().ffp_graph_destroy(g)


def ffp_autotune(n, k, p, a_dtype=FFP_U32, alpha=1, beta=0, flags=0, stream=None) -> dict:
    r = ffp_tune_result()
    _check(lib().ffp_autotune(n, k, p, a_dtype, alpha, beta, flags, _stream(stream), ctypes.byref(r)),
           "ffp_autotune")
    return r.as_dict()


def ffp_tune_lookup(n, k, p, a_dtype=FFP_U32, alpha=1, beta=0, flags=0) -> dict:
    """The depth, tile and placements a call of this shape uses now, and
    whether they come from the tuning table (key "tuned")."""
    r = ffp_tune_result()
    st = _check(lib().ffp_tune_lookup(n, k, p, a_dtype, alpha, beta, flags, ctypes.byref(r)),
                "ffp_tune_lookup")
    d = r.as_dict()
    d["tuned"] = bool(st)
    return d


def ffp_tune_save(path: str):
    _check(lib().ffp_tune_save(os.fsencode(path)), "ffp_tune_save")


def ffp_tune_load(path: str) -> int:
    return _check(lib().ffp_tune_load(os.fsencode(path)), "ffp_tune_load")


def ffp_tune_clear():
    lib().ffp_tune_clear()


def ffp_tune_entries() -> int:
    return int(lib().ffp_tune_entries())


class Graph:
    """A recorded batched call (ffp_graph_* of include/ffp.h).  The recording
    stream must not be the null stream; keep the jobs' tensors alive while the
    graph exists."""

    def __init__(self, handle: int, keep=()):
        self.handle = handle
        self._keep = keep

    @classmethod
    def syrk_batched(cls, jobs, flags=0, stream=None, keep=()):
        return cls(ffp_graph_syrk_batched(jobs, flags, stream), keep)

    @classmethod
    def ldlt_batched(cls, jobs, stream=None, keep=()):
        return cls(ffp_graph_ldlt_batched(jobs, stream), keep)

    def launch(self, stream=None):
        ffp_graph_launch(self.handle, stream)

    @property
    def device_bytes(self) -> int:
        return ffp_graph_device_bytes(self.handle)

    @property
    def nodes(self) -> int:
        return ffp_graph_nodes(self.handle)

    def close(self):
        ffp_graph_destroy(self.handle)
        self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def make_job(A, C, p, alpha=1, beta=0, a_dtype=FFP_U32) -> ffp_job:
    n, k = A.shape
    return ffp_job(n=n, k=k, p=p, alpha=alpha, beta=beta, a_dtype=a_dtype, A=_ptr(A),
                   lda=A.stride(0), C=_ptr(C), ldc=C.stride(0))


def ffp_version() -> str:
    return lib().ffp_version().decode()


# ---- host-only introspection ---------------------------------------------

def field_info(p: int):
    a, b, y = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_int()
    _check(lib().ffp_field_info(p, ctypes.byref(a), ctypes.byref(b), ctypes.byref(y)), "field_info")
    return a.value, b.value, y.value


def host_sqrt(a: int, p: int):
    r = ctypes.c_uint32()
    st = lib().ffp_host_sqrt(a, p, ctypes.byref(r))
    if st == FFP_EINVAL:
        return None
    _check(st, "host_sqrt")
    return r.value


def host_sos(p: int, k: int):
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().ffp_host_sos(p, k, ctypes.byref(a), ctypes.byref(b)), "host_sos")
    return a.value, b.value


def host_nrsyf(p: int, alpha: int, beta: int):
    Y = (ctypes.c_uint32 * 4)()
    _check(lib().ffp_host_nrsyf(p, alpha, beta, Y), "host_nrsyf")
    return [[Y[0], Y[1]], [Y[2], Y[3]]]


def plan_describe(n, k, p, a_dtype=FFP_U32, lda=None, ldc=None, alpha=1, beta=0, flags=0) -> str:
    lda = k if lda is None else lda
    ldc = n if ldc is None else ldc
    size = _check(lib().ffp_plan_describe(n, k, p, a_dtype, lda, ldc, alpha, beta, flags, None, 0),
                  "plan_describe")
    buf = ctypes.create_string_buffer(size + 1)
    _check(lib().ffp_plan_describe(n, k, p, a_dtype, lda, ldc, alpha, beta, flags, buf, size + 1),
           "plan_describe")
    return buf.value.decode()


def complex_plan_describe(n, k, p, herk=False, lda=None, ldc=None, flags=0) -> str:
    """The host schedule of fzsyrk_modp / fherk_modp (planes stacked: the
    imaginary plane n*lda elements after the real one)."""
    lda = k if lda is None else lda
    ldc = n if ldc is None else ldc
    size = _check(lib().ffp_complex_plan_describe(n, k, p, int(herk), lda, n * lda, ldc, n * ldc, flags,
                                                  None, 0), "complex_plan_describe")
    buf = ctypes.create_string_buffer(size + 1)
    lib().ffp_complex_plan_describe(n, k, p, int(herk), lda, n * lda, ldc, n * ldc, flags, buf, size + 1)
    return buf.value.decode()


def complex_plan_levels(n, k, p, herk=False, lda=None, ldc=None, flags=0) -> list:
    """Scheduler level of every operation of complex_plan_describe's plan."""
    lda = k if lda is None else lda
    ldc = n if ldc is None else ldc
    args = (n, k, p, int(herk), lda, n * lda, ldc, n * ldc, flags)
    cnt = _check(lib().ffp_complex_plan_levels(*args, None, 0), "complex_plan_levels")
    buf = (ctypes.c_int32 * max(cnt, 1))()
    _check(lib().ffp_complex_plan_levels(*args, buf, cnt), "complex_plan_levels")
    return list(buf[:cnt])


def plan_levels(n, k, p, a_dtype=FFP_U32, lda=None, ldc=None, alpha=1, beta=0, flags=0) -> list:
    """Scheduler level of every operation of the plan plan_describe prints."""
    lda = k if lda is None else lda
    ldc = n if ldc is None else ldc
    cnt = _check(lib().ffp_plan_levels(n, k, p, a_dtype, lda, ldc, alpha, beta, flags, None, 0),
                 "plan_levels")
    buf = (ctypes.c_int32 * max(cnt, 1))()
    _check(lib().ffp_plan_levels(n, k, p, a_dtype, lda, ldc, alpha, beta, flags, buf, cnt),
           "plan_levels")
    return list(buf[:cnt])


def set_knob(key: str, value: int):
    """ffp_debug_set: process-wide tuning and test knobs."""
    f = lib().ffp_debug_set
    f.argtypes = [ctypes.c_char_p, ctypes.c_int64]
    f.restype = ctypes.c_int
    _check(f(key.encode(), value), "ffp_debug_set")


# ---- tensor conveniences (marshalling only) -------------------------------

def syrk(A, p: int, alpha: int = 1, beta: int = 0, C=None, depth=None, fill_upper=False,
         a_dtype=FFP_U32, force_f64=False, limb3=False, stream=None):
    """lower(C) <- alpha A A^T + beta lower(C) mod p on device tensors.

    A: (n, k) int32 residues (a_dtype FFP_U32), int8 centred residues
    (FFP_I8_CENTERED), or int8 of shape (2, n, k) holding the hi and lo
    limbs (FFP_I8_LIMB2).  Returns C ((n, n) int32)."""
    import torch
    if a_dtype == FFP_I8_LIMB2:
        _, n, k = A.shape
        lda = A.stride(1)
        if A.stride(0) != n * lda:
            raise ValueError("limb planes must be stacked with stride n*lda")
    else:
        n, k = A.shape
        lda = A.stride(0)
    if A.stride(-1) != 1:
        raise ValueError("A must be row-major")
    if C is None:
        C = torch.zeros((n, n), dtype=torch.int32, device=A.device)
    flags = FFP_FILL_UPPER if fill_upper else 0
    if depth is not None:
        flags |= FFP_DEPTH(depth)
    if force_f64:
        flags |= FFP_BASE_F64
    if limb3:
        flags |= FFP_BASE_LIMB3
    fsyrk_modp(n, k, p, A, lda, a_dtype, alpha, beta, C, C.stride(0), flags, stream)
    return C


def syrkbd(A, bdiag, boff, p: int, alpha: int = 1, beta: int = 0, C=None, info=None, depth=None,
           fill_upper=False, stream=None):
    """lower(C) <- alpha A B A^T + beta lower(C) mod p (Algorithm 6) on device
    int32 tensors: A (m, n), B block diagonal given by bdiag (n) and boff
    (n - 1).  Returns C ((m, m) int32)."""
    import torch
    m, n = A.shape
    if A.stride(-1) != 1:
        raise ValueError("A must be row-major")
    if C is None:
        C = torch.zeros((m, m), dtype=torch.int32, device=A.device)
    flags = FFP_FILL_UPPER if fill_upper else 0
    if depth is not None:
        flags |= FFP_DEPTH(depth)
    fsyrkbd_modp(m, n, p, A, A.stride(0), bdiag, boff if n > 1 else None, alpha, beta, C, C.stride(0), info,
                 flags, stream)
    return C


def complex_syrk(A, p: int, herk: bool = False, C=None, depth=None, fill_upper=False, stream=None):
    """lower(C) <- A A^T (herk: A A^H) over F_p[i] on device int32 tensors:
    A of shape (2, n, k) with the real plane first.  Returns C (2, n, n)."""
    import torch
    _, n, k = A.shape
    if A.stride(-1) != 1:
        raise ValueError("A must be row-major")
    if C is None:
        C = torch.zeros((2, n, n), dtype=torch.int32, device=A.device)
    flags = FFP_FILL_UPPER if fill_upper else 0
    if depth is not None:
        flags |= FFP_DEPTH(depth)
    f = fherk_modp if herk else fzsyrk_modp
    f(n, k, p, A, A.stride(1), A.stride(0), C, C.stride(1), C.stride(0), flags, stream)
    return C


def gemm(A, B, p: int, alpha: int = 1, beta: int = 0, C=None, stream=None):
    """C <- alpha A B^T + beta C mod p on device int32 tensors."""
    import torch
    m, k = A.shape
    n = B.shape[0]
    if C is None:
        C = torch.zeros((m, n), dtype=torch.int32, device=A.device)
    fgemm_modp(m, n, k, p, A, A.stride(0), B, B.stride(0), alpha, beta, C, C.stride(0), stream)
    return C


def ldlt_batched(mats, p_list, stream=None):
    """fldlt_modp_batched over device int32 tensors (in place); returns the
    device int64 info tensor (one entry per job)."""
    import torch
    info = torch.zeros(len(mats), dtype=torch.int64, device=mats[0].device)
    arr = (ffp_ldlt_job * len(mats))()
    for j, (S, p) in enumerate(zip(mats, p_list)):
        arr[j] = ffp_ldlt_job(n=S.shape[0], p=p, S=_ptr(S), lds=S.stride(0),
                              info=info.data_ptr() + 8 * j)
    _check(lib().fldlt_modp_batched(len(mats), ctypes.cast(arr, ctypes.c_void_p), _stream(stream)),
           "fldlt_modp_batched")
    return info


def ldlt(S, p: int, stream=None):
    """In-place LDL^T of the lower triangle of S (n x n int32); returns the
    device int64 info tensor (0, or 1-based index of the first zero pivot)."""
    import torch
    n = S.shape[0]
    info = torch.zeros(1, dtype=torch.int64, device=S.device)
    fldlt_modp(n, p, S, S.stride(0), info, stream)
    return info


# ---- request loop ----------------------------------------------------------

class Server:
    """Continuous-batching request loop (ffp_server_* of include/ffp.h)."""

    def __init__(self, hbm_budget: int, max_inflight: int = 64, nstreams: int = 4,
                 simulated: bool = False, ns_per_op: float = 0.02, launch_us: float = 10.0):
        self._h = ctypes.c_void_p()
        if simulated:
            st = lib().ffp_server_create_simulated(hbm_budget, max_inflight, nstreams, ns_per_op,
                                                   launch_us, ctypes.byref(self._h))
        else:
            st = lib().ffp_server_create(hbm_budget, max_inflight, nstreams, ctypes.byref(self._h))
        _check(st, "ffp_server_create")

    def submit_syrk(self, A, p, alpha=1, n=None, k=None, lda=None, timeout_s=0.0) -> int:
        n = A.shape[0] if n is None else n
        k = A.shape[1] if k is None else k
        lda = A.stride(0) if lda is None else lda
        r = ffp_request(kind=FFP_REQ_SYRK, n=n, k=k, p=p, alpha=alpha, A=_ptr(A), lda=lda,
                        timeout_s=timeout_s)
        return self._submit(r)

    def submit_ldlt(self, S, p, n=None, lds=None, timeout_s=0.0) -> int:
        n = S.shape[0] if n is None else n
        lds = S.stride(0) if lds is None else lds
        r = ffp_request(kind=FFP_REQ_LDLT, n=n, k=n, p=p, alpha=0, A=_ptr(S), lda=lds,
                        timeout_s=timeout_s)
        return self._submit(r)

    def cancel(self, ticket: int):
        """Cancels a still-queued request (FfpError if it was already admitted)."""
        _check(lib().ffp_server_cancel(self._h, ticket), "cancel")

    def _submit(self, r) -> int:
        t = ctypes.c_uint64()
        _check(lib().ffp_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)), "submit")
        return t.value

    def status(self, ticket: int) -> ffp_result:
        out = ffp_result()
        _check(lib().ffp_server_status(self._h, ticket, ctypes.byref(out)), "status")
        return out

    def release(self, ticket: int):
        _check(lib().ffp_server_release(self._h, ticket), "release")

    def drain(self, timeout_s: float = 600.0):
        _check(lib().ffp_server_drain(self._h, timeout_s), "drain")

    def poll(self, max_count: int = 256, timeout_s: float = 0.01) -> list:
        """Tickets finished since the last poll (waits up to timeout_s)."""
        buf = (ctypes.c_uint64 * max_count)()
        cnt = ctypes.c_int()
        _check(lib().ffp_server_poll(self._h, buf, max_count, timeout_s, ctypes.byref(cnt)), "poll")
        return list(buf[:cnt.value])

    def fetch(self, ticket: int, out, info_out=None, stream=None):
        """Copies a done request's result into the device tensor out (n x n
        uint32/int32 view) and, for LDL^T, its info word into info_out."""
        _check(lib().ffp_server_fetch(self._h, ticket, _ptr(out), out.stride(0),
                                      _ptr(info_out) if info_out is not None else None,
                                      _stream(stream)), "fetch")

    def stats(self) -> ffp_serve_stats:
        out = ffp_serve_stats()
        _check(lib().ffp_server_stats(self._h, ctypes.byref(out)), "stats")
        return out

    def close(self):
        if self._h:
            lib().ffp_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
