"""CPU tests of the product library's host side: it loads and exports every
entry point declared in include/*.h, and its field routines (Section 3.1)
agree with the pinned oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M):
            if m.group(1) not in ("if", "while", "for", "return", "sizeof", "defined"):
                names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = ffp.lib()
    names = declared_functions()
    assert "fsyrk_modp" in names and "fldlt_modp" in names and "fgemm_modp" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_strerror_and_version():
    assert ffp.strerror(ffp.FFP_EPRIME).startswith("modulus")
    assert "gfx950" in ffp.ffp_version()


PRIMES = [2, 3, 5, 7, 11, 13, 17, 251, 257, 65521, 65537, 131041, 131071, 1000003, 33554393,
          33554467, 94906249, 2147483647]


@pytest.mark.parametrize("p", PRIMES)
def test_field_plan_is_skew_orthogonal(p):
    a, b, y = ffp.field_info(p)
    if p == 2:
        assert (a, b, y) == (1, 0, 1)     # 1 = -1: Y = I
        return
    assert (a * a + b * b) % p == p - 1
    if p % 4 == 1:
        assert b == 0 and y == 1
    elif p % 8 == 3:
        assert a == 1 and y == 2
        assert b == oracle.sqrt_mod(p - 2, p)
    else:
        assert y == 3
        assert (a, b) == oracle.sos(p, p - 1)


def test_field_plan_every_prime_below_2_13():
    for p in range(3, 1 << 13):
        if not oracle.is_prime(p):
            continue
        a, b, _ = ffp.field_info(p)
        assert (a * a + b * b) % p == p - 1, p


def test_host_sqrt_matches_oracle():
    rng = np.random.default_rng(0)
    for p in PRIMES[1:]:                  # odd primes
        for a in rng.integers(0, p, size=40):
            assert ffp.host_sqrt(int(a), p) == oracle.sqrt_mod(int(a), p), (a, p)


def test_host_sos_and_nrsyf_match_oracle():
    rng = np.random.default_rng(1)
    for p in [251, 65521, 65537, 131071, 1000003]:
        for k in rng.integers(0, p, size=20):
            assert ffp.host_sos(p, int(k)) == oracle.sos(p, int(k))
        nonres = [x for x in range(2, min(p, 300)) if oracle.legendre(x, p) == -1][:10]
        for al in nonres:
            for be in nonres:
                assert ffp.host_nrsyf(p, al, be) == oracle.nrsyf(p, al, be).tolist()


def test_non_prime_rejected():
    with pytest.raises(ffp.FfpError):
        ffp.field_info(65535)
    with pytest.raises(ffp.FfpError):
        ffp.plan_describe(8, 8, 91)


def test_workspace_bytes_monotone():
    low = ffp.FFP_DEPTH(2) | ffp.FFP_LOW_MEMORY
    w1 = ffp.ffp_workspace_bytes(1024, 1024, 131071, 0, low)
    w2 = ffp.ffp_workspace_bytes(1024, 4096, 131071, 0, low)
    w3 = ffp.ffp_workspace_bytes(1024, 1024, 131071, 0, low | ffp.FFP_WS_BETA)
    assert w1 == 0 and w2 > 0 and w3 > 0
    # the default (wide) placements trade memory for independent products
    w4 = ffp.ffp_workspace_bytes(1024, 1024, 131071, 0, ffp.FFP_DEPTH(2))
    assert w4 > 0
    L = ffp.lib()
    L.ffp_ldlt_workspace_bytes.restype = ctypes.c_size_t
    L.ffp_ldlt_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_uint32]
    assert L.ffp_ldlt_workspace_bytes(4096, 65537) > 0
    assert L.ffp_ldlt_workspace_bytes(4096, 65535) == 0


def test_syrkbd_argument_checks():
    # validated synchronously, before anything touches a device
    assert ffp.lib().fsyrkbd_modp(4, 4, 2, 16, 4, 16, 16, 1, 0, 16, 4, None, 0, None) == ffp.FFP_EPRIME
    assert ffp.lib().fsyrkbd_modp(4, 4, 15, 16, 4, 16, 16, 1, 0, 16, 4, None, 0, None) == ffp.FFP_EPRIME
    assert ffp.lib().fsyrkbd_modp(4, 4, 7, 16, 4, 16, None, 1, 0, 16, 4, None, 0, None) == ffp.FFP_EINVAL
    assert ffp.lib().fsyrkbd_modp(4, 4, 7, 16, 3, 16, 16, 1, 0, 16, 4, None, 0, None) == ffp.FFP_EINVAL
    assert ffp.lib().fsyrkbd_modp(4, 4, 7, 16, 4, 16, 16, 7, 0, 16, 4, None, 0, None) == ffp.FFP_EINVAL
    assert ffp.lib().fsyrkbd_modp(-1, 4, 7, 16, 4, 16, 16, 1, 0, 16, 4, None, 0, None) == ffp.FFP_EINVAL
    assert ffp.lib().fsyrkbd_modp(0, 4, 7, 16, 4, 16, 16, 1, 0, 16, 4, None, 0, None) == ffp.FFP_OK


def test_complex_argument_checks():
    L = ffp.lib()
    for f in (L.fzsyrk_modp, L.fherk_modp):
        assert f(4, 4, 2, 16, 4, 16, 16, 4, 16, 0, None) == ffp.FFP_EPRIME
        assert f(4, 4, 9, 16, 4, 16, 16, 4, 16, 0, None) == ffp.FFP_EPRIME
        assert f(4, 4, 7, 16, 3, 16, 16, 4, 16, 0, None) == ffp.FFP_EINVAL   # lda < k
        assert f(4, 4, 7, 16, 4, 8, 16, 4, 16, 0, None) == ffp.FFP_EINVAL    # planes of A overlap
        assert f(4, 4, 7, 16, 4, 16, 16, 4, 8, 0, None) == ffp.FFP_EINVAL    # planes of C overlap
        assert f(4, 4, 7, 16, 4, 16, 16, 4, 16, 0x100, None) == ffp.FFP_EINVAL
        assert f(0, 4, 7, 16, 4, 16, 16, 4, 16, 0, None) == ffp.FFP_OK
