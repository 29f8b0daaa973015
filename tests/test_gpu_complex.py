"""GPU parity of fzsyrk_modp (A A^T over F_p[i], Section 3.1) and fherk_modp
(A A^H, Section 3.3) against the oracle's plain sums over F_p[i], bit for
bit: depth 0 (the 2M leaves alone) to 3, ragged shapes that need padding,
the full output (upper triangle mirrored, conjugated for A A^H)."""
import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp
from tests.gpu_util import from_dev_u32, to_dev_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    oracle.build(force=False)
    ffp.lib()


def run(A, p, herk, depth, fill_upper=True):
    import torch
    Ad = to_dev_u32(A)
    C = ffp.complex_syrk(Ad, p, herk=herk, depth=depth, fill_upper=fill_upper)
    torch.cuda.synchronize()
    return from_dev_u32(C)


@pytest.mark.parametrize("herk", [False, True])
@pytest.mark.parametrize("p", [3, 251, 65521, 131071, 1000003, 94906249])
@pytest.mark.parametrize("n,k,depth", [(1, 1, 0), (5, 3, 0), (64, 64, 1), (100, 37, 2), (300, 257, 2),
                                       (512, 512, 3), (130, 1000, 1)])
def test_complex_vs_oracle(herk, p, n, k, depth):
    rng = np.random.default_rng(n + 3 * k + p + int(herk))
    A = rng.integers(0, p, size=(2, n, k), dtype=np.uint64).astype(np.uint32)
    A[:, 0, :] = p - 1
    got = run(A, p, herk, depth)
    want_re, want_im = (oracle.herk if herk else oracle.zsyrk)(A[0], A[1], p)
    assert np.array_equal(got[0], want_re)
    assert np.array_equal(got[1], want_im)


@pytest.mark.parametrize("herk", [False, True])
def test_complex_default_depth_and_lower_only(herk):
    """Default depth on a 2048 x 1536 operand; without FFP_FILL_UPPER only
    the lower triangles are compared (the upper ones are scratch)."""
    p, n, k = 131071, 2048, 1536
    rng = np.random.default_rng(5 + int(herk))
    A = rng.integers(0, p, size=(2, n, k), dtype=np.uint64).astype(np.uint32)
    got = run(A, p, herk, None, fill_upper=False)
    want_re, want_im = (oracle.herk if herk else oracle.zsyrk)(A[0], A[1], p)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(got[0][low], want_re[low])
    assert np.array_equal(got[1][low], want_im[low])


def test_hermitian_diagonal_is_real():
    p, n, k = 65537, 96, 80
    rng = np.random.default_rng(1)
    A = rng.integers(0, p, size=(2, n, k), dtype=np.uint64).astype(np.uint32)
    got = run(A, p, True, 2)
    assert not np.diag(got[1]).any()
    assert np.array_equal(got[0], got[0].T)
    assert np.array_equal((got[1] + got[1].T) % p, np.zeros((n, n), dtype=np.uint32))
