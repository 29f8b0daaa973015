"""GPU parity over the whole range of moduli the product paths accept: the
smallest prime p = 2 (Y = I) and primes past 2^25 up to 94906249, the
largest with p (p - 1) < 2^53, where the FP64 products reduce their
accumulators after every 4-column matrix-core step.  Bit-exact against the
oracle for fsyrk_modp (depth 0-2, both placements, alpha/beta), fgemm_modp,
fldlt_modp and the batched form."""
import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp, inputs
from tests.gpu_util import from_dev_u32, lower_mask, to_dev_u32

pytestmark = pytest.mark.gpu

BIG = [33554467, 94906249]      # the smallest prime past 2^25; the largest accepted


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    oracle.build(force=False)
    ffp.lib()


def run_syrk(A, p, depth, alpha=1, beta=0, C0=None, flags=0):
    import torch
    n, k = A.shape
    Ad = to_dev_u32(A)
    Cd = to_dev_u32(C0) if C0 is not None else torch.zeros((n, n), dtype=torch.int32, device="cuda")
    ffp.fsyrk_modp(n, k, p, Ad, Ad.stride(0), ffp.FFP_U32, alpha, beta, Cd, Cd.stride(0),
                   flags | ffp.FFP_DEPTH(depth))
    torch.cuda.synchronize()
    return from_dev_u32(Cd)


@pytest.mark.parametrize("p", [2] + BIG)
@pytest.mark.parametrize("depth", [0, 1, 2])
@pytest.mark.parametrize("n,k", [(300, 257), (130, 400)])
def test_syrk_extreme_primes(p, depth, n, k):
    A = inputs.uniform((80, p % 1000, depth), n, k, p)
    m = lower_mask(n)
    ref = oracle.syrk(A, p)
    assert np.array_equal(run_syrk(A, p, depth)[m], ref[m])
    assert np.array_equal(run_syrk(A, p, depth, flags=ffp.FFP_LOW_MEMORY)[m], ref[m])
    full = run_syrk(A, p, depth, flags=ffp.FFP_FILL_UPPER)
    assert np.array_equal(full, ref)
    C0 = inputs.uniform((81, p % 1000), n, n, p)
    for alpha, beta in ((p - 1, 1), ((p - 1) // 3, (p + 1) // 2)):
        alpha, beta = alpha % p, beta % p
        got = run_syrk(A, p, depth, alpha, beta, C0)
        assert np.array_equal(got[m], oracle.syrk_ab(A, p, alpha, beta, C0)[m]), (alpha, beta)


@pytest.mark.parametrize("p", BIG)
@pytest.mark.parametrize("depth", [0, 1])
def test_largest_magnitudes(p, depth):
    """Every entry p - 1 (centred to -(p-1)/2): the largest products; the
    closed form is k (p-1)^2 = k mod p."""
    n, k = 200, 1000
    A = np.full((n, k), p - 1, dtype=np.uint32)
    got = run_syrk(A, p, depth)
    m = lower_mask(n)
    assert np.all(got[m] == k % p)
    C0 = np.full((n, n), p - 1, dtype=np.uint32)
    got = run_syrk(A, p, depth, p - 1, p - 1, C0)
    assert np.all(got[m] == ((p - 1) * k + (p - 1) * (p - 1)) % p)


@pytest.mark.parametrize("p", [2] + BIG)
@pytest.mark.parametrize("m,n,k", [(300, 200, 333), (64, 64, 2000), (1, 7, 5)])
def test_gemm_extreme_primes(p, m, n, k):
    import torch
    A = inputs.uniform((82, p % 1000), m, k, p)
    B = inputs.uniform((83, p % 1000), n, k, p)
    C0 = inputs.uniform((84, p % 1000), m, n, p)
    alpha, beta = (p - 1) % p, (p // 2) % p
    Cd = to_dev_u32(C0)
    ffp.gemm(to_dev_u32(A), to_dev_u32(B), p, alpha, beta, C=Cd)
    torch.cuda.synchronize()
    assert np.array_equal(from_dev_u32(Cd), oracle.gemm(A, B, p, alpha, beta, C0))


@pytest.mark.parametrize("p", BIG)
@pytest.mark.parametrize("n", [1, 64, 65, 300])
def test_ldlt_extreme_primes(p, n):
    import torch
    S = inputs.symmetric((85, p % 1000, n), n, p)
    ref, rinfo = oracle.ldlt_packed(S, p)
    Sd = to_dev_u32(S)
    info = ffp.ldlt(Sd, p)
    torch.cuda.synchronize()
    assert int(info.item()) == rinfo
    if rinfo == 0:
        m = lower_mask(n)
        assert np.array_equal(from_dev_u32(Sd)[m], ref[m])


def test_batched_across_the_range():
    import torch
    specs = [(200, 150, 2), (130, 300, 33554467), (257, 100, 94906249), (96, 96, 251),
             (300, 200, 65537), (64, 129, 94906249)]
    jobs, keep, mats = [], [], []
    for j, (n, k, p) in enumerate(specs):
        A = inputs.uniform((86, j), n, k, p)
        Ad = to_dev_u32(A)
        Cd = torch.zeros((n, n), dtype=torch.int32, device="cuda")
        jobs.append(ffp.make_job(Ad, Cd, p))
        keep += [Ad, Cd]
        mats.append((A, p, Cd))
    ffp.fsyrk_modp_batched(jobs)
    torch.cuda.synchronize()
    for A, p, Cd in mats:
        m = lower_mask(A.shape[0])
        assert np.array_equal(from_dev_u32(Cd)[m], oracle.syrk(A, p)[m]), p


def test_out_of_range_primes_refused():
    import torch
    A = torch.zeros((8, 8), dtype=torch.int32, device="cuda")
    C = torch.zeros((8, 8), dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int64, device="cuda")
    for p in (94906297, 4294967291):
        with pytest.raises(ffp.FfpError) as e:
            ffp.fsyrk_modp(8, 8, p, A, 8, ffp.FFP_U32, 1, 0, C, 8)
        assert e.value.status == ffp.FFP_EPRIME
        with pytest.raises(ffp.FfpError) as e:
            ffp.fgemm_modp(8, 8, 8, p, A, 8, A, 8, 1, 0, C, 8)
        assert e.value.status == ffp.FFP_EPRIME
    with pytest.raises(ffp.FfpError) as e:     # LDL^T needs an odd prime
        ffp.fldlt_modp(8, 2, C, 8, info)
    assert e.value.status == ffp.FFP_EPRIME
