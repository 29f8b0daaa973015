"""GPU parity of fsyrk_modp_batched: every job equals the oracle and is
bit-identical to the same job run alone through fsyrk_modp."""
import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp, inputs
from tests.gpu_util import from_dev_u32, lower_mask, set_knob, to_dev_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    oracle.build(force=False)
    ffp.lib()


def run_batch(specs, flags=0):
    """specs: list of (A, p, alpha, beta, C0).  Returns host results."""
    import torch
    devA, devC, jobs = [], [], []
    for A, p, alpha, beta, C0 in specs:
        Ad = to_dev_u32(A)
        Cd = to_dev_u32(C0)
        devA.append(Ad)
        devC.append(Cd)
        jobs.append(ffp.make_job(Ad, Cd, p, alpha, beta))
    ffp.fsyrk_modp_batched(jobs, flags)
    torch.cuda.synchronize()
    return [from_dev_u32(c) for c in devC]


def run_alone(A, p, alpha, beta, C0, flags=0):
    import torch
    Ad = to_dev_u32(A)
    Cd = to_dev_u32(C0)
    n, k = A.shape
    ffp.fsyrk_modp(n, k, p, Ad, k, ffp.FFP_U32, alpha, beta, Cd, n, flags)
    torch.cuda.synchronize()
    return from_dev_u32(Cd)


def mixed_specs(seed, count, nmax=300, primes=(251, 65521, 65537, 131071, 1000003)):
    rng = np.random.default_rng(seed)
    specs = []
    for j in range(count):
        n = int(rng.integers(1, nmax + 1))
        k = int(rng.integers(max(1, n // 2), 2 * n + 1))
        p = int(primes[int(rng.integers(0, len(primes)))])
        alpha = int(rng.integers(0, p)) if j % 3 else 1
        beta = int(rng.integers(0, p)) if j % 2 else 0
        A = inputs.uniform((seed, j), n, k, p)
        C0 = inputs.uniform((seed, j, 1), n, n, p)
        specs.append((A, p, alpha, beta, C0))
    return specs


@pytest.mark.parametrize("persistent", [2, 1, 0])
def test_batch_mixed_matches_oracle_and_alone(persistent):
    """Grouped launches with persistent workgroups (tiles dealt to the XCDs
    in chunks, or plain striding) or one workgroup per tile."""
    set_knob("persistent", persistent)
    try:
        specs = mixed_specs(10, 40)
        outs = run_batch(specs)
        for (A, p, alpha, beta, C0), out in zip(specs, outs):
            n = A.shape[0]
            low = lower_mask(n)
            expect = oracle.syrk_ab(A, p, alpha, beta, C0)
            assert np.array_equal(out[low], expect[low])
            alone = run_alone(A, p, alpha, beta, C0)
            assert np.array_equal(out[low], alone[low])
    finally:
        set_knob("persistent", 2)


@pytest.mark.parametrize("depth", [1, 2])
def test_batch_with_recursion(depth):
    specs = mixed_specs(11, 12, nmax=260, primes=(65537, 131071, 251))
    outs = run_batch(specs, flags=ffp.FFP_DEPTH(depth))
    for (A, p, alpha, beta, C0), out in zip(specs, outs):
        low = lower_mask(A.shape[0])
        assert np.array_equal(out[low], oracle.syrk_ab(A, p, alpha, beta, C0)[low])


def test_batch_fill_upper():
    specs = mixed_specs(12, 10, nmax=120)
    outs = run_batch(specs, flags=ffp.FFP_FILL_UPPER)
    for (A, p, alpha, beta, C0), out in zip(specs, outs):
        full = oracle.syrk_ab(A, p, alpha, beta, C0)
        low = np.tril(full)
        assert np.array_equal(out, low + np.tril(low, -1).T)


def test_batch_empty_and_zero_sized():
    import torch
    assert ffp.fsyrk_modp_batched([]) == 0
    A = torch.zeros((0, 4), dtype=torch.int32, device="cuda")
    C = torch.zeros((0, 0), dtype=torch.int32, device="cuda")
    job = ffp.ffp_job(n=0, k=4, p=65537, alpha=1, beta=0, a_dtype=0, A=A.data_ptr(), lda=4,
                      C=C.data_ptr(), ldc=1)
    assert ffp.fsyrk_modp_batched([job]) == 0


def test_batch_rejects_bad_job_before_enqueue():
    import torch
    specs = mixed_specs(13, 3, nmax=50)
    devA = [to_dev_u32(s[0]) for s in specs]
    devC = [torch.full((s[0].shape[0],) * 2, 7, dtype=torch.int32, device="cuda") for s in specs]
    jobs = [ffp.make_job(a, c, s[1]) for a, c, s in zip(devA, devC, specs)]
    jobs[2].p = 65535      # not prime
    with pytest.raises(ffp.FfpError) as e:
        ffp.fsyrk_modp_batched(jobs)
    assert e.value.status == ffp.FFP_EPRIME
    torch.cuda.synchronize()
    for c in devC:
        assert int((c != 7).sum().item()) == 0     # nothing ran


def test_batch_workload_1024_jobs_all_checked():
    """1024 jobs, n ~ U[32,1024], k ~ U[n/2,2n], p ~ U{251, 65537, 131071},
    seed 3: every job's lower triangle against the oracle."""
    import torch
    shapes = inputs.batch_jobs(3)
    devA, devC, jobs, mats = [], [], [], []
    for j, (n, k, p) in enumerate(shapes):
        A = inputs.batch_matrix(3, j, n, k, p)
        mats.append(A)
        Ad = to_dev_u32(A)
        Cd = torch.zeros((n, n), dtype=torch.int32, device="cuda")
        devA.append(Ad)
        devC.append(Cd)
        jobs.append(ffp.make_job(Ad, Cd, p))
    ffp.fsyrk_modp_batched(jobs)
    torch.cuda.synchronize()
    for j, ((n, k, p), A, Cd) in enumerate(zip(shapes, mats, devC)):
        out = from_dev_u32(Cd)
        rows = oracle.syrk_rows(A, p, 0, n)
        low = lower_mask(n)
        assert np.array_equal(out[low], rows[low]), j


def test_batch_three_limb_base():
    """FFP_BASE_LIMB3 for a whole batch (primes up to 1000003 and the int8
    ones): grouped three-limb products, each job exact."""
    specs = mixed_specs(14, 24, nmax=260)
    outs = run_batch(specs, flags=ffp.FFP_BASE_LIMB3)
    for (A, p, alpha, beta, C0), out in zip(specs, outs):
        low = lower_mask(A.shape[0])
        assert np.array_equal(out[low], oracle.syrk_ab(A, p, alpha, beta, C0)[low])
