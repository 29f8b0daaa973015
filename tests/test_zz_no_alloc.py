"""fsyrk_modp_noalloc (workspace in a static device buffer) against
fsyrk_modp and the oracle, through the C ABI: two calls in a row, the second
on a smaller input, then a shape whose workspace exceeds the buffer."""
import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp, inputs
from tests.gpu_util import from_dev_u32, lower_mask, to_dev_u32

pytestmark = pytest.mark.gpu


def _both(A, p, depth, alpha=1, beta=0, C0=None, flags=0):
    import torch
    n, k = A.shape
    Ad = to_dev_u32(A)
    outs = []
    for fn in (ffp.fsyrk_modp, ffp.fsyrk_modp_noalloc):
        Cd = to_dev_u32(C0) if C0 is not None else torch.zeros((n, n), dtype=torch.int32, device="cuda")
        fn(n, k, p, Ad, Ad.stride(0), ffp.FFP_U32, alpha, beta, Cd, Cd.stride(0),
           flags | ffp.FFP_DEPTH(depth))
        outs.append(Cd)
    torch.cuda.synchronize()
    return [from_dev_u32(c) for c in outs]


def test_noalloc_matches_fsyrk_twice_then_smaller():
    L = lower_mask
    # first call: k > n, depth 2 (the S blocks and P2 of the wide placements
    # live in the scratch buffer), FP64 class
    p = 131071
    A = inputs.uniform(70, 600, 900, p)
    ref, got = _both(A, p, 2)
    assert ffp.ffp_workspace_bytes(600, 900, p, ffp.FFP_U32, ffp.FFP_DEPTH(2)) > 0
    m = L(600)
    assert np.array_equal(got[m], ref[m])
    assert np.array_equal(got[m], oracle.syrk(A, p)[m])
    # second call, smaller input on another class (uint32 packed to int8 in
    # the scratch buffer), alpha/beta form: the buffer still holds the first
    # call's blocks
    p = 251
    A = inputs.uniform(71, 200, 333, p)
    C0 = inputs.uniform(72, 200, 200, p)
    ref, got = _both(A, p, 1, alpha=5, beta=7, C0=C0)
    m = L(200)
    assert np.array_equal(got[m], ref[m])
    assert np.array_equal(got[m], oracle.syrk_ab(A, p, 5, 7, C0)[m])


def test_noalloc_many_grouped_products_and_fill_upper():
    # depth 3 puts more than six products on one level: they run as several
    # launches with inline task tables
    p = 65537
    A = inputs.uniform(73, 512, 512, p)
    ref, got = _both(A, p, 3, flags=ffp.FFP_FILL_UPPER | ffp.FFP_BASE_F64)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, oracle.syrk(A, p))


def test_noalloc_three_limbs():
    # three int8 limbs packed into the scratch buffer, one level of
    # Algorithm 2, alpha/beta form
    p = 131071
    A = inputs.uniform(74, 520, 700, p)
    C0 = inputs.uniform(75, 520, 520, p)
    ref, got = _both(A, p, 1, alpha=3, beta=p - 1, C0=C0, flags=ffp.FFP_BASE_LIMB3)
    m = lower_mask(520)
    assert np.array_equal(got[m], ref[m])
    assert np.array_equal(got[m], oracle.syrk_ab(A, p, 3, p - 1, C0)[m])


def test_noalloc_rejects_workspace_beyond_scratch():
    import torch
    cap = ffp.ffp_noalloc_scratch_bytes()
    n, k, p = 4096, 16384, 131071
    assert ffp.ffp_workspace_bytes(n, k, p, ffp.FFP_U32, ffp.FFP_DEPTH(1)) > cap
    A = torch.zeros((n, k), dtype=torch.int32, device="cuda")
    C = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    with pytest.raises(ffp.FfpError) as e:
        ffp.fsyrk_modp_noalloc(n, k, p, A, k, ffp.FFP_U32, 1, 0, C, n, ffp.FFP_DEPTH(1))
    assert e.value.status == ffp.FFP_ENOMEM
    torch.cuda.synchronize()
    assert int(C.abs().sum().item()) == 0    # nothing was enqueued
