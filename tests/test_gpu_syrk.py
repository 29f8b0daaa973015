"""GPU parity: fsyrk_modp / fgemm_modp through the C-ABI against the oracle.

Bit-exact comparison (integer results).  Small cases compare every entry;
the full-size workloads compare sampled entries, which the oracle computes
one by one, plus symmetry and determinism properties.
"""
import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp, inputs
from tests.gpu_util import (centred_i8, from_dev_u32, limbs, lower_mask, product_launches, set_kblk,
                            set_knob, to_dev_u32)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    oracle.build(force=False)
    ffp.lib()
    yield
    set_kblk(0)


def gpu_syrk(A, p, depth=None, alpha=1, beta=0, C0=None, fill_upper=False, force_f64=False,
             a_dtype=ffp.FFP_U32, limb3=False):
    import torch
    n = A.shape[-2]
    if a_dtype == ffp.FFP_U32:
        Ad = to_dev_u32(A)
    elif a_dtype == ffp.FFP_I8_CENTERED:
        Ad = torch.from_numpy(centred_i8(A, p)).cuda()
    else:
        Ad = torch.from_numpy(limbs(A, p)).cuda()
    Cd = to_dev_u32(C0) if C0 is not None else torch.zeros((n, n), dtype=torch.int32, device="cuda")
    ffp.syrk(Ad, p, alpha, beta, Cd, depth=depth, fill_upper=fill_upper, a_dtype=a_dtype,
             force_f64=force_f64, limb3=limb3)
    torch.cuda.synchronize()
    return from_dev_u32(Cd)


def check_lower(out, expect):
    n = out.shape[0]
    low = lower_mask(n)
    bad = np.argwhere(low & (out != expect))
    assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[:3].tolist()}"


# ------------------------------------------------------------- base kernels

@pytest.mark.parametrize("p", [65537, 131071, 1000003, 33554393])
@pytest.mark.parametrize("m,n,k", [(16, 16, 4), (64, 64, 64), (100, 37, 129), (257, 130, 300)])
def test_gemm_f64_vs_oracle(p, m, n, k):
    import torch
    rng = np.random.default_rng(m * 7 + n + k)
    A = rng.integers(0, p, size=(m, k), dtype=np.uint64).astype(np.uint32)
    B = rng.integers(0, p, size=(n, k), dtype=np.uint64).astype(np.uint32)
    C = rng.integers(0, p, size=(m, n), dtype=np.uint64).astype(np.uint32)
    alpha, beta = int(rng.integers(0, p)), int(rng.integers(0, p))
    Cd = to_dev_u32(C)
    ffp.gemm(to_dev_u32(A), to_dev_u32(B), p, alpha, beta, Cd)
    torch.cuda.synchronize()
    assert np.array_equal(from_dev_u32(Cd), oracle.gemm(A, B, p, alpha, beta, C))


@pytest.mark.parametrize("p", [65537, 131071])
@pytest.mark.parametrize("n,k", [(1, 1), (15, 7), (64, 64), (200, 333), (513, 64)])
def test_syrk_depth0_f64(p, n, k):
    A = inputs.uniform(n + k, n, k, p)
    check_lower(gpu_syrk(A, p, depth=0), oracle.syrk(A, p))


def test_gemm_and_syrk_all_max_entries():
    # all entries p-1: centred -1, every partial sum exact; with a forced
    # k-block of 16 the delayed reduction runs many times.
    p = 131071
    for kb in (0, 16, 48):
        set_kblk(kb)
        A = np.full((70, 1000), p - 1, dtype=np.uint32)
        check_lower(gpu_syrk(A, p, depth=0), oracle.syrk(A, p))
    set_kblk(0)


# -------------------------------------------------------- Algorithm 2 (F64)

@pytest.mark.parametrize("p", [65537, 131071, 1000003])
@pytest.mark.parametrize("depth", [1, 2, 3])
@pytest.mark.parametrize("n,k", [(256, 256), (320, 96), (96, 320), (301, 199)])
def test_syrk_recursive_f64(p, depth, n, k):
    A = inputs.uniform(depth * 100 + n, n, k, p)
    check_lower(gpu_syrk(A, p, depth=depth), oracle.syrk(A, p))


@pytest.mark.parametrize("p", [65537, 131071])
@pytest.mark.parametrize("depth", [0, 1, 2])
def test_syrk_alpha_beta_f64(p, depth):
    n, k = 192, 160
    A = inputs.uniform(11, n, k, p)
    C0 = inputs.uniform(12, n, n, p)
    for alpha, beta in [(p - 1, 1), (5, 7), (1, 0), (3, 0)]:
        out = gpu_syrk(A, p, depth=depth, alpha=alpha, beta=beta, C0=C0)
        check_lower(out, oracle.syrk_ab(A, p, alpha, beta, C0))


def test_config_small_512_p65537_depth1_full_symmetric():
    # 512 x 512, p = 65537, one level of recursion, symmetric output.
    p = 65537
    A = inputs.uniform(0, 512, 512, p)
    out = gpu_syrk(A, p, depth=1, fill_upper=True)
    assert np.array_equal(out, oracle.syrk(A, p))


def test_determinism():
    p = 131071
    A = inputs.uniform(5, 384, 384, p)
    a = gpu_syrk(A, p, depth=2)
    b = gpu_syrk(A, p, depth=2)
    low = lower_mask(384)
    assert np.array_equal(a[low], b[low])


@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("n,k,depth", [(300, 257, 0), (640, 640, 1), (130, 1000, 0)])
def test_f64_tile_variants(tile, n, k, depth):
    p = 131071
    A = inputs.uniform(n + k + tile, n, k, p)
    set_knob("f64_tile", tile)
    try:
        check_lower(gpu_syrk(A, p, depth=depth), oracle.syrk(A, p))
        C0 = inputs.uniform(5, n, n, p)
        check_lower(gpu_syrk(A, p, depth=depth, alpha=7, beta=p - 2, C0=C0),
                    oracle.syrk_ab(A, p, 7, p - 2, C0))
    finally:
        set_knob("f64_tile", 0)


@pytest.mark.parametrize("pipe", [1, 0])
@pytest.mark.parametrize("n,k,depth", [(300, 100, 0), (513, 64, 0), (256, 96, 0), (640, 640, 1),
                                       (130, 1000, 0), (1100, 2052, 0), (300, 257, 0), (384, 32, 1)])
def test_f64_pipe_variant(pipe, n, k, depth):
    """128 x 128 FP64 tiles of 8 waves with the operands as doubles in LDS
    (the default) or as centred int32: partial last k-stage, odd and even
    stage counts, partial panels, general products at depth 1, a k that is
    not a multiple of 4 (the int32 kernel runs) and k past the exact block
    (likewise)."""
    p = 131071
    A = inputs.uniform(n + 3 * k + pipe, n, k, p)
    set_knob("f64_tile", 128)
    set_knob("f64_pipe", pipe)
    try:
        check_lower(gpu_syrk(A, p, depth=depth), oracle.syrk(A, p))
        C0 = inputs.uniform(10, n, n, p)
        check_lower(gpu_syrk(A, p, depth=depth, alpha=7, beta=p - 2, C0=C0),
                    oracle.syrk_ab(A, p, 7, p - 2, C0))
        set_kblk(64)       # exact blocks shorter than k: reductions inside the k-loop
        check_lower(gpu_syrk(A, p, depth=depth, alpha=p - 1, beta=1, C0=C0),
                    oracle.syrk_ab(A, p, p - 1, 1, C0))
    finally:
        set_kblk(0)
        set_knob("f64_pipe", 1)
        set_knob("f64_tile", 0)


@pytest.mark.parametrize("pipe", [1, 0])
@pytest.mark.parametrize("n,k,dtype", [(300, 256, "limb2"), (513, 128, "u32"), (256, 384, "limb2"),
                                       (1000, 640, "u32"), (130, 1000, "u32"), (700, 2048, "limb2")])
def test_limb2_pipe_variant(pipe, n, k, dtype):
    """Two int8 limbs on 128 x 128 tiles with 128-byte k stages, LDS writes
    between the MFMAs (the default) or 64-byte stages: limb operands given
    or packed from uint32, one, two and odd stage counts, partial panels,
    alpha/beta, entries at the ends of the range, k in chunks."""
    p = 65521
    A = inputs.uniform(n + 5 * k, n, k, p)
    A[:3] = p - 1
    A[3:5] = (p - 1) // 2
    a_dtype = ffp.FFP_I8_LIMB2 if dtype == "limb2" else ffp.FFP_U32
    set_knob("i8_dma", 0)
    set_knob("i8_pipe", pipe)
    try:
        check_lower(gpu_syrk(A, p, depth=0, a_dtype=a_dtype), oracle.syrk(A, p))
        C0 = inputs.uniform(11, n, n, p)
        check_lower(gpu_syrk(A, p, depth=0, alpha=p - 1, beta=1, C0=C0, a_dtype=a_dtype),
                    oracle.syrk_ab(A, p, p - 1, 1, C0))
        set_kblk(192)      # chunks of whole 128-byte stages
        check_lower(gpu_syrk(A, p, depth=0, alpha=3, beta=5, C0=C0, a_dtype=a_dtype),
                    oracle.syrk_ab(A, p, 3, 5, C0))
    finally:
        set_kblk(0)
        set_knob("i8_pipe", 1)
        set_knob("i8_dma", 1)


@pytest.mark.parametrize("p", [65537, 131071])
@pytest.mark.parametrize("n,k,depth", [(1024, 1024, 1), (1000, 1500, 2), (768, 2048, 3)])
def test_winograd_general_products(p, n, k, depth):
    """P3 and P4 through one level of Strassen-Winograd (threshold lowered to
    256 so that these sizes take it), with alpha; bit-exact."""
    A = inputs.uniform(n + k + depth, n, k, p)
    set_knob("winograd_min", 256)
    try:
        check_lower(gpu_syrk(A, p, depth=depth), oracle.syrk(A, p))
        check_lower(gpu_syrk(A, p, depth=depth, alpha=p - 1, beta=0),
                    oracle.syrk_ab(A, p, p - 1, 0, np.zeros((n, n), np.uint32)))
    finally:
        set_knob("winograd_min", 0)


@pytest.mark.parametrize("vec", [1, 0])
@pytest.mark.parametrize("p,limb3,depth", [(251, False, 0), (65521, False, 0), (131071, True, 0),
                                           (251, False, 1), (65537, False, 2)])
@pytest.mark.parametrize("n,k,pad", [(37, 70, 0), (300, 257, 3), (130, 1000, 1), (256, 512, 0),
                                     (1040, 1030, 1), (1030, 1024, 0)])
def test_pack_paths(vec, p, limb3, depth, n, k, pad):
    """Representation changes from uint32 (int8, two and three limbs, FP64
    padding): 4 columns per thread or one (single packs of at least 256
    workgroups of 16 x 256 take the former), with aligned and unaligned
    source rows (lda = k + pad) and ragged n and k."""
    import torch
    A = inputs.uniform(n * 7 + k + pad, n, k, p)
    full = np.zeros((n, k + pad), dtype=np.uint32)
    full[:, :k] = A
    Ad = to_dev_u32(full)[:, :k]
    C = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    set_knob("pack_vec", vec)
    try:
        ffp.syrk(Ad, p, C=C, depth=depth, limb3=limb3)
        torch.cuda.synchronize()
        check_lower(from_dev_u32(C), oracle.syrk(A, p))
    finally:
        set_knob("pack_vec", 1)


# ------------------------------------------------------------- int8 paths

@pytest.mark.parametrize("tile", [128, 256])
@pytest.mark.parametrize("n,k", [(300, 256), (600, 192), (513, 64)])
def test_i8_tile_variants(tile, n, k):
    p = 251
    A = inputs.uniform(n + tile, n, k, p)
    set_knob("i8_tile", tile)
    try:
        check_lower(gpu_syrk(A, p, depth=0, a_dtype=ffp.FFP_I8_CENTERED), oracle.syrk(A, p))
        C0 = inputs.uniform(6, n, n, p)
        check_lower(gpu_syrk(A, p, depth=0, alpha=3, beta=5, C0=C0), oracle.syrk_ab(A, p, 3, 5, C0))
    finally:
        set_knob("i8_tile", 0)


@pytest.mark.parametrize("n,k,dtype", [(300, 256, "limb2"), (513, 128, "u32"), (256, 384, "limb2"),
                                       (1000, 640, "u32"), (130, 1000, "u32"), (700, 2048, "limb2")])
def test_limb2_dma_variant(n, k, dtype):
    """Two int8 limbs on 128 x 128 tiles with operands straight to LDS (the
    default): limb operands given or packed from uint32, one, two and odd
    stage counts, partial panels, alpha/beta, entries at the ends of the
    range, k in chunks."""
    p = 65521
    A = inputs.uniform(n + 3 * k, n, k, p)
    A[:3] = p - 1
    A[3:5] = (p - 1) // 2
    a_dtype = ffp.FFP_I8_LIMB2 if dtype == "limb2" else ffp.FFP_U32
    check_lower(gpu_syrk(A, p, depth=0, a_dtype=a_dtype), oracle.syrk(A, p))
    C0 = inputs.uniform(12, n, n, p)
    check_lower(gpu_syrk(A, p, depth=0, alpha=p - 1, beta=1, C0=C0, a_dtype=a_dtype),
                oracle.syrk_ab(A, p, p - 1, 1, C0))
    set_kblk(384)      # chunks of whole 128-byte stages
    try:
        check_lower(gpu_syrk(A, p, depth=0, alpha=3, beta=5, C0=C0, a_dtype=a_dtype),
                    oracle.syrk_ab(A, p, 3, 5, C0))
        check_lower(gpu_syrk(A, p, depth=1), oracle.syrk(A, p))
    finally:
        set_kblk(0)


@pytest.mark.parametrize("n,k,depth", [(6000, 1024, 0), (5000, 640, 0), (6000, 2048, 1)])
def test_i8_split_tail_round(n, k, depth):
    """int8 products whose last round of 256 x 256 tiles is short: that
    round's tiles run as k-chunks (int32 sums in scratch) added by a second
    kernel; partial panels, alpha/beta, against the split switched off and
    the oracle."""
    p = 251
    A = inputs.uniform((46, n, k), n, k, p)
    C0 = inputs.uniform(47, n, n, p)
    want = oracle.syrk_ab(A, p, 3, 5, C0)
    check_lower(gpu_syrk(A, p, depth=depth, alpha=3, beta=5, C0=C0, a_dtype=ffp.FFP_I8_CENTERED), want)
    set_knob("i8_split_tail", 0)
    try:
        check_lower(gpu_syrk(A, p, depth=depth, alpha=3, beta=5, C0=C0, a_dtype=ffp.FFP_I8_CENTERED), want)
    finally:
        set_knob("i8_split_tail", 1)
    check_lower(gpu_syrk(A, p, depth=depth), oracle.syrk(A, p))


@pytest.mark.parametrize("dma", [1, 0])
@pytest.mark.parametrize("n,k", [(300, 256), (513, 128), (1000, 384), (1100, 4096), (256, 128), (600, 1280)])
def test_i8_dma_variants(dma, n, k):
    """256 x 256 int8 tiles with operands loaded straight into LDS (the
    default) or through registers: one, odd and even stage counts, partial
    panels, alpha/beta, k in chunks accumulated through C."""
    p = 251
    A = inputs.uniform(n + 7 * dma + k, n, k, p)
    A[:2] = p - 1
    A[2:4] = (p + 1) // 2
    set_knob("i8_tile", 256)
    set_knob("i8_dma", dma)
    try:
        check_lower(gpu_syrk(A, p, depth=0, a_dtype=ffp.FFP_I8_CENTERED), oracle.syrk(A, p))
        C0 = inputs.uniform(8, n, n, p)
        check_lower(gpu_syrk(A, p, depth=0, alpha=3, beta=5, C0=C0), oracle.syrk_ab(A, p, 3, 5, C0))
        set_kblk(256)      # k in chunks of two stages, accumulated through C
        check_lower(gpu_syrk(A, p, depth=1, alpha=p - 1, beta=1, C0=C0),
                    oracle.syrk_ab(A, p, p - 1, 1, C0))
    finally:
        set_kblk(0)
        set_knob("i8_dma", 1)
        set_knob("i8_tile", 0)


@pytest.mark.parametrize("pipe", [1, 0])
@pytest.mark.parametrize("n,k", [(300, 256), (513, 128), (512, 384), (1000, 640), (1100, 4096), (256, 128)])
def test_i8_pipe_variant(pipe, n, k):
    """256 x 256 int8 tiles with 128-byte k stages, with the LDS writes
    between the MFMAs and the loads two stages ahead (the default) or after
    them: one, two and an odd number of k-stages, partial and full panels,
    general products (depth 1) and k in chunks."""
    p = 251
    A = inputs.uniform(n + k + 11, n, k, p)
    set_knob("i8_tile", 256)
    set_knob("i8_dma", 0)
    set_knob("i8_pipe", pipe)
    try:
        check_lower(gpu_syrk(A, p, depth=0, a_dtype=ffp.FFP_I8_CENTERED), oracle.syrk(A, p))
        C0 = inputs.uniform(9, n, n, p)
        check_lower(gpu_syrk(A, p, depth=0, alpha=3, beta=5, C0=C0), oracle.syrk_ab(A, p, 3, 5, C0))
        if k % 256 == 0:
            check_lower(gpu_syrk(A, p, depth=1, alpha=p - 1, beta=1, C0=C0),
                        oracle.syrk_ab(A, p, p - 1, 1, C0))
            set_kblk(256)      # k in chunks of two stages, accumulated through C
            check_lower(gpu_syrk(A, p, depth=0, alpha=p - 1, beta=1, C0=C0),
                        oracle.syrk_ab(A, p, p - 1, 1, C0))
        # a block length that is a multiple of 64 but not of 128: the chunks
        # of the 128-byte-stage kernel stay whole stages
        set_kblk(192)
        check_lower(gpu_syrk(A, p, depth=0, alpha=2, beta=3, C0=C0), oracle.syrk_ab(A, p, 2, 3, C0))
    finally:
        set_kblk(0)
        set_knob("i8_pipe", 1)
        set_knob("i8_dma", 1)
        set_knob("i8_tile", 0)


@pytest.mark.parametrize("p,a_dtype", [(251, ffp.FFP_U32), (251, ffp.FFP_I8_CENTERED),
                                       (65521, ffp.FFP_U32), (65521, ffp.FFP_I8_LIMB2),
                                       (257, ffp.FFP_U32)])
@pytest.mark.parametrize("depth", [0, 1, 2])
@pytest.mark.parametrize("n,k", [(256, 256), (200, 130), (130, 600)])
def test_syrk_int8_paths(p, a_dtype, depth, n, k):
    A = inputs.uniform(3 * n + k + depth, n, k, p)
    check_lower(gpu_syrk(A, p, depth=depth, a_dtype=a_dtype), oracle.syrk(A, p))


@pytest.mark.parametrize("p", [251, 65521])
def test_int8_alpha_beta_and_forced_kblk(p):
    n, k = 160, 1024
    A = inputs.uniform(21, n, k, p)
    C0 = inputs.uniform(22, n, n, p)
    set_kblk(64)
    out = gpu_syrk(A, p, depth=1, alpha=p - 1, beta=1, C0=C0)
    set_kblk(0)
    check_lower(out, oracle.syrk_ab(A, p, p - 1, 1, C0))


def test_int8_max_entries():
    for p in (251, 65521):
        A = np.full((96, 4096), (p - 1) // 2 + 1, dtype=np.uint32)   # most negative centred value
        check_lower(gpu_syrk(A, p, depth=0), oracle.syrk(A, p))


@pytest.mark.parametrize("p", [65537, 131071, 1000003, 8388593])
@pytest.mark.parametrize("n,k", [(1, 1), (100, 37), (257, 300), (513, 64), (300, 1000)])
def test_syrk_limb3_vs_oracle(p, n, k):
    """Three int8 limbs: ragged shapes over several 128 x 128 tiles, p up to
    the largest prime below 2^23."""
    A = inputs.uniform((41, n, k, p), n, k, p)
    check_lower(gpu_syrk(A, p, limb3=True), oracle.syrk(A, p))


@pytest.mark.parametrize("p", [65537, 131071, 8388593])
@pytest.mark.parametrize("depth", [1, 2, 3])
@pytest.mark.parametrize("n,k", [(256, 256), (300, 1000), (1000, 640), (1030, 2100)])
def test_limb3_recursive(p, depth, n, k):
    """Algorithm 2 over three int8 limbs: the pre-additions in the limb
    planes (16 columns per thread where aligned), plain and accumulate
    forms, wide and Table 3 placements."""
    A = inputs.uniform((43, n, k, p, depth), n, k, p)
    check_lower(gpu_syrk(A, p, depth=depth, limb3=True), oracle.syrk(A, p))
    C0 = inputs.uniform(44, n, n, p)
    check_lower(gpu_syrk(A, p, depth=depth, alpha=p - 1, beta=1, C0=C0, limb3=True),
                oracle.syrk_ab(A, p, p - 1, 1, C0))
    set_knob("wide", 0)
    try:
        check_lower(gpu_syrk(A, p, depth=depth, limb3=True), oracle.syrk(A, p))
    finally:
        set_knob("wide", 1)


@pytest.mark.parametrize("p", [131071, 8388593])
@pytest.mark.parametrize("n,k,depth", [(300, 256, 0), (513, 128, 0), (130, 384, 0), (1000, 1024, 0),
                                       (700, 2048, 1), (1030, 1280, 2)])
def test_limb3_dma_variant(p, n, k, depth):
    """Three int8 limbs on 128 x 64 tiles with operands straight to LDS
    (forced for every k that is a multiple of 128): partial tiles, one and
    odd stage counts, general products of the recursion, alpha/beta, the
    upper fill, k in chunks of whole stages; against the oracle."""
    A = inputs.uniform((48, n, k, p), n, k, p)
    A[:2] = (p - 1) // 2 + 1              # most negative centred value
    A[2:4] = (p - 1) // 2                 # most positive
    C0 = inputs.uniform(49, n, n, p)
    set_knob("l3_dma", 2)
    try:
        check_lower(gpu_syrk(A, p, depth=depth, limb3=True), oracle.syrk(A, p))
        out = gpu_syrk(A, p, depth=depth, alpha=p - 1, beta=1, C0=C0, limb3=True, fill_upper=True)
        check_lower(out, oracle.syrk_ab(A, p, p - 1, 1, C0))
        assert np.array_equal(out, np.tril(out) + np.tril(out, -1).T)
        set_kblk(128)
        try:
            check_lower(gpu_syrk(A, p, depth=depth, alpha=3, beta=5, C0=C0, limb3=True),
                        oracle.syrk_ab(A, p, 3, 5, C0))
        finally:
            set_kblk(0)
    finally:
        set_knob("l3_dma", 1)


def test_limb3_dma_long_k():
    """Largest centred magnitudes over more columns than one exact int32
    block, so the product runs as three k-chunks, each a whole number of
    128-byte stages, on the direct-to-LDS three-limb tile."""
    p = 8388593
    n, k = 130, 2 * 43648
    A = np.full((n, k), (p - 1) // 2 + 1, dtype=np.uint32)
    A[::3] = (p - 1) // 2
    set_knob("l3_dma", 2)
    try:
        check_lower(gpu_syrk(A, p, limb3=True), oracle.syrk(A, p))
    finally:
        set_knob("l3_dma", 1)


@pytest.mark.parametrize("vec", [1, 0])
@pytest.mark.parametrize("p,a_dtype", [(251, ffp.FFP_U32), (251, ffp.FFP_I8_CENTERED), (65521, ffp.FFP_U32),
                                       (65521, ffp.FFP_I8_LIMB2), (3, ffp.FFP_U32), (257, ffp.FFP_U32)])
@pytest.mark.parametrize("depth", [1, 2])
def test_int8_preadditions_vector_or_scalar(vec, p, a_dtype, depth):
    """The int8-class pre-additions 16 columns per thread (where aligned) or
    one: both against the oracle, p = 3 (y = 2) and 257 (y = 1) included."""
    n, k = 600, 1024
    A = inputs.uniform((45, p, depth), n, k, p)
    set_knob("pack_vec", vec)
    try:
        check_lower(gpu_syrk(A, p, depth=depth, a_dtype=a_dtype), oracle.syrk(A, p))
    finally:
        set_knob("pack_vec", 1)


@pytest.mark.parametrize("p", [65537, 8388593])
def test_limb3_alpha_beta_fill_and_forced_kblk(p):
    n, k = 200, 1100
    A = inputs.uniform(42, n, k, p)
    C0 = inputs.uniform(43, n, n, p)
    out = gpu_syrk(A, p, alpha=p - 1, beta=1, C0=C0, limb3=True, fill_upper=True)
    expect = oracle.syrk_ab(A, p, p - 1, 1, C0)
    check_lower(out, expect)
    assert np.array_equal(out, np.tril(out) + np.tril(out, -1).T)
    set_kblk(64)                          # every 64 columns a reduction and a new launch
    out = gpu_syrk(A, p, alpha=3, beta=p - 2, C0=C0, limb3=True)
    set_kblk(0)
    check_lower(out, oracle.syrk_ab(A, p, 3, p - 2, C0))


@pytest.mark.parametrize("kblk", [64, 128, 192, 320])
@pytest.mark.parametrize("n,k", [(130, 640), (257, 1100)])
def test_limb3_small_tile_stage_counts(kblk, n, k):
    """The 64 x 64 three-limb tile, whose second register set loads each
    stage two stages ahead: one, two and odd numbers of 64-byte stages per
    launch (k in chunks of kblk), partial tiles, alpha/beta; against the
    oracle."""
    p = 131071
    A = inputs.uniform((63, n, k), n, k, p)
    C0 = inputs.uniform(64, n, n, p)
    set_kblk(kblk)
    try:
        check_lower(gpu_syrk(A, p, depth=0, alpha=5, beta=7, C0=C0, limb3=True), oracle.syrk_ab(A, p, 5, 7, C0))
    finally:
        set_kblk(0)


def test_limb3_max_entries_long_k():
    """Largest centred magnitudes over more columns than one exact int32
    block (43 648), so the product runs as two k-chunks."""
    for p in (131071, 8388593):
        n, k = 64, 50000
        A = np.full((n, k), (p - 1) // 2 + 1, dtype=np.uint32)   # most negative centred value
        A[::3] = (p - 1) // 2                                     # most positive
        check_lower(gpu_syrk(A, p, limb3=True), oracle.syrk(A, p))


def test_f64_forced_for_small_prime():
    p = 251
    A = inputs.uniform(31, 200, 300, p)
    check_lower(gpu_syrk(A, p, depth=2, force_f64=True), oracle.syrk(A, p))


# ----------------------------------------------------- argument validation

def test_argument_errors():
    import torch
    A = torch.zeros((4, 4), dtype=torch.int32, device="cuda")
    C = torch.zeros((4, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(ffp.FfpError) as e:
        ffp.fsyrk_modp(4, 4, 65535, A, 4, ffp.FFP_U32, 1, 0, C, 4)   # not prime
    assert e.value.status == ffp.FFP_EPRIME
    with pytest.raises(ffp.FfpError) as e:
        ffp.fsyrk_modp(4, 4, 65537, A, 3, ffp.FFP_U32, 1, 0, C, 4)   # lda < k
    assert e.value.status == ffp.FFP_EINVAL
    with pytest.raises(ffp.FfpError) as e:
        ffp.fsyrk_modp(4, 4, 65537, A, 4, ffp.FFP_I8_CENTERED, 1, 0, C, 4)  # int8 needs p <= 251
    assert e.value.status == ffp.FFP_EDTYPE
    with pytest.raises(ffp.FfpError) as e:
        ffp.fsyrk_modp(4, 4, 65537, A, 4, ffp.FFP_U32, 65537, 0, C, 4)   # alpha >= p
    assert e.value.status == ffp.FFP_EINVAL
    assert ffp.fsyrk_modp(0, 4, 65537, A, 4, ffp.FFP_U32, 1, 0, C, 4) == 0


# ------------------------------------------------------ full-size workloads

def _sampled(A, p, out, tile=128, per_tile=2, seed=0):
    """Entries of every lower tile of edge `tile` of the output against the
    oracle: its four corners (those on or below the diagonal), two random
    entries below the diagonal and, on diagonal tiles, two diagonal entries."""
    n = A.shape[0]
    rng = np.random.default_rng(seed)
    nt = (n + tile - 1) // tile
    rows, cols = [], []
    for ti in range(nt):
        r0, r1 = ti * tile, min(n, ti * tile + tile) - 1
        for tj in range(ti + 1):
            c0, c1 = tj * tile, min(n, tj * tile + tile) - 1
            for r, c in ((r0, c0), (r1, c0), (r0, c1), (r1, c1)):
                if c <= r:
                    rows.append(r)
                    cols.append(c)
            rr = rng.integers(r0, r1 + 1, size=per_tile)
            cc = rng.integers(c0, c1 + 1, size=per_tile)
            rows.extend(np.maximum(rr, cc))
            cols.extend(np.minimum(rr, cc))
            if ti == tj:
                d = rng.integers(r0, r1 + 1, size=2)
                rows.extend(d)
                cols.extend(d)
    lo = np.asarray(rows, dtype=np.int64)
    hi = np.asarray(cols, dtype=np.int64)
    expect = oracle.syrk_entries(A, p, lo, hi)
    got = out[lo, hi]
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("wide", [0, 1])
@pytest.mark.parametrize("p,depth", [(131071, 1), (131071, 3), (65537, 2), (1000003, 2)])
@pytest.mark.parametrize("n,k", [(256, 256), (300, 1000), (520, 130)])
def test_syrk_level_scheduler(wide, p, depth, n, k):
    """Independent products grouped per level (and the wide placements)."""
    A = inputs.uniform(n + 3 * k + depth, n, k, p)
    set_knob("wide", wide)
    try:
        check_lower(gpu_syrk(A, p, depth=depth), oracle.syrk(A, p))
        C0 = inputs.uniform(9, n, n, p)
        check_lower(gpu_syrk(A, p, depth=depth, alpha=3, beta=p - 2, C0=C0),
                    oracle.syrk_ab(A, p, 3, p - 2, C0))
    finally:
        set_knob("wide", 1)


def test_program_order_execution_matches():
    p, n, k = 131071, 384, 512
    A = inputs.uniform(44, n, k, p)
    set_knob("leveled", 0)
    try:
        seq = gpu_syrk(A, p, depth=2)
    finally:
        set_knob("leveled", 1)
    check_lower(seq, oracle.syrk(A, p))
    check_lower(gpu_syrk(A, p, depth=2), seq)


@pytest.mark.parametrize("wide", [0, 1])
@pytest.mark.parametrize("k", [8192, 32768])
def test_full_size_8192_p131071_depth3(k, wide):
    import torch
    p, n = 131071, 8192
    A = inputs.uniform(1, n, k, p)
    Ad = to_dev_u32(A)
    Cd = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    set_knob("wide", wide)
    try:
        ffp.syrk(Ad, p, C=Cd, depth=3)
        torch.cuda.synchronize()
    finally:
        set_knob("wide", 1)
    _sampled(A, p, from_dev_u32(Cd))


@pytest.mark.parametrize("k", [8192, 32768])
def test_full_size_8192_p131071_three_limbs(k):
    """The depth-3 workload's shapes on three int8 limbs (as bench.py's
    syrk_8192_p131071_limb3): sampled entries against the oracle."""
    import torch
    p, n = 131071, 8192
    A = inputs.uniform(1, n, k, p)
    Cd = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    ffp.syrk(to_dev_u32(A), p, C=Cd, limb3=True)
    torch.cuda.synchronize()
    _sampled(A, p, from_dev_u32(Cd))


@pytest.mark.parametrize("depth", [0, 1])
def test_three_limbs_planes_near_offset_limit(depth):
    """16384 x 32768, p = 8388593 on three limbs: limb planes of 2^29 bytes,
    so that a panel's three planes in one buffer resource reach 2^30 + 2^22
    bytes of offset; the direct-to-LDS tile must run (kernel variant 14)
    and every 128 x 128 output tile is sampled against the oracle."""
    import torch
    p, n, k = 8388593, 16384, 32768
    A = inputs.uniform((60, depth), n, k, p)
    A[:64] = (p - 1) // 2 + 1             # most negative centred value
    A[-64:] = (p - 1) // 2                # most positive
    Ad = to_dev_u32(A)
    Cd = torch.zeros((n, n), dtype=torch.int32, device="cuda")

    def run():
        ffp.syrk(Ad, p, C=Cd, depth=depth, limb3=True)
        torch.cuda.synchronize()
    assert product_launches(run, variant=14) > 0
    del Ad
    _sampled(A, p, from_dev_u32(Cd), per_tile=1, seed=depth)


@pytest.mark.parametrize("p,a_dtype,dma", [(251, ffp.FFP_I8_CENTERED, 1), (251, ffp.FFP_I8_CENTERED, 0),
                                           (65521, ffp.FFP_I8_LIMB2, 1), (65521, ffp.FFP_I8_LIMB2, 0)])
def test_full_size_16384_int8(p, a_dtype, dma):
    """The 16384^2 workloads in the launch configuration the benchmark
    times: every 256 x 256 output tile sampled against the oracle."""
    import torch
    n = 16384
    A = inputs.uniform(2, n, n, p)
    if a_dtype == ffp.FFP_I8_CENTERED:
        Ad = torch.from_numpy(centred_i8(A, p)).cuda()
    else:
        Ad = torch.from_numpy(limbs(A, p)).cuda()
    Cd = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    set_knob("i8_dma", dma)
    try:
        ffp.syrk(Ad, p, C=Cd, depth=0, a_dtype=a_dtype)
        torch.cuda.synchronize()
    finally:
        set_knob("i8_dma", 1)
    _sampled(A, p, from_dev_u32(Cd), tile=256 if p <= 251 else 128)
