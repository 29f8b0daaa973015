"""GPU parity of fldlt_modp against the oracle's Crout LDL^T (bit-exact:
L and D are unique when every leading minor is nonzero)."""
import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp, inputs
from tests.gpu_util import from_dev_u32, product_launches, to_dev_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    oracle.build(force=False)
    ffp.lib()


def gpu_ldlt(S, p):
    import torch
    Sd = to_dev_u32(S)
    info = ffp.ldlt(Sd, p)
    torch.cuda.synchronize()
    return from_dev_u32(Sd), int(info.item())


def constructed(n, p, seed, zero_at=None):
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(0, p, size=(n, n), dtype=np.uint64), -1).astype(object)
    L[np.arange(n), np.arange(n)] = 1
    D = rng.integers(1, p, size=n).astype(object)
    if zero_at is not None:
        D[zero_at] = 0
    S = np.array((L * D).dot(L.T) % p, dtype=np.uint32)
    return L, D, S


def packed(L, D):
    n = len(D)
    out = np.array(np.tril(L, -1), dtype=np.uint32)
    out[np.arange(n), np.arange(n)] = np.array(D, dtype=np.uint32)
    return out


@pytest.mark.parametrize("p", [65537, 131071, 251, 65521, 1000003])
@pytest.mark.parametrize("n", [1, 5, 64, 65, 130, 300])
def test_ldlt_recovers_constructed(p, n):
    L, D, S = constructed(n, p, seed=n + p)
    out, info = gpu_ldlt(S, p)
    assert info == 0
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(out[low], packed(L, D)[low])


@pytest.mark.parametrize("n", [200, 700, 1500])
def test_ldlt_random_symmetric_vs_oracle(n):
    p = 65537
    S = inputs.symmetric(40 + n, n, p)
    ref, rinfo = oracle.ldlt_packed(S, p)
    out, info = gpu_ldlt(S, p)
    assert info == rinfo
    if info == 0:
        low = np.tril(np.ones((n, n), dtype=bool))
        assert np.array_equal(out[low], ref[low])


@pytest.mark.parametrize("where", [0, 1, 63, 64, 100, 250])
def test_ldlt_zero_pivot_reported(where):
    p, n = 65537, 256
    _, _, S = constructed(n, p, seed=where, zero_at=where)
    _, rinfo = oracle.ldlt_packed(S, p)
    assert rinfo == where + 1
    _, info = gpu_ldlt(S, p)
    assert info == where + 1


def test_ldlt_many_nonresidues_odd_count():
    # all pivots non-residues (3 is a non-residue mod 65537): Algorithm 4 on
    # every pair and an extra zero column when the count is odd
    p, n = 65537, 193
    rng = np.random.default_rng(3)
    L = np.tril(rng.integers(0, p, size=(n, n), dtype=np.uint64), -1).astype(object)
    L[np.arange(n), np.arange(n)] = 1
    D = np.array([3 * (i + 1) ** 2 % p for i in range(n)], dtype=object)
    S = np.array((L * D).dot(L.T) % p, dtype=np.uint32)
    out, info = gpu_ldlt(S, p)
    assert info == 0
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(out[low], packed(L, D)[low])


def test_ldlt_4096_sampled_reconstruction():
    p, n = 65537, 4096
    S = inputs.symmetric(77, n, p)
    out, info = gpu_ldlt(S, p)
    if info != 0:
        pytest.skip(f"drawn matrix has a zero pivot at {info} (probability about n/p)")
    L = np.tril(out.astype(np.int64), -1)
    L[np.arange(n), np.arange(n)] = 1
    D = out[np.arange(n), np.arange(n)].astype(np.int64)
    rng = np.random.default_rng(0)
    for _ in range(300):
        i, j = sorted(rng.integers(0, n, size=2))[::-1]
        m = min(i, j) + 1
        # (L D L^T)_ij = sum_l L_il D_l L_jl, exact with Python ints
        v = sum(int(L[i, l]) * int(D[l]) * int(L[j, l]) for l in range(m)) % p
        assert v == int(S[i, j]), (i, j)


def test_ldlt_batched_equals_alone_and_oracle():
    """fldlt_modp_batched: jobs of different order and prime (int8, limb and
    FP64 Schur updates), one with a zero pivot, each bit-identical to the
    job alone and to the oracle."""
    import torch
    specs = [(1, 65537), (64, 65537), (65, 131071), (130, 251), (300, 65521), (700, 65537),
             (256, 65537)]
    mats = []
    for i, (n, p) in enumerate(specs):
        if i == len(specs) - 1:
            _, _, S = constructed(n, p, seed=5, zero_at=100)
        else:
            S = inputs.symmetric(900 + i, n, p)
        mats.append(S)
    dev = [to_dev_u32(S) for S in mats]
    info = ffp.ldlt_batched(dev, [p for _, p in specs])
    torch.cuda.synchronize()
    infos = info.cpu().numpy()
    for (n, p), S, Sd, inf in zip(specs, mats, dev, infos):
        alone, ainfo = gpu_ldlt(S, p)
        ref, rinfo = oracle.ldlt_packed(S, p)
        assert inf == ainfo == rinfo, (n, p)
        if inf == 0:
            low = np.tril(np.ones((n, n), dtype=bool))
            out = from_dev_u32(Sd)
            assert np.array_equal(out[low], alone[low])
            assert np.array_equal(out[low], ref[low])
    assert infos[-1] == 101


@pytest.mark.parametrize("p", [65537, 131071, 251])
def test_ldlt_products_folded_or_launched_agree(p):
    """Three-limb Schur updates as steps of the per-level launch (the
    default) or through the product schedule's own launches: bit-identical
    results (an input with nonzero pivots: after a zero pivot the contents
    are unspecified)."""
    from tests.gpu_util import set_knob
    n = 700
    _, _, S = constructed(n, p, seed=960 + p % 7)
    outs = []
    for fold in (1, 0):
        set_knob("ldlt_fold", fold)
        try:
            outs.append(gpu_ldlt(S, p))
        finally:
            set_knob("ldlt_fold", 1)
    (a, ia), (b, ib) = outs
    assert ia == ib
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(a[low], b[low])
    ref, rinfo = oracle.ldlt_packed(S, p)
    assert ia == rinfo == 0
    assert np.array_equal(a[low], ref[low])


def _freivalds_ldlt(S, out, p, rounds=3, seed=0):
    """L D L^T x = S x mod p for random x (a wrong factorisation passes with
    probability at most p^-rounds); exact in int64 for p < 2^24, n <= 8192."""
    n = S.shape[0]
    L = np.tril(out.astype(np.int64), -1)
    L[np.arange(n), np.arange(n)] = 1
    D = out[np.arange(n), np.arange(n)].astype(np.int64)
    Sl = S.astype(np.int64)
    rng = np.random.default_rng(seed)
    for _ in range(rounds):
        x = rng.integers(0, p, size=n, dtype=np.int64)
        y = (L.T @ x) % p
        y = (D * y) % p
        z = (L @ y) % p
        assert np.array_equal(z, (Sl @ x) % p)


def _big_ldlt_case(n, p, seed0):
    for attempt in range(4):
        S = inputs.symmetric((seed0, attempt), n, p)
        out, info = gpu_ldlt(S, p)
        if info == 0:
            return S, out
    pytest.fail("no draw with a generic rank profile in 4 attempts")


def test_ldlt_schur_update_through_algorithm2():
    """n = 8192, p = 131071: the top Schur update (n2 = 4096, k = 4097
    padded) runs on three int8 limbs through one level of Algorithm 2, so
    its products are launched by that plan (updates at depth 0 are steps of
    the LDL^T kernel and launch none).  The leading 1024 x 1024 block of L
    and D (the factorisation of the leading block) against the oracle's
    Crout LDL^T; the whole factorisation by Freivalds' check of
    L D L^T = S."""
    p, n = 131071, 8192
    ffp.ffp_tune_clear()
    plan = ffp.plan_describe(4096, 4224, p, lda=4224, ldc=n, alpha=p - 1, beta=1, flags=ffp.FFP_BASE_LIMB3)
    assert " cls=3 " in plan.splitlines()[0]
    res = {}
    nl = product_launches(lambda: res.update(case=_big_ldlt_case(n, p, 51)), cls=3)
    assert nl > 0, "no three-limb product launched by a Schur update's plan"
    S, out = res["case"]
    m = 1024
    ref, rinfo = oracle.ldlt_packed(S[:m, :m].copy(), p)
    assert rinfo == 0
    low = np.tril(np.ones((m, m), dtype=bool))
    assert np.array_equal(out[:m, :m][low], ref[low])
    _freivalds_ldlt(S, out, p)


def test_ldlt_fp64_table4_schur_path():
    """p above 2^23: the Schur updates run on FP64 matrix cores through the
    Table 4 schedule (alpha = p - 1, beta = 1) at depth 1 for the top node
    of n = 4096 (n2 = 2048)."""
    p = (1 << 23) + 1
    while not oracle.is_prime(p):
        p += 2
    n = 4096
    ffp.ffp_tune_clear()
    plan = ffp.plan_describe(2048, 2176, p, lda=2176, ldc=n, alpha=p - 1, beta=1)
    head = plan.splitlines()[0]
    assert " depth=1 " in head and " cls=0 " in head
    S, out = _big_ldlt_case(n, p, 52)
    m = 768
    ref, rinfo = oracle.ldlt_packed(S[:m, :m].copy(), p)
    assert rinfo == 0
    low = np.tril(np.ones((m, m), dtype=bool))
    assert np.array_equal(out[:m, :m][low], ref[low])
    _freivalds_ldlt(S, out, p)
