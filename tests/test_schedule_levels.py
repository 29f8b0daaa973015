"""Host-logic tests of the level scheduler (ffp_plan_levels).

Operations of one level must be independent.  The schedule is executed on
the CPU (tests/plansim.py) level by level, with the operations of each
level in reverse program order: a dependency the scheduler missed (a read of
memory an earlier operation of the same level writes, or a write over
memory it still reads) shows as a result different from the oracle's,
since the workspace starts as garbage.  Covers the placements of Tables 3
and 4 and the wide variant, whose independent products share levels, with
and without the pass that moves the products of small launches later.
"""
import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp, inputs
from tests import plansim
from tests.test_plan_sim import _operand_bytes


@pytest.fixture(params=[0, 1], ids=["table3", "wide"])
def wide(request):
    ffp.set_knob("wide", request.param)
    yield request.param
    ffp.set_knob("wide", 1)


@pytest.fixture(autouse=True, params=[1, 0], ids=["merged", "asap"])
def merge_products(request):
    """With and without moving the products of small launches to later
    levels (both schedules must keep every dependency)."""
    ffp.set_knob("merge_products", request.param)
    yield request.param
    ffp.set_knob("merge_products", 1)


def check_reordered(n, k, p, depth, alpha=1, beta=0, a_dtype=ffp.FFP_U32, seed=0):
    A = inputs.uniform(seed, n, k, p)
    rng = np.random.default_rng(seed + 1)
    C0 = rng.integers(0, 2**32, size=(n, n), dtype=np.uint64).astype(np.uint32)
    if beta:
        C0 = np.where(np.tril(np.ones((n, n), bool)), inputs.uniform(seed + 2, n, n, p), C0)
    a_bytes, lda = _operand_bytes(A, p, a_dtype)
    flags = ffp.FFP_DEPTH(depth)
    text = ffp.plan_describe(n, k, p, a_dtype, lda, n, alpha, beta, flags)
    levels = ffp.plan_levels(n, k, p, a_dtype, lda, n, alpha, beta, flags)
    plan = plansim.parse(text)
    assert len(levels) == len(plan.ops)
    order = sorted(range(len(levels)), key=lambda i: (levels[i], -i))
    out = plansim.simulate(text, p, a_bytes, C0.copy(), order=order)
    expect = oracle.syrk_ab(A, p, alpha, beta, C0.copy())
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(out[low], expect[low])
    return plan, levels


@pytest.mark.parametrize("p", [65537, 131071])
@pytest.mark.parametrize("depth", [1, 2, 3])
@pytest.mark.parametrize("n,k", [(64, 64), (48, 160), (64, 24)])
def test_levels_table3_f64(wide, p, depth, n, k):
    check_reordered(n, k, p, depth)


@pytest.mark.parametrize("depth", [1, 2])
def test_levels_table4(wide, depth):
    check_reordered(64, 48, 131071, depth, alpha=5, beta=7)
    check_reordered(32, 96, 65537, depth, alpha=65536, beta=1)


@pytest.mark.parametrize("p,a_dtype", [(251, ffp.FFP_I8_CENTERED), (65521, ffp.FFP_I8_LIMB2),
                                       (251, ffp.FFP_U32)])
def test_levels_int8_classes(wide, p, a_dtype):
    check_reordered(64, 256, p, 2, a_dtype=a_dtype)


def test_wide_products_share_levels():
    ffp.set_knob("wide", 1)
    try:
        plan, levels = check_reordered(64, 256, 131071, 3)
    finally:
        ffp.set_knob("wide", 1)
    per_level = {}
    for o, lv in zip(plan.ops, levels):
        if o.kind in (plansim.OP_GEMM, plansim.OP_SYRK):
            per_level[lv] = per_level.get(lv, 0) + 1
    # 27 leaf products and 26 general products over far fewer levels
    assert sum(per_level.values()) == 53
    assert max(per_level.values()) >= 6
    assert len(per_level) <= 20


def test_small_launch_products_move_later():
    """8192 x 32768 at depth 3: the eight leaves on blocks of A (the chains
    of P1 and P2) are ready at level 0, where they alone would form a launch
    of 288 tiles of 128 x 128; they join the large launch of a later level."""
    n, k, p = 8192, 32768, 131071
    text = ffp.plan_describe(n, k, p, flags=ffp.FFP_DEPTH(3))
    kinds = [int(line.split()[1]) for line in text.splitlines()[1:]]
    prods = [i for i, kd in enumerate(kinds) if kd in (2, 3)]
    ffp.set_knob("merge_products", 0)
    asap = ffp.plan_levels(n, k, p, flags=ffp.FFP_DEPTH(3))
    ffp.set_knob("merge_products", 1)
    merged = ffp.plan_levels(n, k, p, flags=ffp.FFP_DEPTH(3))
    assert sum(asap[i] == 0 for i in prods) == 8
    assert sum(merged[i] == 0 for i in prods) == 0
    assert all(merged[i] >= asap[i] for i in prods)
    assert all(merged[i] == asap[i] for i in range(len(kinds)) if i not in prods)
    assert len(set(merged[i] for i in prods)) < len(set(asap[i] for i in prods))


@pytest.mark.parametrize("p", [65537, 131071])
@pytest.mark.parametrize("n,k,depth", [(64, 64, 1), (96, 160, 2), (128, 48, 1), (64, 256, 3)])
def test_winograd_general_products(p, n, k, depth):
    """General products P3, P4 through one level of Strassen-Winograd (the
    size threshold lowered to 16): the plan holds the additions, and run in
    program order and level by level (reverse order inside a level) it still
    computes A A^T."""
    ffp.set_knob("winograd_min", 16)
    try:
        plan, levels = check_reordered(n, k, p, depth)
        kinds = [o.kind for o in plan.ops]
        assert plansim.OP_LINCOMB in kinds
        A = inputs.uniform(3, n, k, p)
        text = ffp.plan_describe(n, k, p, flags=ffp.FFP_DEPTH(depth))
        out = plansim.simulate(text, p, A.astype(np.uint32).tobytes(), np.zeros((n, n), np.uint32))
        low = np.tril(np.ones((n, n), dtype=bool))
        assert np.array_equal(out[low], oracle.syrk(A, p)[low])
    finally:
        ffp.set_knob("winograd_min", 0)


def test_winograd_only_for_plain_wide_fp64():
    """No Strassen-Winograd additions under Table 4 (beta != 0), with the
    Table 3 placements, on int8 paths or below the size threshold."""
    ffp.set_knob("winograd_min", 16)
    try:
        def has_lincomb(*args, **kw):
            text = ffp.plan_describe(*args, **kw)
            return any(int(l.split()[1]) == plansim.OP_LINCOMB for l in text.splitlines()[1:])
        assert has_lincomb(64, 64, 65537, flags=ffp.FFP_DEPTH(1))
        assert not has_lincomb(64, 64, 65537, alpha=3, beta=2, flags=ffp.FFP_DEPTH(1))
        assert not has_lincomb(64, 64, 65537, flags=ffp.FFP_DEPTH(1) | ffp.FFP_LOW_MEMORY)
        assert not has_lincomb(64, 64, 251, flags=ffp.FFP_DEPTH(1))
        ffp.set_knob("winograd_min", 64)
        assert not has_lincomb(64, 64, 65537, flags=ffp.FFP_DEPTH(1))
    finally:
        ffp.set_knob("winograd_min", 0)
