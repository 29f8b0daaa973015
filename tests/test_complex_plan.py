"""CPU simulation of the schedules of fzsyrk_modp and fherk_modp (Algorithm 2
over F_p[i] with Y = i I, or with conjugate transposition and
Y = (a + ib) I; 3M general products, 2M leaves) against the oracle's plain
A A^T and A A^H over F_p[i]."""
import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp
from tests import plansim


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)
    ffp.lib()


def rand_planes(n, k, p, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, p, size=(2, n, k), dtype=np.uint64).astype(np.uint32)


@pytest.mark.parametrize("herk", [False, True])
@pytest.mark.parametrize("p", [3, 7, 251, 65537, 131071, 1000003])
@pytest.mark.parametrize("n,k,depth", [(1, 1, 0), (5, 3, 0), (8, 8, 1), (12, 20, 2), (17, 9, 1), (32, 48, 3),
                                       (40, 16, 2)])
def test_complex_schedule_matches_oracle(herk, p, n, k, depth):
    A = rand_planes(n, k, p, seed=n * 31 + k + p)
    text = ffp.complex_plan_describe(n, k, p, herk=herk, flags=ffp.FFP_DEPTH(depth) | ffp.FFP_FILL_UPPER)
    got = plansim.simulate_complex(text, p, A)
    want_re, want_im = (oracle.herk if herk else oracle.zsyrk)(A[0], A[1], p)
    assert np.array_equal(got[0], want_re)
    assert np.array_equal(got[1], want_im)


@pytest.mark.parametrize("herk", [False, True])
def test_complex_schedule_reverse_level_order(herk):
    """Operations of one level run in reverse order (and the workspace starts
    as garbage): the level scheduler's edges cover every dependency."""
    p, n, k, depth = 131071, 24, 40, 2
    A = rand_planes(n, k, p, seed=9)
    flags = ffp.FFP_DEPTH(depth)
    text = ffp.complex_plan_describe(n, k, p, herk=herk, flags=flags)
    plan = plansim.parse(text)
    lv = ffp.complex_plan_levels(n, k, p, herk=herk, flags=flags)
    assert len(lv) == len(plan.ops)
    order = sorted(range(len(lv)), key=lambda i: (lv[i], -i))
    got = plansim.simulate_complex(text, p, A, order=order)
    want_re, want_im = (oracle.herk if herk else oracle.zsyrk)(A[0], A[1], p)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(got[0][low], want_re[low])
    assert np.array_equal(got[1][low], want_im[low])
