"""Host logic of the autotuner's table (no device needed): shape classes,
what a table entry changes in the emitted schedule (and that the schedule
it selects still computes A A^T mod p, through the CPU plan simulator),
workspace figures, save/load, malformed files, and that the LDL^T driver
ignores the table."""
import os

import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp, inputs
from tests import plansim

CLS_F64, CLS_I8, CLS_LIMB2 = 0, 1, 2


@pytest.fixture(autouse=True)
def clean_table():
    ffp.lib()
    ffp.ffp_tune_clear()
    yield
    ffp.ffp_tune_clear()


def write_table(tmp_path, rows, name="t.txt"):
    path = os.path.join(str(tmp_path), name)
    with open(path, "w") as f:
        f.write("# cls log2n log2k accumulate lowmem depth tile wide base ms\n")
        for r in rows:
            f.write(" ".join(str(x) for x in r) + "\n")
    return path


def head(text):
    return dict(kv.split("=") for kv in text.splitlines()[0].split()[1:])


def test_entry_selects_depth_tile_and_placements(tmp_path):
    # n = 1000 -> ceil(log2) = 10; k = 700 -> 10; FP64 class for p = 131071
    path = write_table(tmp_path, [(CLS_F64, 10, 10, 0, 0, 2, 128, 0, 0, 1.5)])
    before = head(ffp.plan_describe(1000, 700, 131071))
    assert before["tuned"] == "0"
    assert ffp.ffp_tune_load(path) == 1
    assert ffp.ffp_tune_entries() == 1
    h = head(ffp.plan_describe(1000, 700, 131071))
    assert (h["depth"], h["tile"], h["wide"], h["tuned"]) == ("2", "128", "0", "1")
    look = ffp.ffp_tune_lookup(1000, 700, 131071)
    assert look["tuned"] and (look["depth"], look["tile"], look["wide"]) == (2, 128, 0)
    assert look["ms"] == pytest.approx(1.5)
    # same class: other sizes in the same power-of-two buckets
    assert head(ffp.plan_describe(513, 513, 131071))["tuned"] == "1"
    # other classes are untouched
    assert head(ffp.plan_describe(1025, 700, 131071))["tuned"] == "0"
    assert head(ffp.plan_describe(1000, 700, 131071, alpha=2))["tuned"] == "0"
    assert head(ffp.plan_describe(1000, 700, 131071, flags=ffp.FFP_LOW_MEMORY))["tuned"] == "0"
    assert head(ffp.plan_describe(1000, 700, 251))["tuned"] == "0"


def test_forced_depth_keeps_rule_but_matching_depth_takes_tile(tmp_path):
    ffp.ffp_tune_load(write_table(tmp_path, [(CLS_F64, 10, 10, 0, 0, 2, 64, 1, 0, 0.0)]))
    h = head(ffp.plan_describe(1000, 700, 131071, flags=ffp.FFP_DEPTH(1)))
    assert (h["depth"], h["tile"], h["tuned"]) == ("1", "0", "0")
    h = head(ffp.plan_describe(1000, 700, 131071, flags=ffp.FFP_DEPTH(2)))
    assert (h["depth"], h["tile"], h["tuned"]) == ("2", "64", "0")


def test_workspace_figure_follows_the_table(tmp_path):
    n, k, p = 1000, 1800, 131071
    ws_rule = ffp.ffp_workspace_bytes(n, k, p)
    ffp.ffp_tune_load(write_table(tmp_path, [(CLS_F64, 10, 11, 0, 0, 3, 0, 1, 0, 0.0)]))
    ws_tuned = ffp.ffp_workspace_bytes(n, k, p)
    assert ws_tuned == int(head(ffp.plan_describe(n, k, p, lda=k, ldc=n))["ws"])
    assert ws_tuned != ws_rule
    forced = ffp.ffp_workspace_bytes(n, k, p, flags=ffp.FFP_DEPTH(3))
    assert ws_tuned == forced
    ffp.ffp_tune_clear()
    assert ffp.ffp_workspace_bytes(n, k, p) == ws_rule


@pytest.mark.parametrize("row,n,k,p,alpha,beta,a_dtype", [
    ((CLS_F64, 6, 7, 0, 0, 2, 128, 0, 0, 0.0), 40, 72, 131071, 1, 0, ffp.FFP_U32),
    ((CLS_F64, 6, 6, 1, 0, 1, 64, 1, 0, 0.0), 48, 40, 65537, 5, 3, ffp.FFP_U32),
    ((CLS_I8, 6, 6, 0, 0, 1, 256, 1, 0, 0.0), 64, 64, 251, 1, 0, ffp.FFP_U32),
    ((CLS_LIMB2, 6, 6, 0, 1, 2, 0, 0, 0, 0.0), 64, 48, 65521, 1, 0, ffp.FFP_U32),
])
def test_tuned_schedule_computes_the_product(tmp_path, row, n, k, p, alpha, beta, a_dtype):
    lowmem = row[4]
    ffp.ffp_tune_load(write_table(tmp_path, [row]))
    flags = ffp.FFP_LOW_MEMORY if lowmem else 0
    text = ffp.plan_describe(n, k, p, a_dtype, k, n, alpha, beta, flags)
    h = head(text)
    assert h["tuned"] == "1" and h["depth"] == str(row[5])
    A = inputs.uniform((5, n, k), n, k, p)
    C0 = inputs.uniform((6, n), n, n, p)
    out = plansim.simulate(text, p, A.astype(np.uint32).tobytes(), C0.copy())[:, :n]
    expect = oracle.syrk_ab(A, p, alpha, beta, C0.copy())
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(out[low], expect[low])


def test_entry_moves_fp64_shape_to_three_limbs(tmp_path):
    """A base-3 entry puts an FP64-path shape (p = 131071) on three int8
    limbs at depth 0; the emitted schedule still computes A A^T; the pinned
    workspace figure follows."""
    n, k, p = 200, 300, 131071
    ffp.ffp_tune_load(write_table(tmp_path, [(CLS_F64, 8, 9, 0, 0, 0, 0, 1, 3, 0.5)]))
    text = ffp.plan_describe(n, k, p, ffp.FFP_U32, k, n)
    h = head(text)
    assert (h["cls"], h["depth"], h["tuned"]) == ("3", "0", "1")
    look = ffp.ffp_tune_lookup(n, k, p)
    assert look["tuned"] and look["base"] == 3
    A = inputs.uniform((12, n, k), n, k, p)
    C0 = inputs.uniform((13, n), n, n, p)
    out = plansim.simulate(text, p, A.astype(np.uint32).tobytes(), C0.copy())[:, :n]
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(out[low], oracle.syrk_ab(A, p, 1, 0, C0.copy())[low])
    assert ffp.ffp_workspace_bytes(n, k, p) == ffp.ffp_workspace_bytes(n, k, p, flags=ffp.FFP_BASE_LIMB3)
    # a forced FP64 base or an int8-path prime ignores the entry's base
    assert head(ffp.plan_describe(n, k, p, flags=ffp.FFP_BASE_F64))["cls"] == "0"


def test_save_load_roundtrip(tmp_path):
    rows = [(CLS_F64, 13, 13, 0, 0, 3, 128, 1, 0, 45.25), (CLS_I8, 14, 14, 0, 0, 0, 256, 1, 0, 2.9),
            (CLS_LIMB2, 12, 12, 1, 1, 1, 0, 0, 0, 3.5), (CLS_F64, 10, 11, 0, 0, 0, 0, 1, 3, 1.25)]
    ffp.ffp_tune_load(write_table(tmp_path, rows))
    out = os.path.join(str(tmp_path), "saved.txt")
    ffp.ffp_tune_save(out)
    ffp.ffp_tune_clear()
    assert ffp.ffp_tune_entries() == 0
    assert ffp.ffp_tune_load(out) == 4
    lines = sorted(ln.split() for ln in open(out) if not ln.startswith("#"))
    assert [tuple(int(x) for x in ln[:9]) for ln in lines] == sorted(r[:9] for r in rows)


@pytest.mark.parametrize("bad", [
    "0 10 10 0 0 2 96 1 0 1.0",    # tile not offered by the FP64 kernels
    "2 10 10 0 0 2 128 1 0 1.0",   # limb kernels have one tile
    "4 10 10 0 0 2 0 1 0 1.0",     # no such class
    "0 10 10 2 0 2 0 1 0 1.0",
    "0 10 10 0 0 9 0 1 0 1.0",     # depth beyond the flag range
    "0 10 10 0 0 1 0 1 3 1.0",     # three-limb base only at depth 0
    "1 10 10 0 0 0 0 1 3 1.0",     # three-limb base only for FP64-path shapes
    "0 10 10 0 0 0 64 1 3 1.0",    # ... with the launch-rule tile
    "0 10 10 0 0 2 0 1 0",         # missing field
    "zero 10 10 0 0 2 0 1 0 1.0",
])
def test_malformed_file_changes_nothing(tmp_path, bad):
    good = write_table(tmp_path, [(CLS_F64, 9, 9, 0, 0, 1, 64, 1, 0, 0.0)], "good.txt")
    assert ffp.ffp_tune_load(good) == 1
    path = os.path.join(str(tmp_path), "bad.txt")
    with open(path, "w") as f:
        f.write("0 11 11 0 0 1 64 1 0 0.0\n" + bad + "\n")
    with pytest.raises(ffp.FfpError):
        ffp.ffp_tune_load(path)
    assert ffp.ffp_tune_entries() == 1
    with pytest.raises(ffp.FfpError):
        ffp.ffp_tune_load(os.path.join(str(tmp_path), "missing.txt"))


def test_ldlt_ignores_the_table(tmp_path):
    before = [ffp.ffp_ldlt_workspace_bytes(n, 65537) for n in (300, 1000, 2500)]
    # depth 2 everywhere: different from the built-in rule for these updates
    rows = [(CLS_F64, ln, lk, acc, lm, 2, 0, 1, 0, 0.0)
            for ln in range(6, 13) for lk in range(6, 13) for acc in (0, 1) for lm in (0, 1)]
    ffp.ffp_tune_load(write_table(tmp_path, rows))
    after = [ffp.ffp_ldlt_workspace_bytes(n, 65537) for n in (300, 1000, 2500)]
    assert before == after


def test_autotune_argument_errors():
    with pytest.raises(ffp.FfpError):
        ffp.ffp_autotune(0, 16, 65537, stream=0)
    with pytest.raises(ffp.FfpError):
        ffp.ffp_autotune(16, 16, 65537, flags=ffp.FFP_DEPTH(1), stream=0)
