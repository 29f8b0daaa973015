"""GPU runs of the autotuner: a tuned choice is one of the candidates, it is
what later calls of the shape class use, and results stay exact (oracle)
for plain, batched and served calls that follow the table."""
import os

import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp, inputs
from tests.gpu_util import centred_i8, from_dev_u32, lower_mask, to_dev_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    oracle.build(force=False)
    ffp.lib()


@pytest.fixture(autouse=True)
def clean_table():
    ffp.ffp_tune_clear()
    yield
    ffp.ffp_tune_clear()


@pytest.mark.parametrize("n,k,p,a_dtype,alpha,beta", [
    (1024, 1024, 131071, ffp.FFP_U32, 1, 0),
    (700, 1300, 65537, ffp.FFP_U32, 5, 3),
    (512, 512, 251, ffp.FFP_I8_CENTERED, 1, 0),
    (384, 256, 65521, ffp.FFP_U32, 1, 0),
])
def test_autotune_then_exact_call(n, k, p, a_dtype, alpha, beta):
    import torch
    print(f"autotune n={n} k={k} p={p} dtype={a_dtype}", flush=True)
    r = ffp.ffp_autotune(n, k, p, a_dtype, alpha, beta)
    assert r["candidates"] >= 1 and r["ms"] > 0 and r["rule_ms"] > 0
    assert r["ms"] <= r["rule_ms"] * 1.5 + 0.05
    look = ffp.ffp_tune_lookup(n, k, p, a_dtype, alpha, beta)
    assert look["tuned"] and (look["depth"], look["tile"], look["wide"]) == (r["depth"], r["tile"], r["wide"])
    A = inputs.uniform((11, n, k), n, k, p)
    C0 = inputs.uniform((12, n), n, n, p)
    if a_dtype == ffp.FFP_I8_CENTERED:
        Ad = torch.from_numpy(centred_i8(A, p)).cuda()
    else:
        Ad = to_dev_u32(A)
    Cd = to_dev_u32(C0)
    ffp.fsyrk_modp(n, k, p, Ad, k, a_dtype, alpha, beta, Cd, n)
    torch.cuda.synchronize()
    out = from_dev_u32(Cd)
    low = lower_mask(n)
    assert np.array_equal(out[low], oracle.syrk_ab(A, p, alpha, beta, C0)[low])


def test_table_drives_batched_and_served_calls(tmp_path):
    """Entries that force depths 1-2, the Table 3 placements, both tiles and
    the three-limb base: batched jobs and served requests stay exact;
    entries cleared while requests wait do not change their workspace
    (fixed at submission)."""
    import torch
    rows = ["0 8 8 0 0 2 64 0 0 0", "0 8 9 0 0 1 128 1 0 0", "1 8 8 0 0 1 128 0 0 0", "0 9 9 0 0 2 128 1 0 0",
            "0 9 10 0 0 0 0 1 3 0"]
    path = os.path.join(str(tmp_path), "t.txt")
    with open(path, "w") as f:
        f.write("\n".join(rows) + "\n")
    assert ffp.ffp_tune_load(path) == 5
    specs = [(200, 240, 131071), (256, 300, 65537), (180, 180, 251), (400, 400, 131071), (150, 90, 65537),
             (300, 700, 131071)]
    mats = [inputs.uniform((13, j), n, k, p) for j, (n, k, p) in enumerate(specs)]
    devA = [to_dev_u32(A) for A in mats]
    devC = [torch.zeros((n, n), dtype=torch.int32, device="cuda") for n, _, _ in specs]
    jobs = [ffp.make_job(Ad, Cd, p) for Ad, Cd, (_, _, p) in zip(devA, devC, specs)]
    ffp.fsyrk_modp_batched(jobs)
    torch.cuda.synchronize()
    for A, Cd, (n, _, p) in zip(mats, devC, specs):
        low = lower_mask(n)
        assert np.array_equal(from_dev_u32(Cd)[low], oracle.syrk(A, p)[low])

    with ffp.Server(hbm_budget=1 << 30, max_inflight=8, nstreams=2) as srv:
        tickets = [srv.submit_syrk(Ad, p) for Ad, (_, _, p) in zip(devA, specs)]
        ffp.ffp_tune_clear()
        srv.drain()
        for t, A, (n, _, p) in zip(tickets, mats, specs):
            out = torch.zeros((n, n), dtype=torch.int32, device="cuda")
            srv.fetch(t, out)
            torch.cuda.synchronize()
            low = lower_mask(n)
            assert np.array_equal(from_dev_u32(out)[low], oracle.syrk(A, p)[low])
            srv.release(t)
