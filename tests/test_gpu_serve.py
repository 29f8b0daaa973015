"""GPU parity of the request loop: a Poisson stream of mixed A*A^T and LDL^T
requests, served with continuous batching over several streams, gives for
every request exactly the oracle's result and the result of the same job
run alone through fsyrk_modp / fldlt_modp."""
import time

import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp, inputs
from tests.gpu_util import from_dev_u32, lower_mask, to_dev_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    oracle.build(force=False)
    ffp.lib()


def serve(reqs, ops, budget, nstreams=4, max_inflight=32):
    """Submits on the stream's arrival times and, as requests finish (the
    completion queue), copies each result out and releases it, so that a
    tight budget keeps admitting.  Returns (results, infos, stats)."""
    import threading
    import torch
    dev = [to_dev_u32(a) for a in ops]
    torch.cuda.synchronize()
    out = [None] * len(reqs)
    infos = [None] * len(reqs)
    errors = []
    with ffp.Server(budget, max_inflight=max_inflight, nstreams=nstreams) as srv:
        side = torch.cuda.Stream()

        def reaper():
            got = 0
            deadline = time.time() + 120
            while got < len(reqs) and time.time() < deadline:
                for t in srv.poll(64, 0.05):
                    i = t - 1
                    r = reqs[i]
                    res = srv.status(t)
                    if res.state != ffp.FFP_STATE_DONE or not (res.t_submit <= res.t_admit <= res.t_done):
                        errors.append((r, res.state))
                    with torch.cuda.stream(side):
                        C = torch.zeros((r["n"], r["n"]), dtype=torch.int32, device="cuda")
                        info = torch.zeros(1, dtype=torch.int64, device="cuda")
                        srv.fetch(t, C, info if r["kind"] == "ldlt" else None,
                                  stream=side.cuda_stream)
                    side.synchronize()
                    srv.release(t)
                    out[i] = from_dev_u32(C)
                    infos[i] = int(info.cpu().item())
                    got += 1

        th = threading.Thread(target=reaper)
        th.start()
        t0 = time.perf_counter()
        for i, (r, d) in enumerate(zip(reqs, dev)):
            delay = r["t"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            if r["kind"] == "syrk":
                t = srv.submit_syrk(d, r["p"])
            else:
                t = srv.submit_ldlt(d, r["p"])
            assert t == i + 1
        th.join()
        srv.drain(10.0)
        st = srv.stats()
    assert not errors, errors[:3]
    assert all(o is not None for o in out), "some requests never finished"
    assert st.peak_bytes <= budget
    return out, infos, st


def alone(r, A):
    import torch
    n = r["n"]
    if r["kind"] == "syrk":
        Ad = to_dev_u32(A)
        Cd = torch.zeros((n, n), dtype=torch.int32, device="cuda")
        ffp.syrk(Ad, r["p"], C=Cd)
        torch.cuda.synchronize()
        return from_dev_u32(Cd), 0
    Sd = to_dev_u32(A)
    info = ffp.ldlt(Sd, r["p"])
    torch.cuda.synchronize()
    return from_dev_u32(Sd), int(info.item())


def check(reqs, ops, out, infos):
    for r, A, C, info in zip(reqs, ops, out, infos):
        low = lower_mask(r["n"])
        ref_alone, info_alone = alone(r, A)
        assert np.array_equal(C[low], ref_alone[low]), r
        assert info == info_alone, r
        if r["kind"] == "syrk":
            ref = oracle.syrk(A, r["p"])
            assert np.array_equal(C[low], ref[low]), r
        else:
            ref, rinfo = oracle.ldlt_packed(A, r["p"])
            assert info == rinfo, r
            if info == 0:
                assert np.array_equal(C[low], ref[low]), r


def test_served_mixed_stream():
    reqs = inputs.request_stream(seed=4, nreq=48, rate=3000.0, nmin=32, nmax=600)
    ops = [inputs.request_operand(4, r) for r in reqs]
    out, infos, st = serve(reqs, ops, budget=1 << 30)
    assert st.completed == len(reqs)
    assert st.units <= len(reqs)
    check(reqs, ops, out, infos)


def test_served_tight_budget_and_one_stream():
    # the arena fits about two requests: admission waits for completions and
    # releases, results still exact
    reqs = inputs.request_stream(seed=9, nreq=16, rate=50000.0, nmin=100, nmax=300)
    ops = [inputs.request_operand(9, r) for r in reqs]
    big = max(r["n"] for r in reqs)
    ws = max(ffp.ffp_workspace_bytes(r["n"], r["k"], r["p"]) if r["kind"] == "syrk"
             else ffp.ffp_ldlt_workspace_bytes(r["n"], r["p"]) for r in reqs)
    budget = 2 * (big * ((big + 3) // 4 * 4) * 4 + 4096 + ws)
    out, infos, st = serve(reqs, ops, budget=budget, nstreams=1, max_inflight=4)
    assert st.peak_inflight <= 4
    check(reqs, ops, out, infos)


def test_served_degenerate_requests():
    # n = 1, k = 1 and odd sizes at the small end, one of each kind
    reqs = [
        {"id": 0, "t": 0.0, "kind": "syrk", "n": 1, "k": 1, "p": 131071},
        {"id": 1, "t": 0.0, "kind": "syrk", "n": 3, "k": 1, "p": 251},
        {"id": 2, "t": 0.0, "kind": "ldlt", "n": 1, "k": 1, "p": 65537},
        {"id": 3, "t": 0.0, "kind": "syrk", "n": 5, "k": 77, "p": 65521},
        {"id": 4, "t": 0.0, "kind": "ldlt", "n": 65, "k": 65, "p": 65537},
    ]
    ops = [inputs.request_operand(11, r) for r in reqs]
    out, infos, _ = serve(reqs, ops, budget=64 << 20)
    check(reqs, ops, out, infos)
