"""Host-only tests of the request loop's scheduler against a simulated device
(ffp_server_create_simulated: units complete after a modelled time and
compute nothing): admission by memory footprint, arrival order, iteration-
level batching, overlap of units, error handling."""
import threading
import time

import numpy as np
import pytest

from paper_2001_04109_amd import ffp, inputs


def _fake_ptr():
    return 1 << 20      # never dereferenced by the simulated device


def submit_stream(srv, reqs, rate_scale=1.0):
    t0 = time.perf_counter()
    tickets = []
    for r in reqs:
        delay = r["t"] * rate_scale - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        if r["kind"] == "syrk":
            req = ffp.ffp_request(kind=ffp.FFP_REQ_SYRK, n=r["n"], k=r["k"], p=r["p"], alpha=1,
                                  A=_fake_ptr(), lda=r["k"])
        else:
            req = ffp.ffp_request(kind=ffp.FFP_REQ_LDLT, n=r["n"], k=r["n"], p=r["p"], alpha=0,
                                  A=_fake_ptr(), lda=r["n"])
        tickets.append(srv._submit(req))
    return tickets


def release_until_done(srv, tickets, timeout=60.0):
    pending = set(tickets)
    done = {}
    t_end = time.time() + timeout
    while pending and time.time() < t_end:
        for t in list(pending):
            st = srv.status(t)
            if st.state == ffp.FFP_STATE_DONE:
                done[t] = (st.t_submit, st.t_admit, st.t_done)
                srv.release(t)
                pending.discard(t)
        time.sleep(0.0005)
    assert not pending, f"{len(pending)} requests never finished"
    return done


def test_served_stream_scheduling():
    reqs = inputs.request_stream(seed=4, nreq=300, rate=20000.0, nmin=64, nmax=512)
    # budget fits only a handful of results at once
    budget = 8 * 512 * 512 * 4 + 64 * 1024 * 1024
    srv = ffp.Server(budget, max_inflight=32, nstreams=4, simulated=True, ns_per_op=0.05,
                     launch_us=20.0)
    try:
        tickets = submit_stream(srv, reqs)
        done = release_until_done(srv, tickets)
        st = srv.stats()
        assert st.submitted == len(reqs) and st.completed == len(reqs)
        assert st.peak_bytes <= budget
        assert st.units < len(reqs)            # requests were batched
        assert st.max_batch > 1
        assert st.overlapped_units > 0         # units launched while others ran
        # admission in arrival order (FIFO)
        admits = [done[t][1] for t in tickets]
        assert all(b >= a for a, b in zip(admits, admits[1:]))
        for t in tickets:
            s, a, d = done[t]
            assert s <= a <= d
    finally:
        srv.close()


def test_memory_budget_blocks_admission_until_release():
    n = 256
    one = n * n * 4
    srv = ffp.Server(one + ffp.ffp_workspace_bytes(n, n, 65537) + 4096, max_inflight=8,
                     nstreams=2, simulated=True, ns_per_op=0.0, launch_us=1.0)
    try:
        req = ffp.ffp_request(kind=ffp.FFP_REQ_SYRK, n=n, k=n, p=65537, alpha=1, A=_fake_ptr(),
                              lda=n)
        t1 = srv._submit(req)
        t2 = srv._submit(req)
        time.sleep(0.05)
        assert srv.status(t1).state == ffp.FFP_STATE_DONE
        assert srv.status(t2).state == ffp.FFP_STATE_QUEUED    # no room until t1 is released
        srv.release(t1)
        deadline = time.time() + 5
        while srv.status(t2).state != ffp.FFP_STATE_DONE and time.time() < deadline:
            time.sleep(0.001)
        assert srv.status(t2).state == ffp.FFP_STATE_DONE
    finally:
        srv.close()


def test_concurrent_submitters():
    srv = ffp.Server(1 << 34, max_inflight=64, nstreams=4, simulated=True, ns_per_op=0.001,
                     launch_us=5.0)
    tickets = []
    lock = threading.Lock()

    def worker(seed):
        rng = np.random.default_rng(seed)
        mine = []
        for _ in range(50):
            n = int(rng.integers(8, 128))
            req = ffp.ffp_request(kind=ffp.FFP_REQ_SYRK, n=n, k=n, p=131071, alpha=3,
                                  A=_fake_ptr(), lda=n)
            mine.append(srv._submit(req))
        with lock:
            tickets.extend(mine)

    try:
        ths = [threading.Thread(target=worker, args=(s,)) for s in range(4)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        srv.drain(30.0)
        assert sorted(tickets) == list(range(1, 201))
        assert srv.stats().completed == 200
    finally:
        srv.close()


def test_request_validation():
    srv = ffp.Server(1 << 30, simulated=True)
    try:
        bad = ffp.ffp_request(kind=7, n=4, k=4, p=65537, alpha=1, A=_fake_ptr(), lda=4)
        with pytest.raises(ffp.FfpError) as e:
            srv._submit(bad)
        assert e.value.status == ffp.FFP_EINVAL
        with pytest.raises(ffp.FfpError) as e:
            srv._submit(ffp.ffp_request(kind=0, n=4, k=4, p=65535, alpha=1, A=_fake_ptr(), lda=4))
        assert e.value.status == ffp.FFP_EPRIME
        with pytest.raises(ffp.FfpError) as e:
            srv._submit(ffp.ffp_request(kind=0, n=4, k=8, p=65537, alpha=1, A=_fake_ptr(), lda=4))
        assert e.value.status == ffp.FFP_EINVAL     # lda < k
        with pytest.raises(ffp.FfpError) as e:     # result alone exceeds the budget
            srv._submit(ffp.ffp_request(kind=1, n=1 << 16, k=0, p=65537, alpha=0, A=_fake_ptr(),
                                        lda=1 << 16))
        assert e.value.status == ffp.FFP_ENOMEM
    finally:
        srv.close()


def test_completion_queue_returns_each_ticket_once():
    reqs = inputs.request_stream(seed=5, nreq=200, rate=40000.0, nmin=32, nmax=256)
    srv = ffp.Server(1 << 32, max_inflight=64, nstreams=3, simulated=True, ns_per_op=0.02,
                     launch_us=10.0)
    try:
        seen = []
        tickets = submit_stream(srv, reqs)
        t_end = time.time() + 30
        while len(seen) < len(tickets) and time.time() < t_end:
            got = srv.poll(64, 0.05)
            for t in got:
                assert srv.status(t).state == ffp.FFP_STATE_DONE
                srv.release(t)
            seen.extend(got)
        assert sorted(seen) == sorted(tickets)
        assert srv.poll(8, 0.0) == []
        st = srv.stats()
        assert st.completed == len(reqs)
    finally:
        srv.close()


def _one_result_server():
    """A server whose budget holds one 256 x 256 result and its workspace."""
    n = 256
    budget = n * n * 4 + ffp.ffp_workspace_bytes(n, n, 65537) + 4096
    srv = ffp.Server(budget, max_inflight=8, nstreams=2, simulated=True, ns_per_op=0.0,
                     launch_us=1.0)
    req = ffp.ffp_request(kind=ffp.FFP_REQ_SYRK, n=n, k=n, p=65537, alpha=1, A=_fake_ptr(), lda=n)
    return srv, req


def _wait_state(srv, t, state, timeout=5.0):
    deadline = time.time() + timeout
    while srv.status(t).state != state and time.time() < deadline:
        time.sleep(0.001)
    return srv.status(t).state


def test_cancel_queued_request():
    srv, req = _one_result_server()
    try:
        t1 = srv._submit(req)
        t2 = srv._submit(req)
        assert _wait_state(srv, t1, ffp.FFP_STATE_DONE) == ffp.FFP_STATE_DONE
        assert srv.status(t2).state == ffp.FFP_STATE_QUEUED     # no room while t1 is held
        srv.cancel(t2)
        assert srv.status(t2).state == ffp.FFP_ECANCELED
        assert sorted(srv.poll(8, 0.05)) == [t1, t2]
        with pytest.raises(ffp.FfpError) as e:                   # done work is not cancelled
            srv.cancel(t1)
        assert e.value.status == ffp.FFP_EINVAL
        srv.release(t2)                                          # holds no memory: a no-op
        srv.release(t1)
        t3 = srv._submit(req)                                    # the budget is whole again
        assert _wait_state(srv, t3, ffp.FFP_STATE_DONE) == ffp.FFP_STATE_DONE
    finally:
        srv.close()


def test_deadline_fails_request_still_queued():
    srv, req = _one_result_server()
    try:
        t1 = srv._submit(req)
        assert _wait_state(srv, t1, ffp.FFP_STATE_DONE) == ffp.FFP_STATE_DONE
        timed = ffp.ffp_request(kind=req.kind, n=req.n, k=req.k, p=req.p, alpha=1, A=req.A,
                                lda=req.lda, timeout_s=0.02)
        t2 = srv._submit(timed)
        t3 = srv._submit(req)                                    # no deadline: waits
        assert _wait_state(srv, t2, ffp.FFP_ETIMEDOUT) == ffp.FFP_ETIMEDOUT
        assert srv.status(t3).state == ffp.FFP_STATE_QUEUED
        srv.release(t1)
        assert _wait_state(srv, t3, ffp.FFP_STATE_DONE) == ffp.FFP_STATE_DONE
        # a deadline that is met changes nothing
        srv.release(t3)
        t4 = srv._submit(timed)
        assert _wait_state(srv, t4, ffp.FFP_STATE_DONE) == ffp.FFP_STATE_DONE
        bad = ffp.ffp_request(kind=req.kind, n=req.n, k=req.k, p=req.p, alpha=1, A=req.A,
                              lda=req.lda, timeout_s=-1.0)
        with pytest.raises(ffp.FfpError) as e:
            srv._submit(bad)
        assert e.value.status == ffp.FFP_EINVAL
    finally:
        srv.close()
