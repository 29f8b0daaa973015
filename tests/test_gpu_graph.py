"""GPU parity of batched calls recorded as HIP graphs (ffp_graph_*): every
replay equals the eager batched call on the same inputs, bit for bit, and
the oracle on the small jobs.  Replays alternate with eager library work and
host synchronisations, and the inputs are rewritten before each replay."""
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


def syrk_specs(seed, count, nmax=260, primes=(251, 65521, 65537, 131071)):
    rng = np.random.default_rng(seed)
    specs = []
    for j in range(count):
        n = int(rng.integers(1, nmax + 1))
        k = int(rng.integers(max(1, n // 2), 2 * n + 1))
        p = int(primes[j % len(primes)])
        alpha = int(rng.integers(1, p)) if j % 3 == 1 else 1
        beta = int(rng.integers(0, p)) if j % 2 else 0
        specs.append((inputs.uniform((seed, j), n, k, p), p, alpha, beta,
                      inputs.uniform((seed, j, 1), n, n, p)))
    return specs


def upload(specs):
    devA, devC, jobs = [], [], []
    for A, p, alpha, beta, C0 in specs:
        Ad, Cd = to_dev_u32(A), to_dev_u32(C0)
        devA.append(Ad)
        devC.append(Cd)
        jobs.append(ffp.make_job(Ad, Cd, p, alpha, beta))
    return devA, devC, jobs


def reset(devC, specs):
    import torch
    for Cd, (_, _, _, _, C0) in zip(devC, specs):
        Cd.copy_(torch.from_numpy(C0.view(np.int32)))


@pytest.mark.parametrize("flags", [0, ffp.FFP_DEPTH(1)])
def test_syrk_graph_replays_match_eager(flags):
    """30 jobs over four primes (int8, limb and FP64 classes, more than the
    inline task count per class, alpha/beta forms): three replays, two of
    them on a stream other than the recording one."""
    import torch
    specs = syrk_specs(70 + flags, 30)
    devA, devC, jobs = upload(specs)
    ffp.fsyrk_modp_batched(jobs, flags)
    torch.cuda.synchronize()
    eager = [from_dev_u32(c) for c in devC]
    for (A, p, alpha, beta, C0), out in list(zip(specs, eager))[:8]:
        low = lower_mask(A.shape[0])
        assert np.array_equal(out[low], oracle.syrk_ab(A, p, alpha, beta, C0)[low])

    rec = torch.cuda.Stream()
    g = ffp.Graph.syrk_batched(jobs, flags, stream=rec, keep=(devA, devC))
    try:
        assert g.nodes > 0
        other = torch.cuda.Stream()
        for rep in range(3):
            reset(devC, specs)
            torch.cuda.synchronize()
            # eager library work between replays
            X = to_dev_u32(inputs.uniform((71, rep), 96, 64, 65537))
            Y = torch.zeros((96, 96), dtype=torch.int32, device=X.device)
            ffp.fsyrk_modp(96, 64, 65537, X, 64, ffp.FFP_U32, 1, 0, Y, 96)
            torch.cuda.synchronize()
            s = rec if rep == 0 else other
            g.launch(stream=s)
            torch.cuda.synchronize()
            for (A, _, _, _, _), out, Cd in zip(specs, eager, devC):
                low = lower_mask(A.shape[0])
                assert np.array_equal(from_dev_u32(Cd)[low], out[low]), rep
    finally:
        g.close()


def test_syrk_graph_inputs_read_at_replay():
    """A replay reads the operands as they are when it runs: new contents of
    A give the new product."""
    import torch
    specs = syrk_specs(80, 9, nmax=200)
    devA, devC, jobs = upload(specs)
    rec = torch.cuda.Stream()
    with ffp.Graph.syrk_batched(jobs, 0, stream=rec, keep=(devA, devC)) as g:
        for rep in range(2):
            new = []
            for j, (Ad, (A, p, alpha, beta, C0)) in enumerate(zip(devA, specs)):
                A2 = inputs.uniform((81, rep, j), A.shape[0], A.shape[1], p)
                Ad.copy_(torch.from_numpy(A2.view(np.int32)))
                new.append((A2, p, alpha, beta, C0))
            reset(devC, specs)
            torch.cuda.synchronize()
            g.launch(stream=rec)
            torch.cuda.synchronize()
            for (A2, p, alpha, beta, C0), Cd in zip(new, devC):
                low = lower_mask(A2.shape[0])
                assert np.array_equal(from_dev_u32(Cd)[low], oracle.syrk_ab(A2, p, alpha, beta, C0)[low])


def test_ldlt_graph_replays_match_eager():
    import torch
    specs = [(64, 65537), (65, 131071), (130, 251), (300, 65521), (520, 65537), (9, 65537)]
    mats = [inputs.symmetric(950 + i, n, p) for i, (n, p) in enumerate(specs)]
    dev = [to_dev_u32(S) for S in mats]
    info = ffp.ldlt_batched(dev, [p for _, p in specs])
    torch.cuda.synchronize()
    eager = [from_dev_u32(Sd) for Sd in dev]
    eager_info = info.cpu().numpy().copy()
    for (n, p), S, out, inf in list(zip(specs, mats, eager, eager_info))[:3]:
        ref, rinfo = oracle.ldlt_packed(S, p)
        assert inf == rinfo == 0
        low = lower_mask(n)
        assert np.array_equal(out[low], ref[low])

    info2 = torch.full((len(specs),), -7, dtype=torch.int64, device=dev[0].device)
    jobs = [ffp.ffp_ldlt_job(n=n, p=p, S=Sd.data_ptr(), lds=Sd.stride(0), info=info2.data_ptr() + 8 * j)
            for j, ((n, p), Sd) in enumerate(zip(specs, dev))]
    rec = torch.cuda.Stream()
    with ffp.Graph.ldlt_batched(jobs, stream=rec, keep=(dev, info2)) as g:
        assert g.nodes > 0 and g.device_bytes > 0
        for rep in range(3):
            for Sd, S in zip(dev, mats):
                Sd.copy_(torch.from_numpy(S.view(np.int32)))
            info2.fill_(-7)
            torch.cuda.synchronize()
            g.launch(stream=rec)
            torch.cuda.synchronize()
            assert np.array_equal(info2.cpu().numpy(), eager_info), rep
            for (n, _), Sd, out in zip(specs, dev, eager):
                low = lower_mask(n)
                assert np.array_equal(from_dev_u32(Sd)[low], out[low]), (rep, n)


def test_graph_empty_batch_and_errors():
    import torch
    rec = torch.cuda.Stream()
    with ffp.Graph.syrk_batched([], 0, stream=rec) as g:
        assert g.nodes == 0
        g.launch(stream=rec)
    A = to_dev_u32(inputs.uniform((90,), 16, 16, 251))
    C = torch.zeros((16, 16), dtype=torch.int32, device=A.device)
    job = ffp.make_job(A, C, 251)
    with pytest.raises(ffp.FfpError):
        ffp.ffp_graph_syrk_batched([job], 0, stream=0)          # null stream
    bad = ffp.make_job(A, C, 250)
    with pytest.raises(ffp.FfpError):
        ffp.ffp_graph_syrk_batched([bad], 0, stream=rec)       # not prime
    torch.cuda.synchronize()
