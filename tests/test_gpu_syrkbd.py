"""GPU parity of fsyrkbd_modp (Algorithm 6, odd characteristic: A B A^T for
B block diagonal with scalar and antidiagonal 2 x 2 blocks) against the
oracle's plain triple sum, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import ffp
from tests.gpu_util import from_dev_u32, to_dev_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    oracle.build(force=False)
    ffp.lib()


def block_diagonal(n, p, nblocks, nonres_parity, seed):
    """bdiag, boff of a block diagonal B with `nblocks` antidiagonal 2 x 2
    blocks at random non-overlapping places and random scalar blocks whose
    count of quadratic non-residues has the given parity (None: any)."""
    rng = np.random.default_rng(seed)
    bdiag = rng.integers(0, p, size=n, dtype=np.uint64).astype(np.uint32)
    boff = np.zeros(max(n - 1, 0), dtype=np.uint32)
    free = list(range(n - 1))
    rng.shuffle(free)
    taken = np.zeros(n, dtype=bool)
    placed = 0
    for j in free:
        if placed == nblocks:
            break
        if taken[j] or taken[j + 1]:
            continue
        taken[j] = taken[j + 1] = True
        boff[j] = rng.integers(1, p)
        bdiag[j] = bdiag[j + 1] = 0
        placed += 1
    assert placed == nblocks, "not enough room for the blocks"
    scal = [j for j in range(n) if not taken[j]]
    if nonres_parity is not None and scal:
        nr = sum(1 for j in scal if oracle.legendre(int(bdiag[j]), p) == -1)
        if nr % 2 != nonres_parity:
            # flip one scalar between a residue and a non-residue
            j = scal[0]
            want = -1 if oracle.legendre(int(bdiag[j]), p) != -1 else 1
            v = 1
            while oracle.legendre(v, p) != want:
                v += 1
            bdiag[j] = v
    return bdiag, boff


def run(A, bdiag, boff, p, alpha=1, beta=0, C0=None, depth=None):
    import torch
    m, n = A.shape
    Ad = to_dev_u32(A)
    bd = to_dev_u32(bdiag)
    bo = to_dev_u32(boff) if n > 1 else None
    Cd = to_dev_u32(C0) if C0 is not None else torch.zeros((m, m), dtype=torch.int32, device=Ad.device)
    info = torch.full((1,), -7, dtype=torch.int64, device=Ad.device)
    ffp.syrkbd(Ad, bd, bo, p, alpha=alpha, beta=beta, C=Cd, info=info, depth=depth)
    torch.cuda.synchronize()
    return from_dev_u32(Cd), int(info.item())


CASES = [
    # m, n, p, antidiagonal blocks, parity of the scalar non-residue count
    (1, 1, 65537, 0, 1),
    (65, 65, 65537, 7, 0),
    (65, 65, 131071, 8, 1),
    (300, 65, 251, 3, 1),
    (65, 300, 65521, 40, 0),
    (300, 300, 1000003, 51, 1),
    (300, 300, 3, 20, 0),
    (2048, 300, 131071, 33, 0),
    (300, 2048, 65537, 301, 1),
    (2048, 2048, 251, 512, 1),
    (257, 129, 33554467, 10, 1),
]


@pytest.mark.parametrize("m,n,p,nb,par", CASES)
def test_syrkbd_vs_oracle(m, n, p, nb, par):
    rng = np.random.default_rng(m * 7 + n + p)
    A = rng.integers(0, p, size=(m, n), dtype=np.uint64).astype(np.uint32)
    bdiag, boff = block_diagonal(n, p, nb, par, seed=m + n)
    got, info = run(A, bdiag, boff, p)
    assert info == 0
    want = oracle.syrkbd(A, bdiag, boff, p)
    low = np.tril(np.ones((m, m), dtype=bool))
    assert np.array_equal(got[low], want[low])


@pytest.mark.parametrize("depth", [0, 1, 2])
@pytest.mark.parametrize("p", [65537, 131071, 251])
def test_syrkbd_alpha_beta_and_depth(depth, p):
    m, n = 520, 333
    rng = np.random.default_rng(depth + p)
    A = rng.integers(0, p, size=(m, n), dtype=np.uint64).astype(np.uint32)
    C0 = rng.integers(0, p, size=(m, m), dtype=np.uint64).astype(np.uint32)
    bdiag, boff = block_diagonal(n, p, 60, depth % 2, seed=p)
    alpha, beta = int(rng.integers(1, p)), int(rng.integers(1, p))
    got, info = run(A, bdiag, boff, p, alpha=alpha, beta=beta, C0=C0, depth=depth)
    assert info == 0
    want = oracle.syrkbd(A, bdiag, boff, p, alpha=alpha, beta=beta, C=C0)
    low = np.tril(np.ones((m, m), dtype=bool))
    assert np.array_equal(got[low], want[low])


def test_syrkbd_all_antidiagonal_and_all_zero():
    p = 65537
    m, n = 100, 64
    rng = np.random.default_rng(3)
    A = rng.integers(0, p, size=(m, n), dtype=np.uint64).astype(np.uint32)
    bdiag = np.zeros(n, dtype=np.uint32)
    boff = np.zeros(n - 1, dtype=np.uint32)
    boff[0::2] = rng.integers(1, p, size=n // 2)
    got, info = run(A, bdiag, boff, p)
    assert info == 0
    want = oracle.syrkbd(A, bdiag, boff, p)
    low = np.tril(np.ones((m, m), dtype=bool))
    assert np.array_equal(got[low], want[low])
    # B = 0: the product vanishes
    got, info = run(A, np.zeros(n, dtype=np.uint32), np.zeros(n - 1, dtype=np.uint32), p)
    assert info == 0 and not got[low].any()


@pytest.mark.parametrize("bad", ["overlap", "diag_in_block", "too_large"])
def test_syrkbd_reports_malformed_blocks(bad):
    p = 131071
    m, n = 40, 20
    A = np.ones((m, n), dtype=np.uint32)
    bdiag = np.zeros(n, dtype=np.uint32)
    boff = np.zeros(n - 1, dtype=np.uint32)
    if bad == "overlap":
        boff[5] = boff[6] = 3
        want = 7          # column 6 ends one block and starts another
    elif bad == "diag_in_block":
        boff[9] = 4
        bdiag[10] = 1
        want = 10
    else:
        bdiag[13] = p
        want = 14
    _, info = run(A, bdiag, boff, p)
    assert info == want
