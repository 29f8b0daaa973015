"""Host-only check of the division-free leaf elimination the LDL^T leaf
kernel uses: step k replaces M[i][j] by a_k M[i][j] - M[i][k] M[k][j] with
a_k = M[k][k]; then D[k] = a_k / (a_0 ... a_{k-1}) and L[i][k] = M[i][k] / a_k
(M[i][k] as it stands at step k).  Compared with the oracle's Crout LDL^T,
including the index of the first zero pivot."""
import numpy as np
import pytest

import oracle
from paper_2001_04109_amd import inputs


def division_free_ldlt(S, p):
    n = S.shape[0]
    M = [[int(S[i][j]) for j in range(n)] for i in range(n)]
    for k in range(n):
        a = M[k][k]
        if a == 0:
            return None, k + 1
        for i in range(k + 1, n):
            for j in range(k + 1, i + 1):
                M[i][j] = (a * M[i][j] - M[i][k] * M[j][k]) % p
    out = np.zeros((n, n), dtype=np.uint32)
    g = 1
    for k in range(n):
        a = M[k][k]
        out[k, k] = a * pow(g, p - 2, p) % p
        ainv = pow(a, p - 2, p)
        for i in range(k + 1, n):
            out[i, k] = M[i][k] * ainv % p
        g = g * a % p
    return out, 0


@pytest.mark.parametrize("p", [3, 251, 65537, 131071, 33554393])
@pytest.mark.parametrize("n", [1, 2, 7, 33, 64])
def test_division_free_leaf_matches_crout(p, n):
    S = inputs.symmetric(n * 7 + p % 1000, n, p)
    ref, info = oracle.ldlt_packed(S, p)
    out, zinfo = division_free_ldlt(S, p)
    assert zinfo == info
    if info == 0:
        low = np.tril(np.ones((n, n), dtype=bool))
        assert np.array_equal(out[low], ref[low])


def test_division_free_leaf_zero_pivot_index():
    p, n = 65537, 12
    rng = np.random.default_rng(1)
    L = np.tril(rng.integers(0, p, size=(n, n)), -1).astype(object)
    L[np.arange(n), np.arange(n)] = 1
    D = rng.integers(1, p, size=n).astype(object)
    D[5] = 0
    S = np.array((L * D).dot(L.T) % p, dtype=np.uint32)
    _, info = oracle.ldlt_packed(S, p)
    assert info == 6
    assert division_free_ldlt(S, p)[1] == 6
