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


# ---------------------------------------------------------------------------
# The leaf's pivot classification from prefix products, Algorithm 5's pairing
# as the fused step computes it, and the recursion whose triangular solves
# use inverses assembled from the leaves.

def test_leaf_pivot_classes_from_prefix_products():
    """D_k = a_k / (a_0 ... a_(k-1)); its inverse is (a_0 ... a_(k-1)) / a_k and
    its Legendre symbol is that of a_k times those of a_0 .. a_(k-1)."""
    for p in (3, 7, 251, 65537, 131071):
        rng = np.random.default_rng(p)
        a = rng.integers(1, p, size=64)
        g, gi = 1, 1
        for k in range(64):
            ak = int(a[k])
            x = pow(ak, (p - 3) // 2, p)
            ai = x * x % p * ak % p
            assert ai == pow(ak, p - 2, p)
            nra = x * ak % p == p - 1
            below = sum(1 for t in range(k) if oracle.legendre(int(a[t]), p) == -1)
            nr = nra != (below % 2 == 1)
            dk = ak * gi % p
            assert dk * g % p == ak
            assert (oracle.legendre(dk, p) == -1) == nr
            assert ai * g % p == pow(dk, p - 2, p)
            g, gi = g * ak % p, gi * ai % p


def algorithm5_columns(D, p):
    """Column operations (j1, s1, j2, s2) of Abar = L Delta for the pivots D,
    worked out per column as the fused step does: rank of a non-residue from
    the count before it, partner the next or previous non-residue."""
    n1 = len(D)
    s = 2
    while oracle.legendre(s, p) != -1:
        s += 1
    c = oracle.sqrt_mod(s - 1, p)
    sinv = pow(s, p - 2, p)
    flag = [oracle.legendre(int(d), p) == -1 for d in D]
    root = [oracle.sqrt_mod(int(d) * sinv % p if f else int(d), p) for d, f in zip(D, flag)]
    cols = []
    for col in range(n1 + 1):
        if col == n1:
            total = sum(flag)
            if total % 2 == 1:
                i = max(t for t in range(n1) if flag[t])
                cols.append((i, c * root[i] % p, -1, 0))
            else:
                cols.append((-1, 0, -1, 0))
            continue
        if not flag[col]:
            cols.append((col, root[col], -1, 0))
            continue
        rank = sum(flag[:col])
        if rank % 2 == 0:
            nxt = [t for t in range(col + 1, n1) if flag[t]]
            if nxt:
                j = nxt[0]
                cols.append((col, root[col], j, (p - c * root[j] % p) % p))
            else:
                cols.append((col, root[col], -1, 0))
        else:
            i = max(t for t in range(col) if flag[t])
            cols.append((i, c * root[i] % p, col, root[col]))
    return cols


@pytest.mark.parametrize("p", [3, 7, 11, 251, 65537, 131071])
def test_algorithm5_pairing_reproduces_l_d_lt(p):
    """Abar Abar^T = L D L^T for the fused step's pairing (any mix of residues
    and non-residues, odd and even non-residue counts)."""
    rng = np.random.default_rng(p + 5)
    for n1, rows in [(1, 3), (2, 4), (5, 6), (9, 7), (16, 5)]:
        D = rng.integers(1, p, size=n1)
        L = rng.integers(0, p, size=(rows, n1)).astype(object)
        cols = algorithm5_columns(D, p)
        Ab = np.zeros((rows, n1 + 1), dtype=object)
        for q, (j1, s1, j2, s2) in enumerate(cols):
            if j1 >= 0:
                Ab[:, q] += L[:, j1] * s1
            if j2 >= 0:
                Ab[:, q] += L[:, j2] * s2
        lhs = Ab.dot(Ab.T) % p
        rhs = (L * D.astype(object)).dot(L.T) % p
        assert np.array_equal(lhs, rhs), (n1, rows)


def unit_lower_inverse_doubling(L, p):
    """The leaf's inverse of a unit lower triangular matrix of order 2^e:
    [[A, 0], [X, C]]^-1 = [[A^-1, 0], [-C^-1 X A^-1, C^-1]] on blocks of 1, 2, 4..."""
    n = L.shape[0]
    Li = np.eye(n, dtype=object)
    b = 1
    while b < n:
        for a0 in range(0, n, 2 * b):
            c0 = a0 + b
            T = L[c0:c0 + b, a0:a0 + b].dot(Li[a0:a0 + b, a0:a0 + b]) % p
            Li[c0:c0 + b, a0:a0 + b] = (-Li[c0:c0 + b, c0:c0 + b].dot(T)) % p
        b *= 2
    return Li


def test_unit_lower_inverse_by_doubling():
    for p in (3, 65537, 131071):
        rng = np.random.default_rng(p)
        n = 64
        L = np.tril(rng.integers(0, p, size=(n, n)), -1).astype(object)
        L[np.arange(n), np.arange(n)] = 1
        Li = unit_lower_inverse_doubling(L, p)
        assert np.array_equal(L.dot(Li) % p, np.eye(n, dtype=object))


def split_point(n, leaf):
    h = (n + 1) // 2
    return (h + leaf - 1) // leaf * leaf


def ldlt_with_assembled_inverses(S, p, leaf):
    """The recursion of the device driver with leaves of order `leaf`:
    W = S21 L11^-T with L11^-1 assembled from the children's inverses,
    L21 = W D1^-1, S22 -= L21 D1 L21^T; returns (L, D) packed and the
    inverse of the whole unit factor as the recursion builds it."""
    n = S.shape[0]
    A = np.array(S, dtype=object) % p
    Linv = np.zeros((n, n), dtype=object)

    def rec(o, m):
        if m <= leaf:
            blk = A[o:o + m, o:o + m]
            Lb = np.eye(m, dtype=object)
            D = np.zeros(m, dtype=object)
            W = blk.copy()
            for k in range(m):
                D[k] = W[k, k] % p
                if D[k] == 0:
                    raise ZeroDivisionError(o + k + 1)
                inv = pow(int(D[k]), p - 2, p)
                for i in range(k + 1, m):
                    Lb[i, k] = W[i, k] * inv % p
                for i in range(k + 1, m):
                    for j in range(k + 1, i + 1):
                        W[i, j] = (W[i, j] - Lb[i, k] * D[k] * Lb[j, k]) % p
            A[o:o + m, o:o + m] = np.tril(Lb, -1) + np.diag(D)
            Linv[o:o + m, o:o + m] = unit_lower_inverse_doubling(Lb, p) if m & (m - 1) == 0 else \
                np.array([[int(x) for x in r] for r in _inv_unit(Lb, p)], dtype=object)
            return
        n1 = split_point(m, leaf)
        n2 = m - n1
        rec(o, n1)
        I11 = Linv[o:o + n1, o:o + n1]
        W = A[o + n1:o + m, o:o + n1].dot(I11.T) % p
        D1 = np.array([A[o + k, o + k] for k in range(n1)], dtype=object)
        D1inv = np.array([pow(int(d), p - 2, p) for d in D1], dtype=object)
        L21 = W * D1inv % p
        A[o + n1:o + m, o:o + n1] = L21
        T1 = L21.dot(I11) % p
        S22 = A[o + n1:o + m, o + n1:o + m]
        A[o + n1:o + m, o + n1:o + m] = (S22 - (L21 * D1).dot(L21.T)) % p
        rec(o + n1, n2)
        I22 = Linv[o + n1:o + m, o + n1:o + m]
        Linv[o + n1:o + m, o:o + n1] = (-I22.dot(T1)) % p

    rec(0, n)
    return np.tril(A), Linv


def _inv_unit(L, p):
    n = L.shape[0]
    X = np.eye(n, dtype=object)
    for i in range(n):
        for j in range(i):
            X[i, j] = (-sum(L[i, t] * X[t, j] for t in range(j, i))) % p
    return X


@pytest.mark.parametrize("p,n,leaf", [(65537, 37, 4), (131071, 64, 8), (251, 29, 4), (7, 16, 2)])
def test_recursion_with_assembled_inverses_matches_crout(p, n, leaf):
    # S = L D L^T with nonzero pivots (generic rank profile for any p)
    rng = np.random.default_rng(n + p % 97)
    L0 = np.tril(rng.integers(0, p, size=(n, n)), -1).astype(object)
    L0[np.arange(n), np.arange(n)] = 1
    D0 = rng.integers(1, p, size=n).astype(object)
    S = np.array((L0 * D0).dot(L0.T) % p, dtype=np.uint32)
    ref, info = oracle.ldlt_packed(S, p)
    assert info == 0
    got, Linv = ldlt_with_assembled_inverses(S, p, leaf)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(np.array(got, dtype=np.uint64)[low], ref.astype(np.uint64)[low])
    Lunit = np.tril(np.array(got, dtype=object), -1) + np.eye(n, dtype=object)
    assert np.array_equal(Lunit.dot(Linv) % p, np.eye(n, dtype=object))


@pytest.mark.parametrize("p", [3, 251, 65537, 131071, 262139])
def test_lazy_leaf_elimination_stays_exact(p):
    """The leaf's elimination for p < 2^18 in doubles: entries centred, every
    second step left unreduced, pivot and published column always reduced,
    quotients rounded to nearest.  Every intermediate value stays an integer
    below 2^53 (so each product and sum is exact), and the result matches the
    integer recurrence."""
    n = 64
    rng = np.random.default_rng(p)
    S = rng.integers(0, p, size=(n, n))
    S = np.tril(S) + np.tril(S, -1).T
    half = (p - 1) // 2
    M = np.where(S > half, S - p, S).astype(np.float64)
    pd = float(p)
    pinv = 1.0 / pd

    def cred(v):
        return v - np.rint(v * pinv) * pd

    biggest = 0.0
    ref = [[int(S[i][j]) for j in range(n)] for i in range(n)]
    for k in range(n):
        col = M[:, k].copy()
        # the published column is reduced whenever the previous step was lazy
        if k > 0 and (k - 1) % 4 in (0, 2):
            col = cred(col)
        a = col[k]
        assert a == np.rint(a) and abs(a) <= (p + 1) / 2
        if a == 0.0:
            break
        upd = a * M - np.outer(col, col)
        biggest = max(biggest, float(np.max(np.abs(upd[k + 1:, k + 1:]))) if k + 1 < n else 0.0)
        if k % 4 in (1, 3):
            upd = cred(upd)
        mask = np.zeros((n, n), dtype=bool)
        mask[k + 1:, k + 1:] = True
        M = np.where(mask, upd, M)
        ak = ref[k][k]
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                ref[i][j] = (ak * ref[i][j] - ref[i][k] * ref[j][k]) % p
    assert biggest < 2.0 ** 53
    got = np.mod(cred(M), pd).astype(np.int64)
    want = np.array(ref, dtype=np.int64)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(got[low], want[low])
