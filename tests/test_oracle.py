"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests retypes the oracle's formulas: they check it against
brute force on tiny inputs, library routines (numpy matmul on exact integer
or Python-object arrays), closed forms, invariants and the values the paper
prints (Table 5).
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import costmodel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def setup_module(module):
    oracle.build(force=False)


def matmul_exact(X, Y):
    """Exact integer product through numpy's object-array matmul."""
    return np.asarray(X, dtype=object).dot(np.asarray(Y, dtype=object))


def modp(M, p):
    return np.asarray(np.asarray(M, dtype=object) % p, dtype=np.uint64)


def sieve(limit):
    is_p = np.ones(limit, dtype=bool)
    is_p[:2] = False
    for i in range(2, int(limit ** 0.5) + 1):
        if is_p[i]:
            is_p[i * i::i] = False
    return np.nonzero(is_p)[0]


PRIMES_SMALL = [int(q) for q in sieve(600) if q > 2]
PRIMES_16 = [int(q) for q in sieve(1 << 16) if q > 2]


# --------------------------------------------------------------------- field

def test_is_prime_matches_sieve():
    primes = set(int(q) for q in sieve(20000))
    for x in range(20000):
        assert oracle.is_prime(x) == (x in primes), x
    assert oracle.is_prime(4294967291)          # largest prime below 2^32
    assert not oracle.is_prime(65537 * 65521)


def test_legendre_matches_squares_brute_force():
    for p in PRIMES_SMALL[:40]:
        squares = {(x * x) % p for x in range(1, p)}
        for a in range(p):
            expect = 0 if a == 0 else (1 if a in squares else -1)
            assert oracle.legendre(a, p) == expect, (a, p)


def test_sqrt_mod_brute_force_and_canonical():
    for p in PRIMES_SMALL[:60]:
        for a in range(p):
            r = oracle.sqrt_mod(a, p)
            roots = [x for x in range(p) if (x * x) % p == a]
            if roots:
                assert r == min(roots), (a, p)
            else:
                assert r is None


def test_sqrt_closed_forms():
    # 2^16 = -1 mod 65537, so 2^8 is a square root of -1 (Proposition 3.3).
    assert oracle.sqrt_mod(65536, 65537) == 256
    # 2^17 = 1 mod 131071, so (2^9)^2 = 2^18 = 2.
    assert oracle.sqrt_mod(2, 131071) == 512
    # p = 251 = 3 mod 8: -2 is a square (proof of Theorem 4.1); 91^2 = 8281 = 33*251 - 2.
    assert oracle.sqrt_mod(249, 251) == 91
    # p = 3 mod 4: -1 is not a square.
    assert oracle.sqrt_mod(131070, 131071) is None
    assert oracle.sqrt_mod(250, 251) is None


def test_sos_minus_one_every_prime_below_2_16():
    for p in PRIMES_16:
        a, b = oracle.sos(p, p - 1)
        assert (a * a + b * b) % p == p - 1, p
        if p % 4 == 1:
            assert b == 0            # -1 is a square: first branch of Algorithm 3
        else:
            assert b != 0


def test_sos_p3mod8_uses_two_as_smallest_nonresidue():
    # For p = 3 mod 8, 2 is the smallest non-residue, so c = sqrt(1) = 1 and
    # Algorithm 3 returns (a, a) with 2 a^2 = -1.
    for p in [q for q in PRIMES_16 if q % 8 == 3][:200]:
        a, b = oracle.sos(p, p - 1)
        assert a == b and (2 * a * a) % p == p - 1, p


def test_sos_random_targets():
    rng = np.random.default_rng(11)
    for p in [251, 65521, 65537, 131071, 2147483647, 4294967291]:
        for k in rng.integers(0, p, size=50):
            a, b = oracle.sos(p, int(k))
            assert (a * a + b * b) % p == int(k) % p


@pytest.mark.parametrize("p", [251, 65521, 65537, 131071, 131041, 1000003])
def test_skew_orthogonal_y(p):
    # Proposition 3.4: Y = [[a,b],[-b,a]] (x) I_h with a^2+b^2 = -1 gives Y Y^T = -I.
    a, b = oracle.sos(p, p - 1)
    h = 3
    I = np.eye(h, dtype=np.int64)
    Y = np.block([[a * I, b * I], [(p - b) % p * I, a * I]])
    YYt = modp(matmul_exact(Y, Y.T), p)
    assert np.array_equal(YYt, (p - 1) * np.eye(2 * h, dtype=np.uint64))


def test_nrsyf_factors_nonresidue_pairs():
    rng = np.random.default_rng(5)
    for p in [251, 65521, 65537, 131071, 1000003]:
        nonres = [x for x in range(2, min(p, 400)) if oracle.legendre(x, p) == -1]
        for _ in range(20):
            al, be = (int(v) for v in rng.choice(nonres, size=2))
            Y = oracle.nrsyf(p, al, be)
            YYt = modp(matmul_exact(Y, Y.T), p)
            assert YYt.tolist() == [[al, 0], [0, be]], (p, al, be)


def test_nrsyf_rejects_residues():
    with pytest.raises(ValueError):
        oracle.nrsyf(65537, 4, 3)


# ---------------------------------------------------------------- products

def test_syrk_exhaustive_p3_tiny():
    p = 3
    for shape in [(2, 2), (2, 3)]:
        for vals in itertools.product(range(p), repeat=shape[0] * shape[1]):
            A = np.array(vals, dtype=np.uint32).reshape(shape)
            ref = (A.astype(np.int64) @ A.astype(np.int64).T) % p
            assert np.array_equal(oracle.syrk(A, p), ref.astype(np.uint32))


@pytest.mark.parametrize("p", [2, 3, 251, 65521, 65537, 131071, 4294967291])
@pytest.mark.parametrize("n,k", [(1, 1), (7, 3), (5, 11), (16, 16), (33, 70)])
def test_syrk_random_vs_exact_matmul(p, n, k):
    rng = np.random.default_rng(n * 1000 + k)
    A = rng.integers(0, p, size=(n, k), dtype=np.uint64).astype(np.uint32)
    ref = modp(matmul_exact(A, A.T), p).astype(np.uint32)
    C = oracle.syrk(A, p)
    assert np.array_equal(C, ref)
    assert np.array_equal(C, C.T)


@pytest.mark.parametrize("p", [251, 65537, 131071])
def test_syrk_closed_forms(p):
    n, k = 19, 45
    I = np.eye(n, dtype=np.uint32)
    assert np.array_equal(oracle.syrk(I, p), I)
    ones = np.ones((n, k), dtype=np.uint32)
    assert np.all(oracle.syrk(ones, p) == k % p)
    # (p-1)^2 = 1 mod p, so every entry of (-J)(-J)^T is k.
    neg = np.full((n, k), p - 1, dtype=np.uint32)
    assert np.all(oracle.syrk(neg, p) == k % p)
    # Rank one: A = u v^T gives A A^T = (v.v) u u^T.
    rng = np.random.default_rng(1)
    u = rng.integers(0, p, size=n).astype(object)
    v = rng.integers(0, p, size=k).astype(object)
    A = np.array(np.outer(u, v) % p, dtype=np.uint32)
    vv = int(np.dot(v, v))
    expect = np.array((np.outer(u, u) * vv) % p, dtype=np.uint32)
    assert np.array_equal(oracle.syrk(A, p), expect)


def test_syrk_freivalds():
    p = 131071
    rng = np.random.default_rng(2)
    A = rng.integers(0, p, size=(64, 150), dtype=np.uint32)
    C = oracle.syrk(A, p).astype(object)
    for _ in range(3):
        x = rng.integers(0, p, size=64).astype(object)
        lhs = C.dot(x) % p
        rhs = A.astype(object).dot(A.T.astype(object).dot(x)) % p
        assert np.array_equal(lhs, rhs)


def test_syrk_rows_and_entries_agree_with_full():
    p = 65537
    rng = np.random.default_rng(3)
    A = rng.integers(0, p, size=(40, 77), dtype=np.uint32)
    ref = modp(matmul_exact(A, A.T), p).astype(np.uint32)
    R = oracle.syrk_rows(A, p, 10, 25)
    for i in range(10, 25):
        assert np.array_equal(R[i - 10, : i + 1], ref[i, : i + 1])
    rows = rng.integers(0, 40, size=100)
    cols = rng.integers(0, 40, size=100)
    assert np.array_equal(oracle.syrk_entries(A, p, rows, cols), ref[rows, cols])


@pytest.mark.parametrize("p", [251, 65537, 131071, 4294967291])
def test_gemm_alpha_beta_vs_exact_matmul(p):
    rng = np.random.default_rng(p % 1000)
    m, n, k = 13, 21, 37
    A = rng.integers(0, p, size=(m, k), dtype=np.uint64).astype(np.uint32)
    B = rng.integers(0, p, size=(n, k), dtype=np.uint64).astype(np.uint32)
    C = rng.integers(0, p, size=(m, n), dtype=np.uint64).astype(np.uint32)
    alpha, beta = int(rng.integers(0, p)), int(rng.integers(0, p))
    ref = modp(alpha * matmul_exact(A, B.T) + beta * C.astype(object), p).astype(np.uint32)
    assert np.array_equal(oracle.gemm(A, B, p, alpha, beta, C), ref)
    # A B^T differs from B A^T: a transposed operand must show.
    ab = oracle.gemm(A[:, :], A[:5, :], p)
    assert np.array_equal(ab, modp(matmul_exact(A, A[:5].T), p).astype(np.uint32))


@pytest.mark.parametrize("p", [251, 65537, 131071])
def test_syrk_ab_lower_only(p):
    rng = np.random.default_rng(7)
    n, k = 23, 17
    A = rng.integers(0, p, size=(n, k), dtype=np.uint32)
    C = rng.integers(0, p, size=(n, n), dtype=np.uint32)
    alpha, beta = p - 1, 1
    out = oracle.syrk_ab(A, p, alpha, beta, C)
    full = modp(alpha * matmul_exact(A, A.T) + beta * C.astype(object), p).astype(np.uint32)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(out[low], full[low])
    assert np.array_equal(out[~low], C[~low])


def test_syrkd_vs_exact_matmul():
    p = 65537
    rng = np.random.default_rng(9)
    A = rng.integers(0, p, size=(12, 9), dtype=np.uint32)
    d = rng.integers(0, p, size=9, dtype=np.uint32)
    ref = modp(matmul_exact(A.astype(object) * d.astype(object), A.T), p).astype(np.uint32)
    assert np.array_equal(oracle.syrkd(A, d, p), ref)


# ------------------------------------------------------------------- LDL^T

def _random_ldl(n, p, seed):
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(0, p, size=(n, n), dtype=np.uint64), -1).astype(object)
    L[np.arange(n), np.arange(n)] = 1
    D = rng.integers(1, p, size=n).astype(object)
    S = (L * D).dot(L.T) % p
    return L, D, np.array(S, dtype=np.uint32)


@pytest.mark.parametrize("p", [251, 65537, 131071])
@pytest.mark.parametrize("n", [1, 2, 9, 40])
def test_ldlt_recovers_constructed_factors(p, n):
    L0, D0, S = _random_ldl(n, p, seed=n + p)
    L, D, info = oracle.ldlt(S, p)
    assert info == 0
    assert np.array_equal(L.astype(object), L0)
    assert np.array_equal(D.astype(object), D0)


def test_ldlt_reconstruction_random_symmetric():
    from paper_2001_04109_amd import inputs
    p = 65537
    S = inputs.symmetric(21, 50, p)
    L, D, info = oracle.ldlt(S, p)
    assert info == 0
    R = modp((L.astype(object) * D.astype(object)).dot(L.T.astype(object)), p)
    assert np.array_equal(R.astype(np.uint32), S)


def test_ldlt_zero_pivots():
    p = 251
    S = np.array([[0, 3], [3, 5]], dtype=np.uint32)
    assert oracle.ldlt(S, p)[2] == 1
    # leading 2x2 minor 1*4 - 2*2 = 0 -> second pivot vanishes
    S = np.array([[1, 2, 7], [2, 4, 1], [7, 1, 9]], dtype=np.uint32)
    assert oracle.ldlt(S, p)[2] == 2


def test_ldlt_exhaustive_p3_2x2():
    p = 3
    for a, b, c in itertools.product(range(p), repeat=3):
        S = np.array([[a, b], [b, c]], dtype=np.uint32)
        L, D, info = oracle.ldlt(S, p)
        det = (a * c - b * b) % p
        if a == 0:
            assert info == 1
        elif det == 0:
            assert info == 2
        else:
            assert info == 0
            R = (L.astype(np.int64) * D.astype(np.int64)) @ L.T.astype(np.int64) % p
            assert np.array_equal(R, S.astype(np.int64))


# -------------------------------------------------------------- cost model

def _table5():
    rows = {}
    with open(os.path.join(GOLDEN, "table5.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            rows[parts[0]] = [None if v == "-" else int(v) for v in parts[1:]]
    return rows


def test_costmodel_reproduces_table5():
    ns = [4, 8, 16, 32, 64, 128]
    rows = _table5()
    for label, vals in rows.items():
        for n, v in zip(ns, vals):
            if v is None:
                continue
            if label == "syrk":
                got = costmodel.syrk(n)
            elif label.startswith("Syrk-"):
                got = costmodel.syrk_dc(int(label[5:]), n)
            else:
                y, r = int(label[1]), int(label[3:])
                got = costmodel.alg2(y, r, n)
            assert got == v, (label, n, got, v)


def test_costmodel_leading_term_table1():
    # Table 1: 0.8 n^3 with classical general products; t_d -> 0.8.
    assert costmodel.mac_fraction(1) == 0.875
    assert abs(float(costmodel.mac_fraction(40)) - 0.8) < 1e-12
    # ratio of Gy-i to the classical count approaches 0.8 for deep recursion
    n = 1 << 14
    ratio = costmodel.alg2(1, 12, n) / costmodel.syrk(n)
    assert ratio < 0.85


def test_costmodel_additions_remark_4_2():
    # 9 block additions: 6 full m x m and 3 half (lower-triangle) ones.
    for m in [1, 2, 5, 64]:
        assert costmodel.additions_per_level(m) == 6 * m * m + 3 * m * (m + 1) // 2
        assert costmodel.additions_per_level(m) * 2 == 15 * m * m + 3 * m


def test_costmodel_y_constants():
    assert costmodel.y_cost(65537) == 1
    assert costmodel.y_cost(251) == 2       # 251 = 3 mod 8
    assert costmodel.y_cost(131071) == 3    # 131071 = 7 mod 8


# ------------------------------------------- Algorithm 6 (block diagonal B)

def dense_tridiagonal(bdiag, boff):
    n = len(bdiag)
    B = np.zeros((n, n), dtype=object)
    for l in range(n):
        B[l, l] = int(bdiag[l])
    for l in range(n - 1):
        B[l, l + 1] = B[l + 1, l] = int(boff[l])
    return B


def random_block_diagonal(rng, n, p, two_by_two=0.5, char2_gamma=False):
    """Scalar blocks and 2x2 blocks [[0, b], [b, g]] (g = 0 unless char2_gamma)."""
    bdiag = rng.integers(0, p, size=n, dtype=np.uint64).astype(np.uint32)
    boff = np.zeros(max(n - 1, 0), dtype=np.uint32)
    j = 0
    while j < n:
        if j + 1 < n and rng.random() < two_by_two:
            boff[j] = rng.integers(1, p)
            bdiag[j] = 0
            bdiag[j + 1] = rng.integers(0, p) if char2_gamma else 0
            j += 2
        else:
            j += 1
    return bdiag, boff


@pytest.mark.parametrize("p", [2, 3, 7, 251, 65537, 94906249])
def test_syrkbd_vs_dense_exact_matmul(p):
    rng = np.random.default_rng(p)
    for m, n in [(1, 1), (4, 3), (9, 8), (17, 30)]:
        A = rng.integers(0, p, size=(m, n), dtype=np.uint64).astype(np.uint32)
        bdiag = rng.integers(0, p, size=n, dtype=np.uint64).astype(np.uint32)
        boff = rng.integers(0, p, size=max(n - 1, 0), dtype=np.uint64).astype(np.uint32)
        B = dense_tridiagonal(bdiag, boff)
        expect = modp(matmul_exact(matmul_exact(A, B), A.T), p)
        assert np.array_equal(oracle.syrkbd(A, bdiag, boff, p), expect)
        C0 = rng.integers(0, p, size=(m, m), dtype=np.uint64).astype(np.uint32)
        al, be = int(rng.integers(0, p)), int(rng.integers(0, p))
        got = oracle.syrkbd(A, bdiag, boff, p, al, be, C0)
        assert np.array_equal(got, modp(al * matmul_exact(matmul_exact(A, B), A.T) + be * C0.astype(object), p))


def test_syrkbd_exhaustive_p3_tiny():
    p = 3
    for vals in itertools.product(range(p), repeat=4):       # A is 2 x 2
        A = np.array(vals, dtype=np.uint32).reshape(2, 2)
        for b0, b1, e in itertools.product(range(p), repeat=3):
            B = np.array([[b0, e], [e, b1]], dtype=object)
            expect = modp(matmul_exact(matmul_exact(A, B), A.T), p)
            got = oracle.syrkbd(A, [b0, b1], [e], p)
            assert np.array_equal(got, expect)


@pytest.mark.parametrize("p", [65537, 131071, 251])
def test_syrkbd_reduces_to_syrkd_by_the_antidiagonal_factorisation(p):
    """Section 5.2: [[0, b], [b, 0]] = T diag(b/2, -b/2) T^T with
    T = [[1, 1], [1, -1]]: A B A^T equals syrkd of A T with those scalars."""
    rng = np.random.default_rng(5 + p)
    m, n = 13, 10
    bdiag, boff = random_block_diagonal(rng, n, p)
    A = rng.integers(0, p, size=(m, n), dtype=np.uint64).astype(np.uint32)
    AT = A.astype(np.int64).copy()
    d = bdiag.astype(np.int64).copy()
    half = (p + 1) // 2
    for j in range(n - 1):
        if boff[j]:
            b = int(boff[j])
            AT[:, j] = (A[:, j].astype(np.int64) + A[:, j + 1]) % p
            AT[:, j + 1] = (A[:, j].astype(np.int64) - A[:, j + 1]) % p
            d[j] = b * half % p
            d[j + 1] = (p - b * half % p) % p
    got = oracle.syrkbd(A, bdiag, boff, p)
    assert np.array_equal(got, oracle.syrkd(AT.astype(np.uint32), d.astype(np.uint32), p))
    # a diagonal B is Algorithm 5's D
    assert np.array_equal(oracle.syrkbd(A, bdiag, np.zeros(n - 1, np.uint32), p), oracle.syrkd(A, bdiag, p))


def test_characteristic_two_factorisations():
    """Section 5.2's identities in characteristic 2 (F_2): the antitriangular
    block, the antidiagonal block with one extra column, and the
    combination of a scalar block x with an antidiagonal block."""
    p = 2
    tri = np.array([[1, 1], [1, 0]], dtype=object)
    for g in (1,):                      # [[0, 1], [1, g]], gamma != 0; delta = sqrt(g) = 1
        F = matmul_exact(np.array([[1, 0], [0, 1]], dtype=object), tri)
        assert np.array_equal(modp(matmul_exact(F, F.T), p), np.array([[0, 1], [1, g]]))
    F = np.array([[1, 0, 1], [0, 1, 1]], dtype=object)
    assert np.array_equal(modp(matmul_exact(F, F.T), p), np.array([[0, 1], [1, 0]]))
    for x in (0, 1):
        F = np.array([[x, x, x], [1, 0, 1], [0, 1, 1]], dtype=object)
        assert np.array_equal(modp(matmul_exact(F, F.T), p), np.array([[x, 0, 0], [0, 0, 1], [0, 1, 0]]))


# ------------------------------------- products over F_p[i] (Sections 3, 4.1)

def cmul(a, b, p):
    return ((a[0] * b[0] - a[1] * b[1]) % p, (a[0] * b[1] + a[1] * b[0]) % p)


def brute_complex(re, im, p, conj):
    n, k = re.shape
    Cr = np.zeros((n, n), dtype=np.uint64)
    Ci = np.zeros((n, n), dtype=np.uint64)
    for j in range(n):
        for l in range(n):
            acc = (0, 0)
            for t in range(k):
                a = (int(re[j, t]), int(im[j, t]))
                b = (int(re[l, t]), (p - int(im[l, t])) % p if conj else int(im[l, t]))
                c = cmul(a, b, p)
                acc = ((acc[0] + c[0]) % p, (acc[1] + c[1]) % p)
            Cr[j, l], Ci[j, l] = acc
    return Cr, Ci


@pytest.mark.parametrize("p", [3, 7, 131071, 94906247])
def test_herk_and_zsyrk_brute_force(p):
    rng = np.random.default_rng(p)
    for n, k in [(1, 1), (3, 2), (6, 7)]:
        re = rng.integers(0, p, size=(n, k), dtype=np.uint64).astype(np.uint32)
        im = rng.integers(0, p, size=(n, k), dtype=np.uint64).astype(np.uint32)
        for fn, conj in ((oracle.herk, True), (oracle.zsyrk, False)):
            Cr, Ci = fn(re, im, p)
            er, ei = brute_complex(re, im, p, conj)
            assert np.array_equal(Cr, er) and np.array_equal(Ci, ei), (fn.__name__, n, k)


@pytest.mark.parametrize("p", [7, 131071])
def test_herk_and_zsyrk_structure(p):
    rng = np.random.default_rng(3 * p)
    n, k = 9, 11
    re = rng.integers(0, p, size=(n, k), dtype=np.uint64).astype(np.uint32)
    im = rng.integers(0, p, size=(n, k), dtype=np.uint64).astype(np.uint32)
    Hr, Hi = oracle.herk(re, im, p)
    assert np.array_equal(Hr, Hr.T)                          # Hermitian: Re symmetric,
    assert np.array_equal(Hi, (p - Hi.T.astype(np.int64)) % p)   # Im skew-symmetric
    assert not Hi.diagonal().any()                           # real diagonal
    Zr, Zi = oracle.zsyrk(re, im, p)
    assert np.array_equal(Zr, Zr.T) and np.array_equal(Zi, Zi.T)
    zero = np.zeros_like(re)
    # a real A: both are A A^T; A = i B: A A^H = B B^T, A A^T = -B B^T
    for fn in (oracle.herk, oracle.zsyrk):
        r, i = fn(re, zero, p)
        assert np.array_equal(r, oracle.syrk(re, p)) and not i.any()
    r, i = oracle.herk(zero, im, p)
    assert np.array_equal(r, oracle.syrk(im, p)) and not i.any()
    r, i = oracle.zsyrk(zero, im, p)
    assert np.array_equal(r, (p - oracle.syrk(im, p).astype(np.int64)) % p) and not i.any()
    # rank one: C_jl = u_j conj(u_l)
    u = (re[:, :1], im[:, :1])
    r, i = oracle.herk(u[0], u[1], p)
    for j in range(n):
        for l in range(n):
            c = cmul((int(u[0][j, 0]), int(u[1][j, 0])), (int(u[0][l, 0]), (p - int(u[1][l, 0])) % p), p)
            assert (int(r[j, l]), int(i[j, l])) == c
