/*
 * ffp_oracle.c -- CPU oracle for exact symmetric products over Z/pZ.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the GPU path against a plain,
 * slow, obviously correct computation.  It shares no code, header or table
 * with the HIP path.
 *
 * Every function states the passage of Dumas, Pernet and Sedoglavic,
 * "On Fast Multiplication of a Matrix by its Transpose" (ISSAC 2020,
 * arXiv:2001.04109) that defines what it computes.  Where the paper's
 * method reaches a result with a plain definition (the product A*A^T mod p,
 * Proposition 3.2), the oracle is that definition written out with exact
 * 128-bit accumulation and a single reduction.  Where the paper gives an
 * algorithm whose output is not unique (Algorithm 3 SoS, Algorithm 4
 * nrsyf), the oracle follows the algorithm's steps in the paper's order.
 *
 * Conventions: matrices are row-major with a leading dimension in elements;
 * residues are uint32 in [0,p); p < 2^32.  Return value 0 = OK, <0 = bad
 * argument.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

typedef unsigned __int128 u128;

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)

/* ---------------------------------------------------------------------- */
/* Scalar field arithmetic (Section 3.1, Propositions 3.3-3.5)             */
/* ---------------------------------------------------------------------- */

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p)
{
    return (uint64_t)(((u128)a * b) % p);
}

uint64_t oracle_powmod(uint64_t a, uint64_t e, uint64_t p)
{
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = mulmod(r, a, p);
        a = mulmod(a, a, p);
        e >>= 1;
    }
    return r;
}

/* Primality by trial division: plain and obviously correct for p < 2^32. */
int oracle_is_prime(uint64_t p)
{
    if (p < 2) return 0;
    for (uint64_t d = 2; d * d <= p; ++d)
        if (p % d == 0) return 0;
    return 1;
}

/* Legendre symbol (a/p) for odd prime p by Euler's criterion:
 * returns 0 if p | a, 1 if a is a nonzero square, -1 otherwise. */
int oracle_legendre(uint64_t a, uint64_t p)
{
    a %= p;
    if (a == 0) return 0;
    uint64_t t = oracle_powmod(a, (p - 1) / 2, p);
    return t == 1 ? 1 : -1;
}

uint64_t oracle_inv(uint64_t a, uint64_t p)
{
    /* Fermat: a^(p-2) is the inverse of a nonzero a modulo a prime p. */
    return oracle_powmod(a, p - 2, p);
}

/* Square root modulo an odd prime (the "sqrt" of Algorithm 3) by the
 * Tonelli-Shanks method.  Returns the canonical root min(r, p-r), or
 * UINT64_MAX if a is not a square.  p = 2 returns a mod 2. */
uint64_t oracle_sqrt_mod(uint64_t a, uint64_t p)
{
    a %= p;
    if (p == 2) return a;
    if (a == 0) return 0;
    if (oracle_legendre(a, p) != 1) return UINT64_MAX;
    /* p - 1 = q * 2^s with q odd */
    uint64_t q = p - 1, s = 0;
    while ((q & 1) == 0) { q >>= 1; ++s; }
    /* z: any quadratic non-residue */
    uint64_t z = 2;
    while (oracle_legendre(z, p) != -1) ++z;
    uint64_t m = s;
    uint64_t c = oracle_powmod(z, q, p);
    uint64_t t = oracle_powmod(a, q, p);
    uint64_t r = oracle_powmod(a, (q + 1) / 2, p);
    while (t != 1) {
        /* least i with t^(2^i) = 1 */
        uint64_t i = 0, tt = t;
        while (tt != 1) { tt = mulmod(tt, tt, p); ++i; }
        uint64_t b = c;
        for (uint64_t j = 0; j + 1 < m - i; ++j) b = mulmod(b, b, p);
        m = i;
        c = mulmod(b, b, p);
        t = mulmod(t, c, p);
        r = mulmod(r, b, p);
    }
    return r < p - r ? r : p - r;
}

/* Algorithm 3 (SoS): (a,b) with a^2 + b^2 = k mod p, for an odd prime p.
 * Follows the algorithm's steps: if k is a square return (sqrt(k), 0);
 * otherwise take the smallest non-residue s, c = sqrt(s-1), r = k/s,
 * a = sqrt(r), and return (a, a*c).  k = 0 is a square (0 = 0^2 + 0^2). */
int oracle_sos(uint64_t p, uint64_t k, uint64_t* a_out, uint64_t* b_out)
{
    if (p < 3 || !oracle_is_prime(p)) return ORACLE_EINVAL;
    k %= p;
    if (k == 0 || oracle_legendre(k, p) == 1) {
        *a_out = oracle_sqrt_mod(k, p);
        *b_out = 0;
        return ORACLE_OK;
    }
    uint64_t s = 2;
    while (oracle_legendre(s, p) == 1) ++s;
    uint64_t c = oracle_sqrt_mod(s - 1, p);
    uint64_t r = mulmod(k, oracle_inv(s, p), p);
    uint64_t a = oracle_sqrt_mod(r, p);
    *a_out = a;
    *b_out = mulmod(a, c, p);
    return ORACLE_OK;
}

/* Algorithm 4 (nrsyf): for two quadratic non-residues alpha, beta return
 * Y = [[a,b],[c,d]] (row-major in Y[4]) with Y*Y^T = diag(alpha, beta). */
int oracle_nrsyf(uint64_t p, uint64_t alpha, uint64_t beta, uint64_t Y[4])
{
    alpha %= p; beta %= p;
    if (oracle_legendre(alpha, p) != -1 || oracle_legendre(beta, p) != -1)
        return ORACLE_EINVAL;
    uint64_t a, b;
    if (oracle_sos(p, alpha, &a, &b) != ORACLE_OK) return ORACLE_EINVAL;
    /* alpha is a non-residue, so SoS took the non-square branch and a != 0 */
    uint64_t q = mulmod(beta, oracle_inv(alpha, p), p);
    uint64_t d = mulmod(a, oracle_sqrt_mod(q, p), p);
    uint64_t c = (p - mulmod(mulmod(b, d, p), oracle_inv(a, p), p)) % p;
    Y[0] = a; Y[1] = b; Y[2] = c; Y[3] = d;
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Products (Algorithm 2 Ensure; Table 4 operation; Section 5)            */
/* ---------------------------------------------------------------------- */

/* C = A * A^T mod p, the full symmetric n x n result (Algorithm 2 Ensure,
 * exact by Proposition 3.2).  A is n x k. */
int oracle_syrk(int64_t n, int64_t k, uint64_t p, const uint32_t* A, int64_t lda,
                uint32_t* C, int64_t ldc)
{
    if (n < 0 || k < 0 || p < 2 || (n > 0 && (lda < k || ldc < n)))
        return ORACLE_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t* ai = A + i * lda;
        for (int64_t j = 0; j <= i; ++j) {
            const uint32_t* aj = A + j * lda;
            u128 s = 0;
            for (int64_t l = 0; l < k; ++l)
                s += (u128)((uint64_t)ai[l] * (uint64_t)aj[l]);
            uint32_t v = (uint32_t)(s % p);
            C[i * ldc + j] = v;
            C[j * ldc + i] = v;
        }
    }
    return ORACLE_OK;
}

/* Rows [i0, i1) of the lower triangle of A * A^T mod p (row-panel form of
 * oracle_syrk, used to time or check a bounded sample of a large product).
 * out is (i1-i0) x ldo; entries with column > row are left untouched. */
int oracle_syrk_rows(int64_t n, int64_t k, uint64_t p, const uint32_t* A, int64_t lda,
                     int64_t i0, int64_t i1, uint32_t* out, int64_t ldo)
{
    if (n < 0 || k < 0 || p < 2 || i0 < 0 || i1 > n || i0 > i1 || lda < k || ldo < i1)
        return ORACLE_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = i0; i < i1; ++i) {
        const uint32_t* ai = A + i * lda;
        for (int64_t j = 0; j <= i; ++j) {
            const uint32_t* aj = A + j * lda;
            u128 s = 0;
            for (int64_t l = 0; l < k; ++l)
                s += (u128)((uint64_t)ai[l] * (uint64_t)aj[l]);
            out[(i - i0) * ldo + j] = (uint32_t)(s % p);
        }
    }
    return ORACLE_OK;
}

/* Single entries of A * A^T mod p at (rows[t], cols[t]); for sampled checks
 * of products too large for the full oracle. */
int oracle_syrk_entries(int64_t n, int64_t k, uint64_t p, const uint32_t* A, int64_t lda,
                        int64_t npts, const int64_t* rows, const int64_t* cols, uint32_t* out)
{
    if (n < 0 || k < 0 || p < 2 || lda < k) return ORACLE_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < npts; ++t) {
        const uint32_t* ai = A + rows[t] * lda;
        const uint32_t* aj = A + cols[t] * lda;
        u128 s = 0;
        for (int64_t l = 0; l < k; ++l)
            s += (u128)((uint64_t)ai[l] * (uint64_t)aj[l]);
        out[t] = (uint32_t)(s % p);
    }
    return ORACLE_OK;
}

/* C <- (alpha * A * B^T + beta * C) mod p, A is m x k, B is n x k, C is m x n.
 * This is the general product of Algorithm 2 (P3 and P4) in the accumulate
 * form of Table 4. */
int oracle_gemm(int64_t m, int64_t n, int64_t k, uint64_t p,
                const uint32_t* A, int64_t lda, const uint32_t* B, int64_t ldb,
                uint64_t alpha, uint64_t beta, uint32_t* C, int64_t ldc)
{
    if (m < 0 || n < 0 || k < 0 || p < 2 || (m > 0 && ldc < n) || lda < k || ldb < k)
        return ORACLE_EINVAL;
    alpha %= p; beta %= p;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            u128 s = 0;
            for (int64_t l = 0; l < k; ++l)
                s += (u128)((uint64_t)A[i * lda + l] * (uint64_t)B[j * ldb + l]);
            u128 v = (u128)alpha * (uint64_t)(s % p) + (u128)beta * C[i * ldc + j];
            C[i * ldc + j] = (uint32_t)(v % p);
        }
    }
    return ORACLE_OK;
}

/* lower(C) <- (alpha * A * A^T + beta * lower(C)) mod p (the operation of
 * Table 4).  Entries strictly above the diagonal are left untouched. */
int oracle_syrk_ab(int64_t n, int64_t k, uint64_t p, const uint32_t* A, int64_t lda,
                   uint64_t alpha, uint64_t beta, uint32_t* C, int64_t ldc)
{
    if (n < 0 || k < 0 || p < 2 || (n > 0 && (lda < k || ldc < n)))
        return ORACLE_EINVAL;
    alpha %= p; beta %= p;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j <= i; ++j) {
            u128 s = 0;
            for (int64_t l = 0; l < k; ++l)
                s += (u128)((uint64_t)A[i * lda + l] * (uint64_t)A[j * lda + l]);
            u128 v = (u128)alpha * (uint64_t)(s % p) + (u128)beta * C[i * ldc + j];
            C[i * ldc + j] = (uint32_t)(v % p);
        }
    }
    return ORACLE_OK;
}

/* C = A * D * A^T mod p with D = diag(d) (the Ensure of Algorithm 5),
 * full symmetric m x m result; A is m x n. */
int oracle_syrkd(int64_t m, int64_t n, uint64_t p, const uint32_t* A, int64_t lda,
                 const uint32_t* d, uint32_t* C, int64_t ldc)
{
    if (m < 0 || n < 0 || p < 2 || (m > 0 && (lda < n || ldc < m))) return ORACLE_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j <= i; ++j) {
            u128 s = 0;
            for (int64_t l = 0; l < n; ++l)
                s += (u128)mulmod(A[i * lda + l], d[l], p) * A[j * lda + l];
            uint32_t v = (uint32_t)(s % p);
            C[i * ldc + j] = v;
            C[j * ldc + i] = v;
        }
    }
    return ORACLE_OK;
}

/* C <- (alpha * A * B * A^T + beta * C) mod p, the Ensure of Algorithm 6
 * (syrkd with block diagonal scaling, Section 5.2), full symmetric m x m
 * result; A is m x n.  B is the symmetric tridiagonal n x n matrix with
 * diagonal bdiag[0..n) and off-diagonal B[l][l+1] = B[l+1][l] = boff[l]
 * (l < n-1); the block diagonal matrices of Algorithm 6 (scalar blocks and
 * 2 x 2 blocks [[0, beta], [beta, gamma]]) are of this form.  The plain
 * definition: C_ij = sum_l A_il (B A^T)_lj. */
int oracle_syrkbd(int64_t m, int64_t n, uint64_t p, const uint32_t* A, int64_t lda,
                  const uint32_t* bdiag, const uint32_t* boff, uint64_t alpha, uint64_t beta,
                  uint32_t* C, int64_t ldc)
{
    if (m < 0 || n < 0 || p < 2 || (m > 0 && (lda < n || ldc < m))) return ORACLE_EINVAL;
    alpha %= p; beta %= p;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j <= i; ++j) {
            u128 s = 0;
            for (int64_t l = 0; l < n; ++l) {
                /* (B A^T)_lj = B_ll A_jl + B_l,l+1 A_j,l+1 + B_l,l-1 A_j,l-1 */
                u128 t = (u128)bdiag[l] * A[j * lda + l];
                if (l + 1 < n) t += (u128)boff[l] * A[j * lda + l + 1];
                if (l > 0) t += (u128)boff[l - 1] * A[j * lda + l - 1];
                s += (u128)A[i * lda + l] * (uint64_t)(t % p);
            }
            uint64_t prod = (uint64_t)(s % p);
            u128 vij = (u128)alpha * prod + (u128)beta * C[i * ldc + j];
            u128 vji = (u128)alpha * prod + (u128)beta * C[j * ldc + i];
            C[i * ldc + j] = (uint32_t)(vij % p);
            if (j != i) C[j * ldc + i] = (uint32_t)(vji % p);
        }
    }
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Products over F_p[i] = F_p[x]/(x^2 + 1), the field F_{p^2} for p = 3 mod 4 */
/* (Section 3.1 "Over the complex field", Section 3.3, Section 4.1)        */
/* ---------------------------------------------------------------------- */

/* An element a + i b is held as two residues (a, b); a matrix as two
 * planes, re at X and im at X + plane (same leading dimension). */

/* C = A * A^H mod p with A^H the conjugate transpose, conj(a + i b) =
 * a - i b (Section 3.3), full n x n result:
 *   C_jl = sum_t (x_jt + i y_jt)(x_lt - i y_lt)
 *        = sum_t (x_jt x_lt + y_jt y_lt) + i sum_t (y_jt x_lt - x_jt y_lt). */
int oracle_herk(int64_t n, int64_t k, uint64_t p, const uint32_t* A, int64_t lda, int64_t aplane,
                uint32_t* C, int64_t ldc, int64_t cplane)
{
    if (n < 0 || k < 0 || p < 2 || (n > 0 && (lda < k || ldc < n))) return ORACLE_EINVAL;
    const uint32_t* X = A;
    const uint32_t* Y = A + aplane;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t l = 0; l < n; ++l) {
            u128 re = 0, im_pos = 0, im_neg = 0;
            for (int64_t t = 0; t < k; ++t) {
                const uint64_t xj = X[j * lda + t], yj = Y[j * lda + t];
                const uint64_t xl = X[l * lda + t], yl = Y[l * lda + t];
                re += (u128)(xj * xl) + (u128)(yj * yl);
                im_pos += (u128)(yj * xl);
                im_neg += (u128)(xj * yl);
            }
            C[j * ldc + l] = (uint32_t)(re % p);
            C[cplane + j * ldc + l] = (uint32_t)(((uint64_t)(im_pos % p) + p - (uint64_t)(im_neg % p)) % p);
        }
    }
    return ORACLE_OK;
}

/* C = A * A^T mod p over F_p[i] (transposition without conjugation: the
 * complex symmetric product of Section 3.1), full n x n result:
 *   C_jl = sum_t (x_jt x_lt - y_jt y_lt) + i sum_t (x_jt y_lt + y_jt x_lt). */
int oracle_zsyrk(int64_t n, int64_t k, uint64_t p, const uint32_t* A, int64_t lda, int64_t aplane,
                 uint32_t* C, int64_t ldc, int64_t cplane)
{
    if (n < 0 || k < 0 || p < 2 || (n > 0 && (lda < k || ldc < n))) return ORACLE_EINVAL;
    const uint32_t* X = A;
    const uint32_t* Y = A + aplane;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t l = 0; l < n; ++l) {
            u128 re_pos = 0, re_neg = 0, im = 0;
            for (int64_t t = 0; t < k; ++t) {
                const uint64_t xj = X[j * lda + t], yj = Y[j * lda + t];
                const uint64_t xl = X[l * lda + t], yl = Y[l * lda + t];
                re_pos += (u128)(xj * xl);
                re_neg += (u128)(yj * yl);
                im += (u128)(xj * yl) + (u128)(yj * xl);
            }
            C[j * ldc + l] = (uint32_t)(((uint64_t)(re_pos % p) + p - (uint64_t)(re_neg % p)) % p);
            C[cplane + j * ldc + l] = (uint32_t)(im % p);
        }
    }
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Symmetric factorisation S = L * D * L^T (Section 5's use of the product) */
/* ---------------------------------------------------------------------- */

/* Textbook column-by-column (Crout) LDL^T without pivoting, mod an odd
 * prime p.  On entry the lower triangle of S (n x n) holds the symmetric
 * matrix; on exit its strictly lower part holds the unit lower triangular L
 * and its diagonal holds D.  The upper triangle is not read or written.
 *   D_j  = S_jj - sum_{l<j} L_jl^2 D_l
 *   L_ij = (S_ij - sum_{l<j} L_il L_jl D_l) / D_j        (i > j)
 * *info = 0 on success, or j+1 for the first zero pivot D_j (the matrix
 * has no generic rank profile); the factorisation stops there.  The
 * factorisation is unique when every leading principal minor is nonzero. */
int oracle_ldlt(int64_t n, uint64_t p, uint32_t* S, int64_t lds, int64_t* info)
{
    if (n < 0 || p < 3 || (n > 0 && lds < n)) return ORACLE_EINVAL;
    *info = 0;
    for (int64_t j = 0; j < n; ++j) {
        u128 s = 0;
        for (int64_t l = 0; l < j; ++l) {
            uint64_t ljl = S[j * lds + l];
            s += (u128)mulmod(ljl, ljl, p) * S[l * lds + l];
        }
        uint64_t dj = (S[j * lds + j] + p - (uint64_t)(s % p)) % p;
        if (dj == 0) { *info = j + 1; return ORACLE_OK; }
        S[j * lds + j] = (uint32_t)dj;
        uint64_t dinv = oracle_inv(dj, p);
        /* column j of L: W_l = L_jl * D_l is shared by every row i > j */
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            u128 t = 0;
            for (int64_t l = 0; l < j; ++l)
                t += (u128)mulmod(S[i * lds + l], S[j * lds + l], p) * S[l * lds + l];
            uint64_t v = (S[i * lds + j] + p - (uint64_t)(t % p)) % p;
            S[i * lds + j] = (uint32_t)mulmod(v, dinv, p);
        }
    }
    return ORACLE_OK;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (timing of the oracle itself). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
