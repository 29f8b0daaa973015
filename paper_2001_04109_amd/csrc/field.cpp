// Prime-field scalar routines (Section 3.1 of the paper) for the host side
// of the product library.
#include "field.h"

#include <cstdint>

namespace ffp {

static inline uint64_t mul_mod(uint64_t a, uint64_t b, uint64_t p)
{
    return (uint64_t)((unsigned __int128)a * b % p);
}

uint64_t pow_mod(uint64_t a, uint64_t e, uint64_t p)
{
    uint64_t result = 1 % p, base = a % p;
    for (; e; e >>= 1) {
        if (e & 1) result = mul_mod(result, base, p);
        base = mul_mod(base, base, p);
    }
    return result;
}

uint64_t inv_mod(uint64_t a, uint64_t p)
{
    // extended Euclid on (a mod p, p)
    int64_t r0 = (int64_t)p, r1 = (int64_t)(a % p), s0 = 0, s1 = 1;
    while (r1 != 0) {
        int64_t q = r0 / r1, t;
        t = r0 - q * r1; r0 = r1; r1 = t;
        t = s0 - q * s1; s0 = s1; s1 = t;
    }
    if (r0 != 1) return 0;  // not invertible
    return (uint64_t)(s0 < 0 ? s0 + (int64_t)p : s0);
}

// Deterministic Miller-Rabin: bases 2, 7, 61 decide every n < 2^32.
bool is_prime_u32(uint64_t n)
{
    if (n < 2) return false;
    static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 61};
    for (uint64_t q : small) {
        if (n == q) return true;
        if (n % q == 0) return false;
    }
    if (n >= (1ull << 32)) return false;  // outside the supported range
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (uint64_t a : {2ull, 7ull, 61ull}) {
        uint64_t x = pow_mod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool composite = true;
        for (int r = 1; r < s; ++r) {
            x = mul_mod(x, x, n);
            if (x == n - 1) { composite = false; break; }
        }
        if (composite) return false;
    }
    return true;
}

int legendre(uint64_t a, uint64_t p)
{
    // Jacobi symbol (a/p) by quadratic reciprocity; equals the Legendre
    // symbol for prime p.
    uint64_t x = a % p, n = p;
    int sign = 1;
    while (x != 0) {
        while ((x & 1) == 0) {
            x >>= 1;
            uint64_t r = n & 7;
            if (r == 3 || r == 5) sign = -sign;
        }
        uint64_t t = x; x = n; n = t;
        if ((x & 3) == 3 && (n & 3) == 3) sign = -sign;
        x %= n;
    }
    return n == 1 ? sign : 0;
}

uint64_t sqrt_mod(uint64_t a, uint64_t p)
{
    a %= p;
    if (a == 0) return 0;
    if (p == 2) return a;
    if (legendre(a, p) != 1) return UINT64_MAX;
    // Cipolla: find t with t^2 - a a non-residue, then
    // (t + w)^((p+1)/2) in F_p[w]/(w^2 - (t^2 - a)) is a root.
    uint64_t t = 0, w2 = 0;
    for (t = 0; t < p; ++t) {
        w2 = (mul_mod(t, t, p) + p - a) % p;
        if (legendre(w2, p) == -1) break;
    }
    uint64_t r0 = 1, r1 = 0;         // result  r0 + r1 w
    uint64_t b0 = t, b1 = 1;         // base    b0 + b1 w
    for (uint64_t e = (p + 1) / 2; e; e >>= 1) {
        if (e & 1) {
            uint64_t n0 = (mul_mod(r0, b0, p) + mul_mod(mul_mod(r1, b1, p), w2, p)) % p;
            uint64_t n1 = (mul_mod(r0, b1, p) + mul_mod(r1, b0, p)) % p;
            r0 = n0; r1 = n1;
        }
        uint64_t n0 = (mul_mod(b0, b0, p) + mul_mod(mul_mod(b1, b1, p), w2, p)) % p;
        uint64_t n1 = mul_mod(2 % p, mul_mod(b0, b1, p), p);
        b0 = n0; b1 = n1;
    }
    uint64_t r = r0;
    return r < p - r ? r : p - r;
}

void sum_of_squares(uint64_t p, uint64_t k, uint64_t* a, uint64_t* b)
{
    k %= p;
    if (k == 0 || legendre(k, p) == 1) {   // k is a square: (sqrt(k), 0)
        *a = sqrt_mod(k, p);
        *b = 0;
        return;
    }
    uint64_t s = 2;                        // smallest quadratic non-residue
    while (legendre(s, p) == 1) ++s;
    uint64_t c = sqrt_mod(s - 1, p);       // s - 1 is a square
    uint64_t r = mul_mod(k, inv_mod(s, p), p);
    uint64_t x = sqrt_mod(r, p);           // k = x^2 s = x^2 (1 + c^2)
    *a = x;
    *b = mul_mod(x, c, p);
}

bool nrsyf(uint64_t p, uint64_t alpha, uint64_t beta, uint64_t Y[4])
{
    alpha %= p; beta %= p;
    if (legendre(alpha, p) != -1 || legendre(beta, p) != -1) return false;
    uint64_t a, b;
    sum_of_squares(p, alpha, &a, &b);                 // alpha = a^2 + b^2, a != 0
    uint64_t d = mul_mod(a, sqrt_mod(mul_mod(beta, inv_mod(alpha, p), p), p), p);
    uint64_t c = (p - mul_mod(mul_mod(b, d, p), inv_mod(a, p), p)) % p;   // a c + b d = 0
    Y[0] = a; Y[1] = b; Y[2] = c; Y[3] = d;
    return true;
}

bool supported_prime(uint64_t p) { return p >= 2 && p <= kMaxPrime && is_prime_u32(p); }

bool make_field_plan(uint32_t p, FieldPlan* out)
{
    if (p < 2 || !is_prime_u32(p)) return false;
    FieldPlan f;
    f.p = p;
    f.pinv = 1.0 / (double)p;
    if (p == 2) {              // 1^2 + 0^2 = 1 = -1: Y = I
        f.ya = 1;
        f.yb = 0;
        f.ycost = 1;
    } else if (p % 4 == 1) {
        f.ya = (uint32_t)sqrt_mod(p - 1, p);
        f.yb = 0;
        f.ycost = 1;
    } else if (p % 8 == 3) {
        f.ya = 1;
        f.yb = (uint32_t)sqrt_mod(p - 2, p);
        f.ycost = 2;
    } else {
        uint64_t a, b;
        sum_of_squares(p, p - 1, &a, &b);
        f.ya = (uint32_t)a;
        f.yb = (uint32_t)b;
        f.ycost = 3;
    }
    *out = f;
    return true;
}

}  // namespace ffp
