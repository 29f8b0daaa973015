// Device arithmetic on residues in [0,p) for primes p with p^2 < 2^53
// (p <= 94906249): a product of two residues is exact in a double.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ffp {

__device__ inline uint32_t add_m(uint32_t a, uint32_t b, uint32_t p)
{
    uint32_t s = a + b;
    return s >= p ? s - p : s;
}

__device__ inline uint32_t sub_m(uint32_t a, uint32_t b, uint32_t p)
{
    return a >= b ? a - b : a + p - b;
}

// Reduction of a non-negative integer x < 2^53 held in a double: the
// quotient estimate from 1/p is off by at most one, the remainder is exact.
__device__ inline uint32_t mod53(double x, uint32_t p, double pinv)
{
    const double q = floor(x * pinv);
    double r = fma(-q, (double)p, x);
    if (r < 0.0) r += (double)p;
    if (r >= (double)p) r -= (double)p;
    return (uint32_t)r;
}

// a*b mod p: the product of two residues is below p^2 < 2^53, exact in a double.
__device__ inline uint32_t mul_m(uint32_t a, uint32_t b, uint32_t p, double pinv)
{
    return mod53((double)a * (double)b, p, pinv);
}

__device__ inline uint32_t pow_m(uint32_t a, uint32_t e, uint32_t p, double pinv)
{
    uint32_t r = 1, b = a;
    while (e) {
        if (e & 1u) r = mul_m(r, b, p, pinv);
        b = mul_m(b, b, p, pinv);
        e >>= 1;
    }
    return r;
}

// Inverse of a in [1, p) for an odd prime p by the binary extended Euclidean
// algorithm (invariants x1 a = u and x2 a = v mod p); 0 maps to 0.
__device__ inline uint32_t inv_binary(uint32_t a, uint32_t p)
{
    if (a == 0u) return 0u;
    uint32_t u = a, v = p, x1 = 1u, x2 = 0u;
    while (u != 1u && v != 1u) {
        while ((u & 1u) == 0u) {
            u >>= 1;
            x1 = (x1 & 1u) ? (uint32_t)(((uint64_t)x1 + p) >> 1) : x1 >> 1;
        }
        while ((v & 1u) == 0u) {
            v >>= 1;
            x2 = (x2 & 1u) ? (uint32_t)(((uint64_t)x2 + p) >> 1) : x2 >> 1;
        }
        if (u >= v) {
            u -= v;
            x1 = x1 >= x2 ? x1 - x2 : x1 + (p - x2);
        } else {
            v -= u;
            x2 = x2 >= x1 ? x2 - x1 : x2 + (p - x1);
        }
    }
    return u == 1u ? x1 : x2;
}

// Inverse by Fermat's little theorem (0 maps to 0).
__device__ inline uint32_t inv_m(uint32_t a, uint32_t p, double pinv)
{
    return pow_m(a, p - 2, p, pinv);
}

// Euler's criterion: true if a is a non-zero quadratic non-residue.
__device__ inline bool is_nonresidue(uint32_t a, uint32_t p, double pinv)
{
    return a != 0 && pow_m(a, (p - 1) / 2, p, pinv) == p - 1;
}

// Square root of a quadratic residue a (Tonelli-Shanks); z is any
// quadratic non-residue mod p.  Returns the root r with r <= p - r.
__device__ inline uint32_t sqrt_m(uint32_t a, uint32_t z, uint32_t p, double pinv)
{
    if (a == 0) return 0;
    uint32_t q = p - 1, s = 0;
    while ((q & 1u) == 0) { q >>= 1; ++s; }
    uint32_t c = pow_m(z, q, p, pinv);
    uint32_t x = pow_m(a, (q + 1) / 2, p, pinv);
    uint32_t t = pow_m(a, q, p, pinv);
    uint32_t m = s;
    while (t != 1) {
        uint32_t i = 0, u = t;
        while (u != 1 && i < m) { u = mul_m(u, u, p, pinv); ++i; }
        if (i >= m) break;   // not a square: never reached for residues
        uint32_t b = c;
        for (uint32_t j = 0; j + i + 1 < m; ++j) b = mul_m(b, b, p, pinv);
        m = i;
        c = mul_m(b, b, p, pinv);
        t = mul_m(t, c, p, pinv);
        x = mul_m(x, b, p, pinv);
    }
    return x <= p - x ? x : p - x;
}

}  // namespace ffp
