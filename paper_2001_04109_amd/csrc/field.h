// Host-side prime-field routines of the product library: primality, Legendre
// symbols, square roots, Algorithm 3 (SoS), Algorithm 4 (nrsyf) and the
// choice of the skew-orthogonal Y of Section 3.1.
#pragma once
#include <cstdint>

namespace ffp {

bool is_prime_u32(uint64_t p);
uint64_t pow_mod(uint64_t a, uint64_t e, uint64_t p);
uint64_t inv_mod(uint64_t a, uint64_t p);
// Legendre symbol (a/p) for an odd prime p, computed as a Jacobi symbol by
// quadratic reciprocity: 0, 1 or -1.
int legendre(uint64_t a, uint64_t p);
// Canonical square root min(r, p-r) of a square a modulo an odd prime p
// (Cipolla's method); returns UINT64_MAX when a is not a square.
uint64_t sqrt_mod(uint64_t a, uint64_t p);
// Algorithm 3: (a, b) with a^2 + b^2 = k mod p (odd prime p).
void sum_of_squares(uint64_t p, uint64_t k, uint64_t* a, uint64_t* b);
// Algorithm 4: Y = [[y0,y1],[y2,y3]] with Y Y^T = diag(alpha, beta) for two
// quadratic non-residues; returns false if either is a residue.
bool nrsyf(uint64_t p, uint64_t alpha, uint64_t beta, uint64_t Y[4]);

// The skew-orthogonal Y = [[a I, b I], [-b I, a I]] used by Algorithm 2
// (Propositions 3.3 and 3.4, proof of Theorem 4.1):
//   p = 1 mod 4: a = sqrt(-1), b = 0 (Y = i I, cost y = 1);
//   p = 3 mod 8: a = 1, b = sqrt(-2) (y = 2);
//   otherwise    (a, b) = SoS(p, -1) by Algorithm 3 (y = 3).
struct FieldPlan {
    uint32_t p = 0;
    uint32_t ya = 0, yb = 0;  // entries of Y, residues
    int ycost = 0;            // y of Theorem 4.1
    double pinv = 0.0;        // 1/p rounded to nearest
};
// p = 2: a = 1, b = 0 (1 = -1 in characteristic 2, Proposition 3.3).
bool make_field_plan(uint32_t p, FieldPlan* out);

// Largest prime p with p (p - 1) < 2^53: the FP64 base products stay exact
// with a reduction after every 4-column matrix-core step (a reduced
// accumulator, below p, plus four products of centred residues, each at
// most ((p-1)/2)^2), and every product of two residues is exact in a double.
constexpr uint32_t kMaxPrime = 94906249u;
// Moduli the product paths accept: primes 2 <= p <= kMaxPrime.
bool supported_prime(uint64_t p);

}  // namespace ffp
