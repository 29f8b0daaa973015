"""Operation-count model of Algorithm 2 (TEST INFRASTRUCTURE ONLY).

Restates the counts of Section 4.1 and of the appendix threshold study of
Dumas, Pernet and Sedoglavic (arXiv:2001.04109):

* classical products: syrk(n) = n(n+1)(2n-1)/2 field operations for the
  lower triangle of an n x n times n x n product, gemm(n) = n^2 (2n-1);
* Strassen-Winograd (Algorithm 1) with j recursive levels:
  W_j(n) = 7 W_{j-1}(n/2) + 15 (n/2)^2, W_0 = gemm;
* the classical 2x2-block divide and conquer SYRK with four recursive
  calls and two general products (the "Syrk-i" rows of Table 5);
* Algorithm 2 with y-cost Y multiplications (the "Gy-i" rows of Table 5):
  Gy_i(n) = 3 Gy_{i-1}(n/2) + 2 W_{i-1}(n/2) + (7.5 + 2y)(n/2)^2,
  Gy_0 = syrk, which is recurrence (complexity) of Theorem 4.1 with
  2 C_omega (n/2)^omega replaced by two Strassen-Winograd products;
* the fraction of classical multiply-adds left after d levels when the
  base products are classical: t_d = 3/8 t_{d-1} + 1/2, t_0 = 1, whose
  limit 0.8 is the 0.8 n^3 entry of Table 1;
* scalar additions of one level on m x m blocks (Remark 4.2):
  6 m^2 + 3/2 m (m + 1).
"""
from fractions import Fraction


def syrk(n: int) -> int:
    return n * (n + 1) * (2 * n - 1) // 2


def gemm(n: int) -> int:
    return n * n * (2 * n - 1)


def winograd(j: int, n: int) -> int:
    """Field operations of Algorithm 1 applied recursively j times."""
    if j == 0:
        return gemm(n)
    h = n // 2
    return 7 * winograd(j - 1, h) + 15 * h * h


def syrk_dc(i: int, n: int) -> int:
    """Classical 2x2-block divide and conquer SYRK ("Syrk-i" of Table 5).

    Syrk-1 is the classical product; each further level makes four
    recursive calls, two general products by Strassen-Winograd with i-2
    recursive levels... as printed, the general products of Syrk-i use
    W_{i-1}, and the additions are two half additions and one full one.
    """
    if i == 1:
        return syrk(n)
    h = n // 2
    return 4 * syrk_dc(i - 1, h) + 2 * winograd(i - 1, h) + h * (h + 1) + h * h


def alg2(y: float, i: int, n: int):
    """Algorithm 2 with i recursive levels ("Gy-i" of Table 5)."""
    if i == 0:
        return syrk(n)
    h = n // 2
    v = 3 * alg2(y, i - 1, h) + 2 * winograd(i - 1, h) + (Fraction(15, 2) + 2 * Fraction(y)) * h * h
    return v


def mac_fraction(d: int) -> Fraction:
    """Multiply-adds of d levels of Algorithm 2 over classical base products,
    relative to the classical lower-triangle product."""
    t = Fraction(1)
    for _ in range(d):
        t = Fraction(3, 8) * t + Fraction(1, 2)
    return t


def additions_per_level(m: int) -> Fraction:
    """Scalar additions of the 9 block additions of one level, m x m blocks."""
    return 6 * m * m + Fraction(3, 2) * m * (m + 1)


def y_cost(p: int) -> int:
    """Cost constant y of one multiplication by Y (proof of Theorem 4.1)."""
    if p == 2 or p % 4 == 1:
        return 1
    if p % 8 == 3:
        return 2
    return 3
