"""CPU oracle for exact A*A^T mod p and the LDL^T factorisation.

TEST INFRASTRUCTURE ONLY: the product package never imports this package.
Only tests, the smoke check and the CPU-baseline leg of the benchmark use it.
"""
from .oracle import (  # noqa: F401
    build, load, is_prime, legendre, sqrt_mod, inv_mod, sos, nrsyf,
    syrk, syrk_rows, syrk_entries, gemm, syrk_ab, syrkd, ldlt, ldlt_packed,
    syrkbd, herk, zsyrk,
    num_threads, set_num_threads,
)
from . import costmodel  # noqa: F401
