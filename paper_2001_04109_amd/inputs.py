"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws random numbers only; it holds none of the method's
arithmetic.  Every array is drawn on the host with numpy's PCG64
(numpy.random.default_rng) in the documented order, so the GPU path and the
oracle receive the same bytes.

The paper measures on random dense matrices over Z/131071Z; these generators
stand in for them with the shapes and prime fields of the workloads below.
"""
from __future__ import annotations

import numpy as np

BATCH_PRIMES = (251, 65537, 131071)


def uniform(seed, n: int, k: int, p: int) -> np.ndarray:
    """n x k uint32 matrix with entries uniform in [0, p)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, p, size=(n, k), dtype=np.uint32)


def symmetric(seed, n: int, p: int) -> np.ndarray:
    """Symmetric n x n uint32 matrix: upper triangle (with diagonal) uniform in
    [0, p), drawn row-major as one n x n block, then mirrored."""
    rng = np.random.default_rng(seed)
    M = rng.integers(0, p, size=(n, n), dtype=np.uint32)
    U = np.triu(M)
    return U + np.triu(U, 1).T


def batch_jobs(seed: int = 3, njobs: int = 1024, nmin: int = 32, nmax: int = 1024,
               primes=BATCH_PRIMES):
    """Shapes of the batched workload: per job n ~ U[nmin, nmax],
    k ~ U[ceil(n/2), 2n], p ~ U(primes), drawn job by job in that order.
    The matrix of job j is uniform(seed=(seed, j), n, k, p)."""
    rng = np.random.default_rng(seed)
    jobs = []
    for _ in range(njobs):
        n = int(rng.integers(nmin, nmax + 1))
        k = int(rng.integers((n + 1) // 2, 2 * n + 1))
        p = int(primes[int(rng.integers(0, len(primes)))])
        jobs.append((n, k, p))
    return jobs


def batch_matrix(seed: int, j: int, n: int, k: int, p: int) -> np.ndarray:
    return uniform((seed, j), n, k, p)


def request_stream(seed: int = 4, nreq: int = 20000, rate: float = 2000.0,
                   frac_syrk: float = 0.7, nmin: int = 256, nmax: int = 4096,
                   primes=BATCH_PRIMES, ldlt_prime: int = 65537):
    """Poisson request stream of the served workload.

    Draw order per request: exponential inter-arrival gap (mean 1/rate s),
    kind (syrk with probability frac_syrk, else ldlt), n ~ U[nmin, nmax],
    then for syrk k ~ U[ceil(n/2), 2n] and p ~ U(primes); ldlt uses
    ldlt_prime and k = n.  Operands are drawn later from sub-seed (seed, r).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for r in range(nreq):
        t += float(rng.exponential(1.0 / rate))
        is_syrk = bool(rng.random() < frac_syrk)
        n = int(rng.integers(nmin, nmax + 1))
        if is_syrk:
            k = int(rng.integers((n + 1) // 2, 2 * n + 1))
            p = int(primes[int(rng.integers(0, len(primes)))])
        else:
            k = n
            p = ldlt_prime
        reqs.append({"id": r, "t": t, "kind": "syrk" if is_syrk else "ldlt",
                     "n": n, "k": k, "p": p})
    return reqs


def request_operand(seed: int, req: dict) -> np.ndarray:
    if req["kind"] == "syrk":
        return uniform((seed, req["id"]), req["n"], req["k"], req["p"])
    return symmetric((seed, req["id"]), req["n"], req["p"])
