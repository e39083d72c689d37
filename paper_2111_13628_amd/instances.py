"""Seeded synthetic inputs: random k-SAT formulas, random symmetric QAP matrices,
annealing schedules and request mixes.

This module holds no arithmetic of the Monte Carlo method itself.  It only
produces the inputs that both the GPU library and the CPU oracle consume, so
that the two sides see bit-identical problems.

Workload shapes follow the paper's numerics (section "Numerical simulations"):
random 4-SAT near the satisfiability threshold (subsection "4-SAT Problems Near
Computational Phase Transitions", where M = round(alpha * N), e.g. 9.884 * 5000
= 49,420 clauses) and QAP with integer flow/distance matrices (subsection
"Quadratic Assignment Problems").  The paper's own instance sets are not
available; these generators stand in for them.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

DEFAULT_SEED = 20211126


def _frac(alpha) -> Fraction:
    if isinstance(alpha, Fraction):
        return alpha
    if isinstance(alpha, int):
        return Fraction(alpha)
    # decimal string or float literal -> exact decimal fraction
    return Fraction(str(alpha))


def ksat_clause_count(n_vars: int, alpha) -> int:
    """M = round(alpha * N), half-up, computed on the exact decimal value of alpha."""
    a = _frac(alpha)
    return int((a.numerator * n_vars + a.denominator // 2) // a.denominator)


def gen_ksat(n_vars: int, alpha, k: int, seed: int):
    """Random k-SAT formula: M = round(alpha*N) clauses, each with k distinct
    variables drawn uniformly and an independent fair-coin sign per literal.

    Returns (clause_ptr int32[M+1], lits int32[M*k]) in the DIMACS sign
    convention: literal +(v+1) is x_v, -(v+1) is NOT x_v.
    """
    if k > n_vars:
        raise ValueError("k must not exceed the number of variables")
    m = ksat_clause_count(n_vars, alpha)
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.integers(0, n_vars, size=(m, k), dtype=np.int64)
    # redraw rows that repeat a variable until every clause has k distinct ones
    while True:
        s = np.sort(v, axis=1)
        bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
        if bad.size == 0:
            break
        v[bad] = rng.integers(0, n_vars, size=(bad.size, k), dtype=np.int64)
    neg = rng.integers(0, 2, size=(m, k), dtype=np.int64)
    lits = ((v + 1) * (1 - 2 * neg)).astype(np.int32).reshape(-1)
    clause_ptr = (np.arange(m + 1, dtype=np.int64) * k).astype(np.int32)
    return clause_ptr, lits


def gen_ksat_disjoint(n_clauses: int, k: int, seed: int):
    """k-SAT formula whose clauses share no variable: clause a holds variables
    k*a .. k*a+k-1 with fair-coin signs (N = k * n_clauses).  Its energy at
    inverse temperature beta is a sum of independent clause indicators, so its
    equilibrium statistics have closed forms.  Same return convention as
    gen_ksat."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = np.arange(n_clauses * k, dtype=np.int64).reshape(n_clauses, k)
    neg = rng.integers(0, 2, size=(n_clauses, k), dtype=np.int64)
    lits = ((v + 1) * (1 - 2 * neg)).astype(np.int32).reshape(-1)
    clause_ptr = (np.arange(n_clauses + 1, dtype=np.int64) * k).astype(np.int32)
    return clause_ptr, lits


def gen_qap(n: int, seed: int, lo: int = 0, hi: int = 99):
    """Symmetric flow and distance matrices with zero diagonal and integer
    entries uniform in [lo, hi].  Returns (F, D) as int32[n, n]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(2):
        a = rng.integers(lo, hi + 1, size=(n, n), dtype=np.int64)
        a = np.triu(a, 1)
        a = a + a.T
        out.append(a.astype(np.int32))
    return out[0], out[1]


def linear_schedule(beta0: float, beta1: float, n_sweeps: int) -> np.ndarray:
    """beta_t = beta0 + (beta1 - beta0) * t / (S - 1), t = 0..S-1, both ends included."""
    if n_sweeps <= 0:
        return np.zeros(0, dtype=np.float64)
    if n_sweeps == 1:
        return np.array([beta0], dtype=np.float64)
    t = np.arange(n_sweeps, dtype=np.float64)
    return beta0 + (beta1 - beta0) * t / float(n_sweeps - 1)


def profile_schedule(cold: np.ndarray, hot: np.ndarray) -> np.ndarray:
    """Stack per-class schedules into the [class][sweep] layout both sides take
    (class 0 = COLD, class 1 = HOT)."""
    return np.ascontiguousarray(np.stack([cold, hot]).astype(np.float64))


def batch_mix(n_instances: int, seed: int):
    """Mixed k-SAT batch: k in {3,4} by fair coin, N log-uniform in [1000, 20000],
    alpha = 4.15 (k=3) or 9.8 (k=4), replicas 64..512 scaled with N."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_instances):
        k = 3 if rng.integers(0, 2) == 0 else 4
        n = int(round(float(np.exp(rng.uniform(np.log(1000.0), np.log(20000.0))))))
        alpha = "4.15" if k == 3 else "9.8"
        step = min(3, int(np.floor(4.0 * np.log(n / 1000.0) / np.log(20.0))))
        reps = 64 * (2 ** max(0, step))
        out.append(dict(k=k, n=n, alpha=alpha, replicas=reps, seed=seed + 1 + i))
    return out


def serve_ksat_replicas(n: int) -> int:
    """Replicas of a served 4-SAT request: 64, 128 or 256 as N grows over
    [2000, 50000] in thirds of its log range."""
    step = min(2, int(np.floor(3.0 * np.log(n / 2000.0) / np.log(25.0))))
    return 64 * (2 ** max(0, step))


def serve_mix(rate_per_s: float, duration_s: float, seed: int):
    """Poisson request stream: 70 % random 4-SAT (N log-uniform in [2000, 50000],
    alpha 9.7), 30 % QAP (n uniform in [30, 150], entries in [0, 99])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate_per_s))
        if t >= duration_s:
            break
        if rng.uniform() < 0.7:
            n = int(round(float(np.exp(rng.uniform(np.log(2000.0), np.log(50000.0))))))
            reqs.append(dict(kind="ksat", arrival=t, n=n, k=4, alpha="9.7",
                             replicas=serve_ksat_replicas(n), seed=seed + 1 + i))
        else:
            n = int(rng.integers(30, 151))
            reqs.append(dict(kind="qap", arrival=t, n=n, replicas=256, seed=seed + 1 + i))
        i += 1
    return reqs
