"""Closed-form permanents and matrix families used as pins.

Each function states a value fixed by mathematics, independent of any
permanent evaluator.  Citations refer to the paper (Masschelein, Richer &
Ayers) where it names the family.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np


def ones_value(m: int, n: int) -> int:
    """per(J_{m x n}) = n!/(n-m)! for m <= n (Sec. 4, accuracy matrices)."""
    if m > n:
        m, n = n, m
    return math.factorial(n) // math.factorial(n - m)


def ones(m: int, n: int) -> np.ndarray:
    return np.ones((m, n), dtype=np.int64)


def identity_rect(m: int, n: int) -> np.ndarray:
    """Identity with the extra columns filled with zeros (Sec. 4); per = 1."""
    a = np.zeros((m, n), dtype=np.int64)
    for i in range(min(m, n)):
        a[i, i] = 1
    return a


def derangements(n: int) -> int:
    """D_n, the number of permutations without fixed points = per(J - I)
    (perfect matchings of the complete bipartite graph minus a matching,
    Sec. 1.3 graph theory).  D_n = (n-1)(D_{n-1} + D_{n-2})."""
    d = [1, 0]
    for k in range(2, n + 1):
        d.append((k - 1) * (d[-1] + d[-2]))
    return d[n]


def derangement_matrix(n: int) -> np.ndarray:
    return np.ones((n, n), dtype=np.int64) - np.eye(n, dtype=np.int64)


def rect_derangements(m: int, n: int) -> int:
    """Injective maps s:[m]->[n] with s(i) != i for every i (m <= n):
    sum_k (-1)^k C(m, k) (n-k)!/(n-m)!  (inclusion-exclusion over fixed points)."""
    return sum((-1) ** k * math.comb(m, k) * math.factorial(n - k) // math.factorial(n - m)
               for k in range(m + 1))


def rect_derangement_matrix(m: int, n: int) -> np.ndarray:
    return np.ones((m, n), dtype=np.int64) - identity_rect(m, n)


def fibonacci(k: int) -> int:
    a, b = 0, 1
    for _ in range(k):
        a, b = b, a + b
    return a


def tridiagonal_ones(n: int) -> np.ndarray:
    """a_ij = 1 iff |i - j| <= 1; per = F_{n+1} (matchings of a ladder path)."""
    i = np.arange(n)
    return (np.abs(i[:, None] - i[None, :]) <= 1).astype(np.int64)


def hessenberg_ones(n: int) -> np.ndarray:
    """a_ij = 1 iff j <= i + 1; per = 2^(n-1)."""
    i = np.arange(n)
    return (i[None, :] <= i[:, None] + 1).astype(np.int64)


def cycle_plus_identity(n: int) -> np.ndarray:
    """I + P (P the cyclic shift); per = 2 for n >= 3 (the two perfect
    matchings of an even cycle)."""
    a = np.eye(n, dtype=np.int64)
    for i in range(n):
        a[i, (i + 1) % n] += 1
    return a


def elementary_symmetric(v, k: int):
    """e_k(v) by the product-expansion recurrence, exact for ints/Fractions."""
    e = [1] + [0] * k
    for x in v:
        for j in range(k, 0, -1):
            e[j] = e[j] + e[j - 1] * x
    return e[k]


def rank_one_value(u, v) -> int:
    """per(u v^T) for len(u) = m <= len(v) = n: (prod u) * m! * e_m(v)."""
    m = len(u)
    return math.prod(u) * math.factorial(m) * elementary_symmetric(list(v), m)


def det_fraction(rows) -> Fraction:
    """Exact determinant by Gaussian elimination over Fractions."""
    a = [[Fraction(x) for x in r] for r in rows]
    n = len(a)
    det = Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if a[r][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            a[c], a[p] = a[p], a[c]
            det = -det
        det *= a[c][c]
        for r in range(c + 1, n):
            f = a[r][c] / a[c][c]
            if f:
                for k in range(c, n):
                    a[r][k] -= f * a[c][k]
    return det


def cauchy_borchardt(x, y) -> Fraction:
    """Borchardt: per(C) = det(C o C) / det(C) for c_ij = 1/(x_i - y_j),
    square (Sec. 1.4, Eq. caucy_permanent)."""
    c = [[1 / (xi - yj) for yj in y] for xi in x]
    c2 = [[e * e for e in r] for r in c]
    return det_fraction(c2) / det_fraction(c)


def digits_lost(evaluated: float, true: float, macheps: float = 2.0 ** -52) -> float:
    """Sec. 4 Eq. digits_lost: log10(|eval - true|/|true|) - log10(macheps),
    clamped at 0 when the evaluation is exact."""
    if evaluated == true:
        return 0.0
    if true == 0:
        return math.inf
    return max(0.0, math.log10(abs(evaluated - true) / abs(true)) - math.log10(macheps))


def read_worked_example():
    """The worked example file under tests/golden/."""
    path = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")
    lines = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    m, n = int(lines[0][0]), int(lines[0][1])
    a = np.array([[int(x) for x in lines[1 + i]] for i in range(m)], dtype=np.int64)
    return a, int(lines[1 + m][0])
