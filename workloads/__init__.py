"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws matrices; it computes no permanent and holds none of
the method's arithmetic.  Every generator is a pure function of its seed
(NumPy PCG64 via ``default_rng``).

Distributions follow the paper's benchmark section (Sec. 4): random 0/1
matrices and real matrices with entries uniform in [-1, 1]; complex entries
are standard complex Gaussian (real and imaginary parts N(0, 1/2), so
E|z|^2 = 1); the batched workload takes square submatrices of one Haar
unitary (boson-sampling style, Sec. 1.3 photonics paragraph).
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np

__all__ = [
    "uniform", "complex_gauss", "bernoulli", "haar_unitary", "cauchy_dyadic",
    "boson_batch", "bernoulli_batch", "selector_cases", "BatchSpec", "CONFIGS", "config_matrix",
]


def uniform(m: int, n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """m x n float64, i.i.d. uniform on [lo, hi)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=(m, n))


def complex_gauss(m: int, n: int, seed: int) -> np.ndarray:
    """m x n complex128, real and imaginary parts i.i.d. N(0, 1/2)."""
    rng = np.random.default_rng(seed)
    s = np.sqrt(0.5)
    return rng.normal(0.0, s, size=(m, n)) + 1j * rng.normal(0.0, s, size=(m, n))


def bernoulli(m: int, n: int, p: float, seed: int) -> np.ndarray:
    """m x n uint8 0/1 matrix, each entry 1 with probability p."""
    rng = np.random.default_rng(seed)
    return (rng.random(size=(m, n)) < p).astype(np.uint8)


def haar_unitary(N: int, seed: int) -> np.ndarray:
    """N x N Haar-random unitary: QR of a complex Gaussian matrix with the
    phases of R's diagonal moved into Q (Mezzadri's recipe)."""
    z = complex_gauss(N, N, seed)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def cauchy_dyadic(m: int, n: int, seed: int, bits: int = 20):
    """Cauchy matrix c_ij = 1 / (x_i - y_j) with x in [1/4, 3/4] and
    y in [-3/4, -1/4], so every denominator lies in [1/2, 3/2].

    x and y are dyadic rationals k / 2^bits, returned exactly as Fractions
    together with the float64 matrix (each entry rounded once)."""
    rng = np.random.default_rng(seed)
    scale = 1 << bits
    xk = rng.integers(scale // 4, 3 * scale // 4 + 1, size=m)
    yk = rng.integers(-(3 * scale // 4), -(scale // 4) + 1, size=n)
    x = [Fraction(int(k), scale) for k in xk]
    y = [Fraction(int(k), scale) for k in yk]
    c = np.array([[float(1 / (xi - yj)) for yj in y] for xi in x], dtype=np.float64)
    return c, x, y


@dataclass
class BatchSpec:
    """A packed batch of square matrices: matrix b occupies
    data[offset[b] : offset[b] + n[b]*ld[b]] (row-major, leading dimension
    ld[b] elements)."""
    data: np.ndarray          # 1-D, dtype of the matrices
    m: np.ndarray             # int32
    n: np.ndarray             # int32
    offset: np.ndarray        # int64, in elements
    ld: np.ndarray            # int64, in elements

    @property
    def count(self) -> int:
        return int(self.n.shape[0])

    def matrix(self, b: int) -> np.ndarray:
        o, m, n, ld = int(self.offset[b]), int(self.m[b]), int(self.n[b]), int(self.ld[b])
        return self.data[o:o + m * ld].reshape(m, ld)[:, :n]


def boson_batch(count: int, nmin: int, nmax: int, N: int = 64, seed_u: int = 6400,
                seed_idx: int = 6401) -> BatchSpec:
    """``count`` square complex128 submatrices of one seeded N x N Haar unitary.
    Matrix b has order n_b ~ U{nmin..nmax}; its rows and its columns are each a
    sorted random n_b-subset of 0..N-1 (a collision-free boson-sampling input
    and output pattern)."""
    U = haar_unitary(N, seed_u)
    rng = np.random.default_rng(seed_idx)
    ns = rng.integers(nmin, nmax + 1, size=count).astype(np.int32)
    offs = np.zeros(count, dtype=np.int64)
    total = 0
    for b in range(count):
        offs[b] = total
        total += int(ns[b]) * int(ns[b])
    data = np.empty(total, dtype=np.complex128)
    for b in range(count):
        k = int(ns[b])
        rows = np.sort(rng.choice(N, size=k, replace=False))
        cols = np.sort(rng.choice(N, size=k, replace=False))
        data[offs[b]:offs[b] + k * k] = U[np.ix_(rows, cols)].reshape(-1)
    return BatchSpec(data=data, m=ns.copy(), n=ns, offset=offs, ld=ns.astype(np.int64))


def bernoulli_batch(count: int, nmin: int, nmax: int, p: float = 0.5,
                    seed: int = 6500) -> BatchSpec:
    """``count`` square 0/1 matrices (uint8) of orders n_b ~ U{nmin..nmax},
    each entry 1 with probability p (bipartite graphs whose perfect matchings
    the permanent counts), packed contiguously with ld = n_b."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count).astype(np.int32)
    offs = np.zeros(count, dtype=np.int64)
    total = 0
    for b in range(count):
        offs[b] = total
        total += int(ns[b]) * int(ns[b])
    data = (rng.random(size=total) < p).astype(np.uint8)
    return BatchSpec(data=data, m=ns.copy(), n=ns, offset=offs, ld=ns.astype(np.int64))


def selector_cases(count: int, seed: int = 5000, mmin: int = 2, mmax: int = 30,
                   nmax: int = 48):
    """Shape/density/dtype draws for algorithm-selection timing:
    m ~ U{mmin..mmax}, n ~ U{m..nmax}, density in {0.1, ..., 1.0},
    dtype in {f64, c128, b8}.  Returns a list of dicts with a per-case seed."""
    rng = np.random.default_rng(seed)
    dts = ("f64", "c128", "b8")
    out = []
    for c in range(count):
        m = int(rng.integers(mmin, mmax + 1))
        n = int(rng.integers(m, nmax + 1))
        dens = float(rng.integers(1, 11)) / 10.0
        out.append({"m": m, "n": n, "density": dens, "dtype": dts[int(rng.integers(0, 3))],
                    "seed": int(rng.integers(0, 2**31 - 1))})
    return out


def case_matrix(case: dict) -> np.ndarray:
    """The matrix for one selector case: entries from the dtype's distribution,
    each kept with probability ``density`` and zeroed otherwise."""
    m, n, seed = case["m"], case["n"], case["seed"]
    rng = np.random.default_rng(seed)
    keep = rng.random(size=(m, n)) < case["density"]
    if case["dtype"] == "f64":
        a = rng.uniform(-1, 1, size=(m, n))
    elif case["dtype"] == "c128":
        s = np.sqrt(0.5)
        a = rng.normal(0, s, size=(m, n)) + 1j * rng.normal(0, s, size=(m, n))
    else:
        return keep.astype(np.uint8)
    return np.where(keep, a, 0).astype(a.dtype)


# Named single-matrix workloads (the recipes the tests and the benchmark use).
CONFIGS = {
    "u12":   dict(kind="uniform", m=12, n=12, seed=1201),
    "u32":   dict(kind="uniform", m=32, n=32, seed=3201),
    "c32":   dict(kind="complex", m=32, n=32, seed=3202),
    "b28":   dict(kind="bernoulli", m=28, n=28, p=0.5, seed=2801),
    "u20x40": dict(kind="uniform", m=20, n=40, seed=2040),
    "b16x48": dict(kind="bernoulli", m=16, n=48, p=0.3, seed=1648),
    # 30 x 30 sparse 0/1: seed 3031 is the first from 3031 with no zero row or
    # column; seed 3030 has an all-zero row, kept as the degenerate case
    "b30":   dict(kind="bernoulli", m=30, n=30, p=0.15, seed=3031),
    "b30z":  dict(kind="bernoulli", m=30, n=30, p=0.15, seed=3030),
    "u36":   dict(kind="uniform", m=36, n=36, seed=3601),
    # compute-bound shapes of the e_m form (2^27 terms)
    "u28x48": dict(kind="uniform", m=28, n=48, seed=2848),
    "c28x48": dict(kind="complex", m=28, n=48, seed=2849),
}


def config_matrix(name: str) -> np.ndarray:
    c = CONFIGS[name]
    if c["kind"] == "uniform":
        return uniform(c["m"], c["n"], c["seed"])
    if c["kind"] == "complex":
        return complex_gauss(c["m"], c["n"], c["seed"])
    if c["kind"] == "bernoulli":
        return bernoulli(c["m"], c["n"], c["p"], c["seed"])
    raise KeyError(name)
