"""Pins for the CPU oracle: values fixed by the paper or by mathematics.

Every evaluator in ``oracle`` (brute force = the definition, memoised Laplace
expansion, Glynn and Ryser in double-double) is checked against closed forms,
invariants and special cases, and the faster evaluators against the
definition on every small shape.  A dropped term, a wrong sign, a wrong index
or a transposed operand in any of them fails at least one test here.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import closed_forms as cf
import workloads

U = 2.0 ** -53
INT_EVALUATORS = [oracle.per_brute, oracle.per_laplace,
                  lambda a: oracle.per_laplace(a, form=1),
                  lambda a: oracle.per_laplace(a, form=2)]
FP_EVALUATORS = [oracle.per_brute, oracle.per_laplace, oracle.per_glynn, oracle.per_ryser]


def fp_value(v):
    return float(v) if isinstance(v, oracle.DD) else complex(v)


# ---- the paper's worked example (Sec. 3.3) --------------------------------
def test_worked_example_integer():
    a, want = cf.read_worked_example()
    for ev in INT_EVALUATORS:
        assert ev(a) == want
    assert want == 450


def test_worked_example_float():
    a, want = cf.read_worked_example()
    for ev in FP_EVALUATORS:
        v = ev(a.astype(np.float64))
        assert v.frac() == want


# ---- closed forms ----------------------------------------------------------
@pytest.mark.parametrize("m,n", [(m, n) for n in range(1, 10) for m in range(1, n + 1)])
def test_all_ones(m, n):
    want = cf.ones_value(m, n)
    for ev in INT_EVALUATORS:
        assert ev(cf.ones(m, n)) == want
        assert ev(cf.ones(n, m)) == want          # m > n: per(A^T)
    for ev in FP_EVALUATORS:
        assert ev(cf.ones(m, n).astype(np.float64)).frac() == want


@pytest.mark.parametrize("m,n", [(1, 1), (3, 3), (4, 7), (6, 6), (5, 9), (8, 8)])
def test_identity(m, n):
    for ev in INT_EVALUATORS:
        assert ev(cf.identity_rect(m, n)) == 1
    for ev in FP_EVALUATORS:
        assert ev(cf.identity_rect(m, n).astype(np.float64)).frac() == 1


@pytest.mark.parametrize("n", range(1, 11))
def test_derangements(n):
    want = cf.derangements(n)
    a = cf.derangement_matrix(n)
    assert oracle.per_brute(a) == want
    assert oracle.per_laplace(a) == want
    if n <= 9:
        assert oracle.per_glynn(a).frac() == want
        assert oracle.per_ryser(a).frac() == want


@pytest.mark.parametrize("m,n", [(2, 5), (3, 7), (4, 6), (5, 9), (6, 8), (7, 10)])
def test_rect_derangements(m, n):
    want = cf.rect_derangements(m, n)
    a = cf.rect_derangement_matrix(m, n)
    for ev in INT_EVALUATORS:
        assert ev(a) == want
    for ev in FP_EVALUATORS[2:]:
        assert ev(a).frac() == want


@pytest.mark.parametrize("n", range(1, 12))
def test_structured_graphs(n):
    assert oracle.per_laplace(cf.tridiagonal_ones(n)) == cf.fibonacci(n + 1)
    assert oracle.per_laplace(cf.hessenberg_ones(n)) == 2 ** (n - 1)
    if n >= 3:
        assert oracle.per_laplace(cf.cycle_plus_identity(n)) == 2
    if n <= 9:
        assert oracle.per_brute(cf.tridiagonal_ones(n)) == cf.fibonacci(n + 1)
        assert oracle.per_brute(cf.hessenberg_ones(n)) == 2 ** (n - 1)
        assert oracle.per_glynn(cf.hessenberg_ones(n)).frac() == 2 ** (n - 1)
        assert oracle.per_ryser(cf.tridiagonal_ones(n)).frac() == cf.fibonacci(n + 1)


def test_triangular_and_block():
    rng = np.random.default_rng(7)
    t = np.triu(rng.integers(-5, 6, size=(8, 8)))
    for ev in INT_EVALUATORS:
        assert ev(t) == int(np.prod(np.diag(t)))
    b1 = rng.integers(-3, 4, size=(3, 3))
    b2 = rng.integers(-3, 4, size=(4, 4))
    blk = np.zeros((7, 7), dtype=np.int64)
    blk[:3, :3] = b1
    blk[3:, 3:] = b2
    p1, p2 = oracle.per_brute(b1), oracle.per_brute(b2)
    assert oracle.per_brute(b1) == (b1[0, 0] * (b1[1, 1] * b1[2, 2] + b1[1, 2] * b1[2, 1])
                                    + b1[0, 1] * (b1[1, 0] * b1[2, 2] + b1[1, 2] * b1[2, 0])
                                    + b1[0, 2] * (b1[1, 0] * b1[2, 1] + b1[1, 1] * b1[2, 0]))
    for ev in INT_EVALUATORS:
        assert ev(blk) == p1 * p2


@pytest.mark.parametrize("m,n", [(1, 1), (1, 6), (2, 2), (3, 3), (3, 8), (5, 7), (6, 6)])
def test_rank_one(m, n):
    rng = np.random.default_rng(100 + 10 * m + n)
    u = [int(x) for x in rng.integers(-4, 5, size=m)]
    v = [int(x) for x in rng.integers(-4, 5, size=n)]
    a = np.outer(u, v).astype(np.int64)
    want = cf.rank_one_value(u, v)
    if m == n:
        assert want == math.factorial(n) * math.prod(u) * math.prod(v)
    for ev in INT_EVALUATORS:
        assert ev(a) == want


def test_small_cases():
    rng = np.random.default_rng(3)
    for n in range(1, 9):
        r = rng.integers(-9, 10, size=(1, n))
        for ev in INT_EVALUATORS:
            assert ev(r) == int(r.sum())
    a = np.array([[2, -3], [5, 7]])
    for ev in INT_EVALUATORS:
        assert ev(a) == 2 * 7 + (-3) * 5
    z = np.zeros((0, 4))
    assert oracle.per_brute(z.astype(np.int64)) == 1      # empty product
    assert oracle.per_laplace(z.astype(np.int64)) == 1


@pytest.mark.parametrize("seed", range(4))
def test_cauchy_borchardt(seed):
    n = 6 + seed
    c, x, y = workloads.cauchy_dyadic(n, n, seed=900 + seed)
    exact = cf.cauchy_borchardt(x, y)
    # c is the exactly-defined matrix rounded entrywise (relative error <= u);
    # all entries are positive, so the permanent moves by at most ~n u per(C).
    tol = (n + 2) * U * float(exact) + 1e-300
    for ev in FP_EVALUATORS:
        v = ev(c)
        assert abs(v.frac() - exact) <= Fraction(tol), ev


# ---- invariants --------------------------------------------------------------
def rand_int(m, n, seed, lo=-6, hi=7):
    return np.random.default_rng(seed).integers(lo, hi, size=(m, n)).astype(np.int64)


@pytest.mark.parametrize("m,n,seed", [(4, 4, 1), (5, 7, 2), (6, 6, 3), (3, 8, 4), (7, 8, 5)])
def test_permutation_invariance(m, n, seed):
    a = rand_int(m, n, seed)
    rng = np.random.default_rng(seed + 50)
    b = a[rng.permutation(m)][:, rng.permutation(n)]
    for ev in INT_EVALUATORS:
        assert ev(a) == ev(b)


@pytest.mark.parametrize("n,seed", [(3, 1), (5, 2), (7, 3)])
def test_transpose(n, seed):
    a = rand_int(n, n, seed)
    for ev in INT_EVALUATORS:
        assert ev(a) == ev(np.ascontiguousarray(a.T))


@pytest.mark.parametrize("m,n,seed", [(4, 4, 11), (5, 8, 12), (6, 6, 13)])
def test_row_multilinearity(m, n, seed):
    a = rand_int(m, n, seed)
    rng = np.random.default_rng(seed)
    i = int(rng.integers(0, m))
    x, y = rand_int(1, n, seed + 1)[0], rand_int(1, n, seed + 2)[0]
    alpha, beta = 3, -5
    ax, ay, az = a.copy(), a.copy(), a.copy()
    ax[i], ay[i] = x, y
    az[i] = alpha * x + beta * y
    d = np.array(rng.integers(-4, 5, size=m), dtype=np.int64)
    for ev in INT_EVALUATORS:
        assert ev(az) == alpha * ev(ax) + beta * ev(ay)
        assert ev(d[:, None] * a) == int(np.prod(d)) * ev(a)


@pytest.mark.parametrize("m,n,seed", [(4, 4, 21), (5, 7, 22), (6, 6, 23)])
def test_laplace_row_expansion(m, n, seed):
    a = rand_int(m, n, seed)
    total = sum(int(a[0, j]) * oracle.per_brute(np.delete(a[1:], j, axis=1)) for j in range(n))
    assert oracle.per_brute(a) == total
    assert oracle.per_laplace(a) == total


@pytest.mark.parametrize("m,n,seed", [(4, 4, 31), (3, 6, 32), (5, 5, 33)])
def test_complex_symmetries(m, n, seed):
    a = workloads.complex_gauss(m, n, seed)
    for ev in FP_EVALUATORS:
        p = complex(ev(a))
        tol = 1e-13 * (1 + abs(p))
        assert abs(complex(ev(np.conj(a))) - np.conj(p)) <= tol
        assert abs(complex(ev(1j * a)) - (1j ** m) * p) <= tol
        assert abs(complex(ev(-a)) - (-1) ** m * p) <= tol
    # real part embedding: a real matrix as complex has a real permanent
    r = workloads.uniform(m, n, seed)
    v = complex(oracle.per_brute(r.astype(np.complex128)))
    assert v.imag == 0.0 and abs(v.real - float(oracle.per_brute(r))) <= 1e-14 * (1 + abs(v))


def test_unitary_submatrix_bound():
    u = workloads.haar_unitary(16, 77)
    rng = np.random.default_rng(5)
    for k in range(2, 8):
        r = np.sort(rng.choice(16, k, replace=False))
        c = np.sort(rng.choice(16, k, replace=False))
        assert abs(complex(oracle.per_brute(u[np.ix_(r, c)]))) <= 1 + 1e-12


# ---- integer semantics: arithmetic modulo 2^128 ------------------------------
def test_int128_wraparound():
    # per(c J_8) = 8! c^8 with c = 2^15 is about 5e40 > 2^127: the oracle returns
    # the residue modulo 2^128 in signed form.
    c = 1 << 15
    a = np.full((8, 8), c, dtype=np.int64)
    v = math.factorial(8) * c ** 8
    r = v % (1 << 128)
    if r >> 127:
        r -= 1 << 128
    assert oracle.per_brute(a) == r
    assert oracle.per_laplace(a) == r
    # a value just inside int128: per(J_33) = 33! < 2^127 would be too slow; use
    # 7 x 7 with entries 2^17: 7! 2^119 ~ 3.4e39 > 2^127 -> wraps too
    a = np.full((7, 7), 1 << 17, dtype=np.int64)
    v = math.factorial(7) * (1 << 17) ** 7
    r = v % (1 << 128)
    r = r - (1 << 128) if r >> 127 else r
    assert oracle.per_brute(a) == r


def test_negative_values_exact():
    a = -cf.ones(9, 9)
    assert oracle.per_brute(a) == -math.factorial(9)
    assert oracle.per_laplace(a) == -math.factorial(9)


# ---- the faster evaluators against the definition on every small shape -------
@pytest.mark.parametrize("n", range(1, 9))
def test_laplace_equals_definition_int(n):
    rng = np.random.default_rng(1000 + n)
    for m in range(1, n + 1):
        a = rng.integers(-3, 4, size=(m, n)).astype(np.int64)
        ref = oracle.per_brute(a)
        assert oracle.per_laplace(a, form=1) == ref
        assert oracle.per_laplace(a, form=2) == ref
        assert oracle.per_laplace(np.ascontiguousarray(a.T)) == ref
        assert oracle.per_glynn(a).frac() == ref
        assert oracle.per_ryser(a).frac() == ref


@pytest.mark.parametrize("n", range(1, 9))
def test_fp_evaluators_against_definition(n):
    rng = np.random.default_rng(2000 + n)
    for m in range(1, n + 1):
        a = rng.uniform(-1, 1, size=(m, n))
        absref = float(oracle.per_brute(np.abs(a)))
        ref = oracle.per_brute(a).frac()
        for ev in FP_EVALUATORS[1:]:
            assert abs(ev(a).frac() - ref) <= Fraction(4 * n * U * absref), (ev, m, n)
        z = workloads.complex_gauss(m, n, 3000 + 10 * n + m)
        refc = complex(oracle.per_brute(z))
        absz = float(oracle.per_brute(np.abs(z)))
        for ev in FP_EVALUATORS[1:]:
            assert abs(complex(ev(z)) - refc) <= 8 * n * U * absz + 1e-300


def test_glynn_partial_ranges_add_up():
    a = workloads.uniform(10, 10, 44)
    whole = oracle.per_glynn(a, partial=True).frac()
    parts = sum(oracle.per_glynn(a, k0=k, k1=k + 64, partial=True).frac() for k in range(0, 512, 64))
    assert abs(whole - parts) <= Fraction(1e-25) * (1 + abs(whole))
    assert abs(whole / 2 ** 9 - oracle.per_brute(a).frac()) <= Fraction(1e-12)


def test_thread_count_does_not_change_integer_result():
    a = rand_int(10, 10, 99, 0, 2)
    assert oracle.per_brute(a, nthreads=1) == oracle.per_brute(a, nthreads=5)
    assert oracle.per_laplace(a, nthreads=1) == oracle.per_laplace(a, nthreads=3)
