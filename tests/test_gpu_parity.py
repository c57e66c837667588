"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer results must match bit for bit.  Floating-point results must satisfy
|gpu - ref| <= 1e-11 per(|A|) (the criterion the library is built to), and
the tests additionally check a tighter, size-aware bound derived from the
arithmetic: each of the T terms carries a relative rounding error of a few
n u, so |error| <= c n u per(|A|) for a small constant c.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads
from tests import closed_forms as cf
from tests.gpu_util import dev, run_algo, ref_value, abs_ref, ALGOS, formula_abs_sums

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
CRIT = 1e-11


def check_fp(got, ref, absref, n, tight=64.0, label=""):
    err = abs(complex(got) - complex(ref))
    assert err <= CRIT * absref + 1e-300, (label, got, ref, absref)
    assert err <= tight * n * U * absref + 1e-300, (label, got, ref, absref, err / absref)


# ---- the paper's worked example -------------------------------------------
@pytest.mark.parametrize("algo", ALGOS)
def test_worked_example(algo):
    a, want = cf.read_worked_example()
    assert run_algo(algo, dev(a)) == want
    assert run_algo(algo, dev(a.astype(np.uint8) % 2)) == oracle.per_brute(a % 2)
    assert run_algo(algo, dev(a.astype(np.float64))) == float(want)
    assert run_algo(algo, dev(a.astype(np.complex128) * (1 + 1j))) == complex(want * (1 + 1j) ** 3)


# ---- every small shape against the definition -------------------------------
SHAPES = [(m, n) for n in range(1, 9) for m in range(1, n + 1)]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("m,n", SHAPES)
def test_small_int_exact(algo, m, n):
    rng = np.random.default_rng(100 * m + n)
    a = rng.integers(-3, 4, size=(m, n)).astype(np.int64)
    want = oracle.per_brute(a)
    assert run_algo(algo, dev(a)) == want
    assert run_algo(algo, dev(np.ascontiguousarray(a.T))) == want   # m > n: per(A^T)
    b = (rng.random((m, n)) < 0.6).astype(np.uint8)
    assert run_algo(algo, dev(b)) == oracle.per_brute(b.astype(np.int64))


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("m,n", SHAPES)
def test_small_fp(algo, m, n):
    a = workloads.uniform(m, n, 7000 + 10 * m + n)
    ref = oracle.per_brute(a)
    check_fp(run_algo(algo, dev(a)), float(ref), float(oracle.per_brute(np.abs(a))), n,
             label=(algo, m, n))
    z = workloads.complex_gauss(m, n, 8000 + 10 * m + n)
    refz = complex(oracle.per_brute(z))
    check_fp(run_algo(algo, dev(z)), refz, float(oracle.per_brute(np.abs(z))), n,
             label=(algo, m, n, "c"))
    got_t = run_algo(algo, dev(np.ascontiguousarray(z.T)))
    check_fp(got_t, refz, float(oracle.per_brute(np.abs(z))), n, label=(algo, m, n, "cT"))


def test_strided_input():
    # lda > n: a view into a wider buffer
    big = workloads.uniform(9, 13, 5)
    a = big[:, 2:9]
    ref = float(oracle.per_brute(np.ascontiguousarray(a)))
    import torch
    t = torch.from_numpy(big).cuda()[:, 2:9]
    assert t.stride(0) == 13
    for algo in ALGOS:
        got = run_algo(algo, t)
        assert abs(got - ref) <= 1e-12 * float(oracle.per_brute(np.abs(a)))


# ---- closed forms ------------------------------------------------------------
@pytest.mark.parametrize("n", [9, 12, 16, 20])
def test_ones_and_identity(n):
    for m in (n // 2, n - 1, n):
        j = np.ones((m, n), dtype=np.uint8)
        want = cf.ones_value(m, n)
        assert run_algo("ryser", dev(j)) == want
        if m == n or n <= 16:
            assert run_algo("glynn", dev(j), flags=1) == want
        i = cf.identity_rect(m, n)
        assert run_algo("ryser", dev(i)) == 1
        assert run_algo("glynn", dev(i)) == 1
        assert run_algo("ryser", dev(i.astype(np.float64))) == 1.0


@pytest.mark.parametrize("n", [10, 16, 20, 24])
def test_derangements_and_graph_counts(n):
    assert run_algo("ryser", dev(cf.derangement_matrix(n).astype(np.uint8))) == cf.derangements(n)
    assert run_algo("glynn", dev(cf.derangement_matrix(n).astype(np.uint8))) == cf.derangements(n)
    assert run_algo("ryser", dev(cf.tridiagonal_ones(n).astype(np.uint8))) == cf.fibonacci(n + 1)
    assert run_algo("glynn", dev(cf.hessenberg_ones(n).astype(np.uint8))) == 2 ** (n - 1)
    assert run_algo("glynn", dev(cf.cycle_plus_identity(n).astype(np.uint8))) == 2
    m = n // 2
    assert run_algo("ryser", dev(cf.rect_derangement_matrix(m, n).astype(np.uint8))) == \
        cf.rect_derangements(m, n)


@pytest.mark.parametrize("n", [8, 14, 20])
def test_cauchy_borchardt(n):
    """Sec. 1.4 Eq. caucy_permanent (Borchardt) as the exact value.  All entries
    are positive, so per(|C|) = per(C) and the 1e-11 per(|A|) criterion is a
    relative bound.  Glynn meets it; Ryser's alternating sum has a condition
    number sum|terms|/per of 4e3 / 7e6 / 1e10 at n = 8 / 14 / 20 and loses
    that many digits in binary64 (the paper reports all algorithms losing
    precision on larger Cauchy matrices, Sec. 4).  Both are held to the bound
    the arithmetic gives: a few n u times the formula's absolute sum."""
    c, x, y = workloads.cauchy_dyadic(n, n, seed=400 + n)
    exact = float(cf.cauchy_borchardt(x, y))
    ryser_abs, glynn_abs = formula_abs_sums(c)
    input_err = (n + 2) * U * exact           # entries rounded once each
    got = run_algo("glynn", dev(c))
    assert abs(got - exact) <= 1e-11 * exact
    assert abs(got - exact) <= 4 * n * U * glynn_abs + input_err
    got = run_algo("ryser", dev(c))
    assert abs(got - exact) <= 4 * n * U * ryser_abs + input_err, (got, exact)
    if n <= 12:
        assert abs(got - exact) <= 1e-11 * exact


def test_rank_one_integer():
    rng = np.random.default_rng(3)
    for m, n in [(10, 10), (8, 14), (12, 20)]:
        u = [int(x) for x in rng.integers(1, 4, size=m)]
        v = [int(x) for x in rng.integers(-2, 3, size=n)]
        a = np.outer(u, v).astype(np.int64)
        want = cf.rank_one_value(u, v)
        assert run_algo("ryser", dev(a)) == want
        assert run_algo("glynn", dev(a)) == want


# ---- the 12 x 12 workload against the definition ------------------------------
def test_u12_against_definition():
    a = workloads.config_matrix("u12")
    ref = oracle.per_brute(a)
    absref = float(oracle.per_brute(np.abs(a)))
    for algo in ALGOS:
        check_fp(run_algo(algo, dev(a)), float(ref), absref, 12, label=algo)


# ---- integers: overflow handling ------------------------------------------------
def test_overflow_precheck_and_wrap():
    import paper_2510_03421_amd as pg
    j = np.ones((25, 25), dtype=np.int64) * 3
    # per = 25! 3^25 ~ 1.3e37: fits int128 but not int64
    want = math.factorial(25) * 3 ** 25
    assert run_algo("ryser", dev(j)) == want
    with pytest.raises(pg.PermError) as e:
        run_algo("ryser", dev(j), out="i64")
    assert e.value.status == -3
    # 30 x 30 of 7s: ~ 6e57, beyond int128 -> refused, unless wrapping is asked
    k = np.full((14, 14), 1 << 20, dtype=np.int64)
    big = math.factorial(14) * (1 << 20) ** 14
    with pytest.raises(pg.PermError):
        run_algo("ryser", dev(k))
    r = big % (1 << 128)
    r = r - (1 << 128) if r >> 127 else r
    assert run_algo("ryser", dev(k), flags=1) == r
    assert run_algo("combinatoric", dev(k[:8, :8]), flags=1) == \
        oracle.per_brute(k[:8, :8])


# ---- argument errors -----------------------------------------------------------
def test_argument_errors():
    import ctypes

    import torch

    import paper_2510_03421_amd as pg
    from paper_2510_03421_amd import _capi as C
    a = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    f = C.lib.perm_glynn
    assert f(4, 4, C.PERM_F64, None, 4, C.PERM_OUT_F64, out.data_ptr(), 0, s) == C.PERM_E_INVALID
    assert f(4, 4, C.PERM_F64, a.data_ptr(), 3, C.PERM_OUT_F64, out.data_ptr(), 0, s) == \
        C.PERM_E_INVALID
    assert f(4, 4, C.PERM_F64, a.data_ptr(), 4, C.PERM_OUT_I128, out.data_ptr(), 0, s) == \
        C.PERM_E_INVALID
    assert f(4, 4, C.PERM_F64, a.data_ptr(), 4, C.PERM_OUT_F64, None, 0, s) == C.PERM_E_INVALID
    assert f(-1, 4, C.PERM_F64, a.data_ptr(), 4, C.PERM_OUT_F64, out.data_ptr(), 0, s) == \
        C.PERM_E_INVALID
    assert f(4, 4, 9, a.data_ptr(), 4, C.PERM_OUT_F64, out.data_ptr(), 0, s) == C.PERM_E_INVALID
    assert f(4, 65, C.PERM_F64, a.data_ptr(), 65, C.PERM_OUT_F64, out.data_ptr(), 0, s) == \
        C.PERM_E_TOO_LARGE
    assert C.lib.perm_combinatoric(16, 16, C.PERM_F64, a.data_ptr(), 16, C.PERM_OUT_F64,
                                   out.data_ptr(), 0, s) == C.PERM_E_TOO_LARGE
    # nothing was written
    out.fill_(7.0)
    f(4, 4, C.PERM_F64, a.data_ptr(), 3, C.PERM_OUT_F64, out.data_ptr(), 0, s)
    torch.cuda.synchronize()
    assert out[0].item() == 7.0


def test_empty_and_degenerate():
    import torch
    for algo in ALGOS:
        assert run_algo(algo, torch.zeros((0, 5), dtype=torch.float64, device="cuda")) == 1.0
        assert run_algo(algo, torch.zeros((0, 0), dtype=torch.int64, device="cuda")) == 1
        assert run_algo(algo, dev(np.array([[2.5]]))) == 2.5
        assert run_algo(algo, dev(np.array([[1, 2, 3, 4]]))) == 10
        assert run_algo(algo, dev(np.zeros((5, 5)))) == 0.0
        z = np.ones((5, 7))
        z[2, :] = 0
        assert run_algo(algo, dev(z)) == 0.0
