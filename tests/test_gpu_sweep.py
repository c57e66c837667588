"""The column sweep (perm_column_sweep) against the oracle: bit-exact for
integer outputs and integer-valued floating-point inputs, within its
summation bound (no cancellation of computed values) on real and complex
inputs, accurate where the inclusion-exclusion forms lose digits (positive
Cauchy matrices), and at full size on the 20 x 40, 16 x 48 and 28 x 28
workloads."""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests import closed_forms as cf
from tests.gpu_util import abs_ref, dev, golden, ref_value

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def run(a, out=None, flags=0):
    import paper_2510_03421_amd as pg
    return pg.column_sweep(dev(a), out=out, flags=flags).value()


SHAPES = [(m, n) for n in range(1, 9) for m in range(1, n + 1)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_small_exact(m, n):
    rng = np.random.default_rng(800 * m + n)
    a = rng.integers(-4, 5, size=(m, n))
    want = oracle.per_brute(a.astype(np.int64))
    assert run(a.astype(np.int64)) == want
    assert run(np.ascontiguousarray(a.T).astype(np.int64)) == want        # m > n
    assert run(a.astype(np.float64)) == float(want)                        # exact in binary64
    z = a.astype(np.complex128) * (2 + 1j)
    assert run(z) == complex(want * (2 + 1j) ** m)
    b = (rng.random((m, n)) < 0.5).astype(np.uint8)
    assert run(b) == oracle.per_brute(b.astype(np.int64))


@pytest.mark.parametrize("m,n,seed", [(6, 9, 1), (10, 14, 2), (12, 12, 3), (14, 30, 4), (18, 22, 5),
                                      (20, 48, 6)])
def test_random_within_summation_bound(m, n, seed):
    """Each state sums products of input entries; the rounding error of the
    result is at most about (m + n) u per(|A|) (forward error of a sum of
    products of length m + n)."""
    a = workloads.uniform(m, n, 8100 + seed)
    ref = oracle.per_laplace(a)
    pabs = oracle.per_laplace(np.abs(a))
    got = run(a)
    assert abs(got - (ref.hi + ref.lo)) <= 2 * (m + n) * U * pabs.hi, (got, ref)
    z = workloads.complex_gauss(m, n, 8200 + seed)
    rz = oracle.per_laplace(z)
    pz = oracle.per_laplace(np.abs(z))
    gz = run(z)
    err = abs(gz - complex(rz.re.hi + rz.re.lo, rz.im.hi + rz.im.lo))
    assert err <= 4 * (m + n) * U * pz.hi, (gz, rz)


@pytest.mark.parametrize("n", [14, 20])
def test_positive_cauchy_keeps_its_digits(n):
    """C_ij = 1 / (x_i - y_j) > 0: per(|C|) = per(C), so the sweep is accurate
    to a few (2n) u in relative terms, where Ryser's signed sum over subsets
    loses several digits (Borchardt's identity gives the exact value)."""
    import paper_2510_03421_amd as pg
    c, x, y = workloads.cauchy_dyadic(n, n, 8300 + n)
    exact = cf.cauchy_borchardt(x, y)
    # the input is the rounded matrix: compare with the oracle on the same input
    ref = oracle.per_laplace(c)
    got = run(c)
    assert abs(got - (ref.hi + ref.lo)) <= 4 * n * U * abs(ref.hi)
    # the rounded input differs from the exact Cauchy matrix by ~n u relative
    assert abs(got - float(exact)) <= 8 * n * U * abs(float(exact))
    r = pg.ryser(dev(c)).value()
    assert abs(got - (ref.hi + ref.lo)) < abs(r - (ref.hi + ref.lo)) or r == got


def test_full_size_workloads():
    rec = golden()["u20x40"]
    a = workloads.config_matrix("u20x40")
    got = run(a)
    assert abs(got - ref_value(rec)) <= 2 * 60 * U * abs_ref(rec)
    assert abs(got - ref_value(rec)) <= 1e-11 * abs_ref(rec)
    b = workloads.config_matrix("b16x48")
    assert run(b) == ref_value(golden()["b16x48"])
    b28 = workloads.config_matrix("b28")
    assert run(b28) == ref_value(golden()["b28"])


def test_closed_forms_and_limits():
    import paper_2510_03421_amd as pg
    assert run(cf.derangement_matrix(20).astype(np.uint8)) == cf.derangements(20)
    assert run(cf.rect_derangement_matrix(12, 40).astype(np.uint8)) == cf.rect_derangements(12, 40)
    assert run(np.ones((10, 25), dtype=np.uint8)) == cf.ones_value(10, 25)
    assert run(np.zeros((0, 4))) == 1.0
    with pytest.raises(pg.PermError) as ei:
        run(np.ones((29, 30)))
    assert ei.value.status == -2
    # 0/1 input whose permanent cannot exceed 2^127 needs no wrap; a large one
    # is refused unless PERM_FLAG_WRAP (then exact modulo 2^128)
    big = np.full((20, 20), 1 << 20, dtype=np.int64)
    with pytest.raises(pg.PermError) as ei:
        run(big)
    assert ei.value.status == -3
    got = run(big, flags=pg._capi.PERM_FLAG_WRAP)
    assert (got - math.factorial(20) * 2 ** 400) % 2 ** 128 == 0
