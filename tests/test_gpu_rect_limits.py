"""Rectangular Ryser by size (Sec. 1.2 Eq. ryser_rectangle) at its size
limits: 64 columns (the widest subset walk the library accepts), short and
transposed shapes, real, complex and exact-integer inputs, against the
oracle's memoised Laplace sum (memory 2^m), and the refusals just past the
limits."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev, run_algo

pytestmark = pytest.mark.gpu

CRIT = 1e-11      # |error| <= 1e-11 per(|A|)

WIDE = [(1, 64, 1), (2, 64, 2), (3, 64, 3), (5, 64, 4), (8, 64, 5), (10, 64, 6), (7, 57, 7),
        (11, 64, 8)]


def dd_value(r):
    return r.hi + r.lo


@pytest.mark.parametrize("m,n,seed", WIDE)
def test_wide_real(m, n, seed):
    a = workloads.uniform(m, n, 6400 + seed)
    want = dd_value(oracle.per_laplace(a))
    scale = dd_value(oracle.per_laplace(np.abs(a)))
    got = run_algo("ryser", dev(a))
    assert abs(got - want) <= CRIT * scale, (got, want, scale)
    # m > n reads A^T in place: the same sum
    got_t = run_algo("ryser", dev(np.ascontiguousarray(a.T)))
    assert abs(got_t - want) <= CRIT * scale, (got_t, want, scale)


@pytest.mark.parametrize("m,n,seed", WIDE[:6])
def test_wide_complex(m, n, seed):
    z = workloads.complex_gauss(m, n, 6500 + seed)
    r = oracle.per_laplace(z)
    want = complex(dd_value(r.re), dd_value(r.im))
    scale = dd_value(oracle.per_laplace(np.abs(z)))
    got = run_algo("ryser", dev(z))
    assert abs(got - want) <= CRIT * scale, (got, want, scale)


@pytest.mark.parametrize("m,n,seed", [(1, 64, 1), (3, 64, 2), (6, 64, 3), (9, 64, 4), (11, 60, 5)])
def test_wide_integer_exact(m, n, seed):
    rng = np.random.default_rng(6600 + seed)
    a = rng.integers(-3, 4, size=(m, n)).astype(np.int64)
    want = oracle.per_laplace(a)
    assert run_algo("ryser", dev(a)) == want
    b = (rng.random((m, n)) < 0.4).astype(np.uint8)
    assert run_algo("ryser", dev(b)) == oracle.per_laplace(b.astype(np.int64))
    assert run_algo("ryser", dev(np.ascontiguousarray(b.T))) == \
        oracle.per_laplace(b.astype(np.int64))


def test_auto_at_64_columns_and_refusals():
    import paper_2510_03421_amd as pg
    a = workloads.uniform(3, 64, 6701)
    want = dd_value(oracle.per_laplace(a))
    scale = dd_value(oracle.per_laplace(np.abs(a)))
    r = pg.auto(dev(a))
    # Glynn (n <= 48) and the e_m form (n <= 48) refuse 64 columns; Ryser by
    # size and the definition (64 * 63 * 62 maps) both run
    assert pg.ALGORITHMS[r.algo] in ("ryser", "combinatoric")
    assert abs(r.value() - want) <= CRIT * scale
    for shape, fn in [((3, 65), pg.ryser), ((41, 64), pg.ryser), ((3, 49), pg.glynn),
                      ((3, 64), pg.glynn)]:
        with pytest.raises(pg.PermError) as ei:
            fn(dev(np.ones(shape)))
        assert ei.value.status == -2, (shape, fn)
