"""Square Glynn (n <= 16) and square Ryser (n <= 15) run in one workgroup
and one launch (staging, walk, reduction and normalisation together).  These
tests hold that path to the oracle at the orders on both sides of its limit
(13..16 for Glynn, 13..16 for Ryser: 16 runs on the multi-kernel engine),
for real, complex and exact-integer outputs, and compare it with the engine's
whole-width chunk (perm_gray_chunk always runs the engine) within the
formulas' rounding bound."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev, formula_abs_sums

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def dd_value(r):
    return r.hi + r.lo


@pytest.mark.parametrize("n", [13, 14, 15, 16])
def test_real_against_oracle_and_engine(n):
    import paper_2510_03421_amd as pg
    a_h = workloads.uniform(n, n, 7700 + n)
    a = dev(a_h)
    want = dd_value(oracle.per_laplace(a_h))
    ryser_abs, glynn_abs = formula_abs_sums(a_h)
    g = pg.glynn(a, out="dd").value()
    r = pg.ryser(a, out="dd").value()
    assert abs((g[0] + g[1]) - want) <= 8 * (n + 8) * U * glynn_abs, (n, g, want)
    assert abs((r[0] + r[1]) - want) <= 8 * (n + 8) * U * ryser_abs, (n, r, want)
    # the engine's walk of the same sum (one chunk of full width)
    ge = pg.gray_chunk(a, "glynn", n - 1, 0, out="dd").value()
    re = pg.gray_chunk(a, "ryser", n, 0, out="dd").value()
    assert abs((g[0] + g[1]) - (ge[0] + ge[1])) <= 16 * (n + 8) * U * glynn_abs
    assert abs((r[0] + r[1]) - (re[0] + re[1])) <= 16 * (n + 8) * U * ryser_abs


@pytest.mark.parametrize("n", [13, 16])
def test_complex_against_oracle(n):
    import paper_2510_03421_amd as pg
    a_h = workloads.complex_gauss(n, n, 7800 + n)
    want = oracle.per_laplace(a_h)
    want = complex(want.re.hi + want.re.lo, want.im.hi + want.im.lo)
    scale = dd_value(oracle.per_laplace(np.abs(a_h)))
    for fn in (pg.glynn, pg.ryser):
        got = fn(dev(a_h)).value()
        assert abs(got - want) <= 1e-11 * scale, (n, fn, got, want)
    ge = pg.gray_chunk(dev(a_h), "glynn", n - 1, 0).value()
    assert abs(pg.glynn(dev(a_h)).value() - ge) <= 1e-13 * scale


@pytest.mark.parametrize("n", [13, 15, 16])
def test_exact_integers(n):
    import paper_2510_03421_amd as pg
    rng = np.random.default_rng(7900 + n)
    a = rng.integers(-4, 5, size=(n, n)).astype(np.int64)
    want = oracle.per_laplace(a)
    assert pg.glynn(dev(a)).value() == want
    assert pg.ryser(dev(a)).value() == want
    b = (rng.random((n, n)) < 0.5).astype(np.uint8)
    wb = oracle.per_laplace(b.astype(np.int64))
    assert pg.ryser(dev(b)).value() == wb
    assert pg.glynn(dev(b)).value() == wb
    assert pg.ryser(dev(b), out="i64").value() == wb
    # transposed and strided reads
    assert pg.ryser(dev(np.ascontiguousarray(a.T))).value() == want
    import torch
    big = torch.zeros(n, n + 5, dtype=torch.int64)
    big[:, :n] = torch.from_numpy(a)
    assert pg.glynn(big.cuda()[:, :n]).value() == want


def test_orders_one_to_three_and_profile():
    import paper_2510_03421_amd as pg
    assert pg.glynn(dev(np.array([[2.5]]))).value() == 2.5
    assert pg.ryser(dev(np.array([[-3]], dtype=np.int64))).value() == -3
    a = np.array([[1.0, 2.0], [3.0, 4.0]])
    assert pg.glynn(dev(a)).value() == 10.0 and pg.ryser(dev(a)).value() == 10.0
    b = np.arange(1, 10, dtype=np.int64).reshape(3, 3)
    assert pg.glynn(dev(b)).value() == 450 and pg.ryser(dev(b)).value() == 450
    # the one-launch path records its kernel for the timing API too
    pg.profile_enable(True)
    try:
        pg.glynn(dev(workloads.uniform(12, 12, 1201)))
        assert pg.profile_last_ms() > 0.0
    finally:
        pg.profile_enable(False)
