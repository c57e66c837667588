"""The largest vector lengths of each engine kind: real and complex Glynn at
n = 41 (the first order of the n = 41..48 instantiations), exact-integer
Glynn and Ryser at n = 40 (the integer limit), complex Glynn at n = 37 (one
wave per SIMD).

References: block-diagonal matrices with shuffled rows and columns.  Their
permanent is the product of the blocks' permanents (oracle; exact for
integer entries), and the absolute sum of Glynn's formula (Sec. 1.2
Eq. glynn) factorises over the blocks too,
    2^-(n-1) sum_{delta_1 = +1} prod_j |c_j(delta)| = 2^-n prod_b S_b,
    S_b = sum over all sign vectors of block b of prod_{j in b} |c_j|,
so the rounding bound of a binary64 evaluation is known at any size.  With
integer entries every column sum is exact, and only the products and the
accumulation round: |error| <= (n + 8) u per term, with a margin."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def block_matrix(sizes, seed, entries):
    """Block-diagonal matrix with the given block sizes, rows and columns
    shuffled; returns (matrix, blocks)."""
    rng = np.random.default_rng(seed)
    n = sum(sizes)
    blocks = [entries(rng, k) for k in sizes]
    dtype = np.result_type(*[b.dtype for b in blocks])
    a = np.zeros((n, n), dtype=dtype)
    o = 0
    for b in blocks:
        k = b.shape[0]
        a[o:o + k, o:o + k] = b
        o += k
    a = a[rng.permutation(n)][:, rng.permutation(n)]
    return np.ascontiguousarray(a), blocks


def block_abs_sum(blocks):
    """2^-n prod_b S_b: the absolute sum of Glynn's formula for the matrix."""
    total = 1.0
    n = 0
    for b in blocks:
        k = b.shape[0]
        n += k
        idx = np.arange(2 ** k)
        d = 1.0 - 2.0 * ((idx[:, None] >> np.arange(k)) & 1)
        total *= float(np.abs(np.prod(d @ b, axis=1)).sum())
    return total / 2.0 ** n


def exact_product(blocks):
    p = 1
    for b in blocks:
        p *= int(oracle.per_laplace(b.astype(np.int64)))
    return p


def small_ints(rng, k):
    return rng.integers(-3, 4, size=(k, k)).astype(np.float64)


def gauss_ints(rng, k):
    return (rng.integers(-2, 3, size=(k, k)) + 1j * rng.integers(-2, 3, size=(k, k))).astype(
        np.complex128)


def zero_one(rng, k):
    return (rng.random((k, k)) < 0.6).astype(np.uint8)


def test_real_glynn_n41():
    import paper_2510_03421_amd as pg
    a, blocks = block_matrix([8, 8, 8, 8, 9], 4101, small_ints)
    want = exact_product(blocks)
    hi, lo = pg.glynn(dev(a), out="dd").value()
    bound = 4 * (41 + 8) * U * block_abs_sum(blocks) + 4 * U * abs(want)
    assert abs((hi + lo) - want) <= bound, (hi + lo, want, bound)


def test_complex_glynn_n37_and_n41():
    import paper_2510_03421_amd as pg
    for n, sizes, seed in [(37, [7, 7, 7, 8, 8], 3701), (41, [8, 8, 8, 8, 9], 4102)]:
        a, blocks = block_matrix(sizes, seed, gauss_ints)
        want = 1
        for b in blocks:
            r = oracle.per_laplace(b)
            want *= complex(r.re.hi + r.re.lo, r.im.hi + r.im.lo)
        got = pg.glynn(dev(a)).value()
        # a complex product rounds each factor by at most about 3u in modulus
        bound = 16 * (n + 8) * U * block_abs_sum(blocks) + 8 * U * abs(want)
        assert abs(got - want) <= bound, (n, got, want, bound)


def test_integer_glynn_and_ryser_n40():
    import paper_2510_03421_amd as pg
    b, blocks = block_matrix([8, 8, 8, 8, 8], 4001, zero_one)
    want = exact_product(blocks)
    assert pg.glynn(dev(b)).value() == want          # int128, n - 1 = 39 sign bits
    assert pg.ryser(dev(b)).value() == want          # int128, 2^40 column sets
    # the same matrix as binary64: every column sum and partial product is an
    # integer below 2^53 except the full products, so only the bound holds
    f = pg.glynn(dev(b.astype(np.float64)), out="dd").value()
    bound = 4 * (40 + 8) * U * block_abs_sum([x.astype(np.float64) for x in blocks]) + 4 * U * want
    assert abs((f[0] + f[1]) - want) <= bound
