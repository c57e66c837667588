"""Chunks of the Gray-code sums (perm_gray_chunk) against the oracle's sums
over the same Gray-index ranges, chunk by chunk, and their totals against the
whole-sum entry points: the sharding (or resume) of one permanent."""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev, golden, ref_value

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def chunk_values(a, algo, B, flags=0, out=None):
    """Every chunk of width 2^B, as Python complex numbers (dd summed)."""
    import paper_2510_03421_amd as pg
    m, n = sorted(a.shape)
    nbits = (n - 1) if algo == "glynn" else n
    vals = []
    for c in range(2 ** (nbits - B)):
        v = pg.gray_chunk(a, algo, B, c, out=out, flags=flags).value()
        if out == "cdd":
            vals.append(complex(v[0][0] + v[0][1], v[1][0] + v[1][1]))
        elif out == "dd":
            vals.append(complex(v[0] + v[1]))
        else:
            vals.append(complex(v))
    return vals


def chunk_abs_sums(a, B, pad=1.0):
    """Per chunk of 2^B Gray indices: the sum of |terms| of Glynn's formula
    on a (padded with rows of `pad`), scaled as the sum is -- the scale of
    the chunk's rounding error."""
    m, n = a.shape
    ap = np.vstack([a, np.full((n - m, n), pad, dtype=a.dtype)])
    k = np.arange(2 ** (n - 1), dtype=np.int64)
    g = k ^ (k >> 1)
    d = np.ones((len(k), n))
    d[:, 1:] = 1 - 2 * ((g[:, None] >> np.arange(n - 1)) & 1)
    terms = np.abs(np.prod(d @ ap, axis=1))
    per_chunk = terms.reshape(-1, 2 ** B).sum(axis=1)
    return per_chunk / 2.0 ** (n - 1) / math.factorial(n - m)


def dd_sum(vals):
    return complex(math.fsum(v.real for v in vals), math.fsum(v.imag for v in vals))


@pytest.mark.parametrize("cplx", [False, True])
def test_each_chunk_matches_the_oracle_range(cplx):
    """12 x 12 Glynn in 32 chunks of 2^6 terms: each chunk against the oracle's
    double-double sum over the same Gray indices (scaled as the whole sum)."""
    import paper_2510_03421_amd as pg
    a_h = workloads.complex_gauss(12, 12, 8101) if cplx else workloads.uniform(12, 12, 8101)
    a = dev(a_h)
    out = "cdd" if cplx else "dd"
    vals = chunk_values(a, "glynn", 6, out=out)
    scale = float(oracle.per_laplace(np.abs(a_h)))
    bound = chunk_abs_sums(a_h, 6)
    for c, v in enumerate(vals):
        r = oracle.per_glynn(a_h, k0=c * 64, k1=(c + 1) * 64)
        want = complex(r) if cplx else complex(r.hi + r.lo)
        assert abs(v - want) <= 8 * 12 * U * bound[c], (c, v, want, bound[c])
    whole = pg.glynn(a, out=out).value()
    whole = complex(whole[0][0] + whole[0][1], whole[1][0] + whole[1][1]) if cplx else \
        complex(whole[0] + whole[1])
    assert abs(dd_sum(vals) - whole) <= 1e-13 * scale


def test_rectangular_ones_padding_chunks_match_the_oracle():
    """6 x 14 with the printed rows of ones: every chunk against the oracle's
    padded sum over the same range; the default (scaled padding) chunks add
    up to the permanent."""
    import paper_2510_03421_amd as pg
    from paper_2510_03421_amd import _capi as C
    a_h = workloads.uniform(6, 14, 8102)
    a = dev(a_h)
    vals = chunk_values(a, "glynn", 9, flags=C.PERM_FLAG_PAD_ONES, out="dd")
    bound = chunk_abs_sums(a_h, 9)
    for c, v in enumerate(vals):
        r = oracle.per_glynn(a_h, k0=c * 512, k1=(c + 1) * 512)
        want = r.hi + r.lo
        assert abs(v.real - want) <= 8 * 14 * U * bound[c], (c, v, want, bound[c])
    ref = oracle.per_laplace(a_h)
    ref = ref.hi + ref.lo
    scaled = dd_sum(chunk_values(a, "glynn", 9, out="dd")).real
    assert abs(scaled - ref) <= 1e-12 * abs(ref)


def test_u32_in_16_chunks_and_the_whole_chunk():
    """The 32 x 32 workload summed from 16 chunks of 2^27 terms equals the
    single call to rounding; the chunk of width 2^31 is the single call,
    bitwise."""
    import paper_2510_03421_amd as pg
    rec = golden()["u32"]
    a = dev(workloads.config_matrix("u32"))
    whole = pg.glynn(a, out="dd").value()
    assert pg.gray_chunk(a, "glynn", 31, 0, out="dd").value() == whole
    total = dd_sum(chunk_values(a, "glynn", 27, out="dd")).real
    assert abs(total - (whole[0] + whole[1])) <= 1e-12 * abs(whole[0])
    assert abs(total - ref_value(rec)) <= 1e-11 * abs(ref_value(rec))


def test_ryser_square_chunks():
    import paper_2510_03421_amd as pg
    a_h = workloads.uniform(20, 20, 8103)
    a = dev(a_h)
    whole = pg.ryser(a, out="dd").value()
    assert pg.gray_chunk(a, "ryser", 20, 0, out="dd").value() == whole
    total = dd_sum(chunk_values(a, "ryser", 16, out="dd")).real
    pabs = float(oracle.per_laplace(np.abs(a_h)))
    assert abs(total - (whole[0] + whole[1])) <= 1e-11 * pabs
    ref = oracle.per_laplace(a_h)
    assert abs(total - (ref.hi + ref.lo)) <= 1e-11 * pabs


def test_chunk_arguments():
    import torch

    import paper_2510_03421_amd as pg
    a = dev(workloads.uniform(8, 8, 8104))
    bad = [("glynn", 0, 0), ("glynn", 8, 0), ("glynn", 3, 16), ("ryser", 9, 0)]
    for algo, B, c in bad:
        with pytest.raises(pg.PermError) as ei:
            pg.gray_chunk(a, algo, B, c)
        assert ei.value.status == -1, (algo, B, c)
    with pytest.raises(pg.PermError) as ei:                       # integer outputs
        pg.gray_chunk(dev(np.ones((5, 5), dtype=np.uint8)), "glynn", 2, 0)
    assert ei.value.status == -5
    with pytest.raises(pg.PermError) as ei:                       # rectangular Ryser
        pg.gray_chunk(dev(workloads.uniform(3, 6, 1)), "ryser", 3, 0)
    assert ei.value.status == -5
    with pytest.raises(pg.PermError) as ei:
        pg.gray_chunk(a, "combinatoric", 3, 0)
    assert ei.value.status == -5
    assert pg.gray_chunk(torch.zeros((0, 4), dtype=torch.float64, device="cuda"), "glynn", 0, 0
                         ).value() == 1.0
    one = dev(np.array([[2.5]]))
    assert pg.gray_chunk(one, "glynn", 0, 0).value() == 2.5
