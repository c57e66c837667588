"""The e_m form of the rectangular Glynn sum (perm_glynn_esym) against the
oracle: bit-exact for integer outputs and for floating-point results on
integer-valued inputs below 2^53, within the rounding bound of the formula on
real and complex inputs, and at full size on the 20x40 and 16x48 workloads."""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev, golden, ref_value, abs_ref

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def run(a, out=None):
    import paper_2510_03421_amd as pg
    return pg.glynn_esym(dev(a), out=out).value()


def esym_abs_sum(a):
    """2^-(m-1) sum over sign vectors (delta_1 = +1) of e_m(|c(delta)|), c the
    column sums: each term of the formula is evaluated with a relative error
    of a few n u against this scale."""
    m, n = a.shape
    tot = 0.0
    for bits in range(2 ** (m - 1)):
        d = np.array([1] + [(-1) ** ((bits >> i) & 1) for i in range(m - 1)])
        c = np.abs(d @ a)
        e = np.zeros(m + 1)
        e[0] = 1.0
        for j in range(n):
            e[1:] = e[1:] + c[j] * e[:-1]
        tot += e[m]
    return tot / 2 ** (m - 1)


SHAPES = [(m, n) for n in range(1, 9) for m in range(1, n + 1)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_small_integer_valued_exact(m, n):
    rng = np.random.default_rng(300 * m + n)
    a = rng.integers(-3, 4, size=(m, n))
    want = oracle.per_brute(a.astype(np.int64))
    assert run(a.astype(np.float64)) == float(want)
    assert run(np.ascontiguousarray(a.T).astype(np.float64)) == float(want)   # m > n
    z = a.astype(np.complex128) * (1 - 2j)
    assert run(z) == complex(want * (1 - 2j) ** m)
    assert run(a.astype(np.int64)) == want                       # exact int128 output
    b = (rng.random((m, n)) < 0.6).astype(np.uint8)
    assert run(b) == oracle.per_brute(b.astype(np.int64))


@pytest.mark.parametrize("m,n,seed", [(3, 11, 1), (6, 14, 2), (9, 20, 3), (12, 24, 4), (12, 12, 5),
                                      (5, 40, 6), (1, 30, 7)])
def test_random_against_oracle(m, n, seed):
    a = workloads.uniform(m, n, 9100 + seed)
    ref = oracle.per_laplace(a)
    want = ref.hi + ref.lo
    got = run(a)
    bound = 8 * n * U * esym_abs_sum(a) + 4 * U * abs(want)
    assert abs(got - want) <= bound, (got, want, bound)
    z = workloads.complex_gauss(m, n, 9200 + seed)
    refz = oracle.per_laplace(z)
    wz = complex(refz.re.hi + refz.re.lo, refz.im.hi + refz.im.lo)
    gz = run(z)
    bz = 16 * n * U * esym_abs_sum(np.abs(z)) + 4 * U * abs(wz)
    assert abs(gz - wz) <= bz, (gz, wz, bz)


def test_u20x40_full_size():
    rec = golden()["u20x40"]
    a = workloads.config_matrix("u20x40")
    want = ref_value(rec)
    got = run(a)
    assert abs(got - want) <= 1e-11 * abs_ref(rec)        # the accuracy criterion
    assert abs(got - want) <= 1e-12 * abs(want)            # and far inside it
    hi, lo = run(a, out="dd")
    assert abs((hi + lo) - want) <= 1e-12 * abs(want)


def test_b16x48_full_size():
    rec = golden()["b16x48"]
    b = workloads.config_matrix("b16x48")
    want = ref_value(rec)
    assert run(b) == want                                  # bit-exact, int128
    got = run(b.astype(np.float64))
    assert abs(got - want) <= 1e-12 * want, (got, want)


def test_integer_overflow_precheck_and_wrap():
    import paper_2510_03421_amd as pg
    # 20 x 30 ones: per = 30!/10! ~ 2^86; the e_m sum 2^19 per fits int128
    assert run(np.ones((20, 30), dtype=np.uint8)) == math.factorial(30) // math.factorial(10)
    # 32 x 40 ones: per = 40!/8! ~ 2^144 does not fit: refused ...
    big = np.ones((32, 40), dtype=np.uint8)
    with pytest.raises(pg.PermError) as ei:
        run(big)
    assert ei.value.status == -3
    # ... and with PERM_FLAG_WRAP exact modulo 2^(128 - 31)
    got = pg.glynn_esym(dev(big), flags=pg._capi.PERM_FLAG_WRAP).value()
    assert (got - math.factorial(40) // math.factorial(8)) % 2 ** 97 == 0


def test_square_matches_glynn_and_limits():
    import paper_2510_03421_amd as pg
    a = workloads.uniform(14, 14, 9301)
    g = pg.glynn(dev(a)).value()
    e = run(a)
    assert abs(g - e) <= 1e-13 * oracle.per_laplace(np.abs(a)).hi
    assert run(np.zeros((0, 5))) == 1.0
    with pytest.raises(pg.PermError) as ei:
        run(np.ones((33, 40)))
    assert ei.value.status == -2
    with pytest.raises(pg.PermError) as ei:
        run(np.ones((3, 49)))
    assert ei.value.status == -2
    assert pg.glynn_esym(dev(np.ones((3, 5), dtype=np.uint8))).value() == 60
    assert pg.glynn_esym(dev(np.ones((3, 5), dtype=np.uint8)), out="f64").value() == 60.0


def test_auto_uses_the_e_m_form_when_it_needs_far_fewer_operations():
    import paper_2510_03421_amd as pg
    rec = golden()["u20x40"]
    r = pg.auto(dev(workloads.config_matrix("u20x40")))
    assert pg.ALGORITHMS[r.algo] == "glynn_esym"
    assert abs(r.value() - ref_value(rec)) <= 1e-12 * abs(ref_value(rec))
    # square at 28 the stored timings give the e_m form 0.52 ms against
    # Glynn's 0.30 ms, so it is not chosen.  (At 14 x 15 both
    # take launch time, and the stored timings favour the e_m form.)
    a = workloads.uniform(28, 28, 9401)
    r = pg.auto(dev(a))
    assert pg.ALGORITHMS[r.algo] != "glynn_esym"
    g = pg.glynn(dev(a)).value()
    assert abs(r.value() - g) <= 1e-11 * abs(pg.glynn(dev(np.abs(a))).value())
    # exact integer output, through the integer kind of the e_m form (at
    # 10 x 30 it runs several times faster than rectangular Ryser; at 6 x 20
    # all paths take the launch time and the choice is open)
    b = (np.random.default_rng(5).random((10, 30)) < 0.5).astype(np.uint8)
    r = pg.auto(dev(b))
    assert pg.ALGORITHMS[r.algo] == "glynn_esym"
    assert r.value() == oracle.per_laplace(b.astype(np.int64))


def test_workspace_release_then_rectangular_ryser_again():
    """Releasing the cached tables and the pool leaves every path working."""
    import paper_2510_03421_amd as pg
    b = (np.random.default_rng(8).random((6, 20)) < 0.5).astype(np.uint8)
    want = oracle.per_laplace(b.astype(np.int64))
    assert pg.ryser(dev(b)).value() == want
    pg.workspace_release()
    assert pg.ryser(dev(b)).value() == want
    assert run(b) == want


@pytest.mark.parametrize("n", [20, 27, 36, 43, 47])
def test_integer_kind_in_every_instantiation_range(n):
    """Exact int128 results at column counts in each range of the integer
    kernels (1..24, 25..32, 33..40, 41..44, 45..48) against the oracle."""
    rng = np.random.default_rng(9400 + n)
    a = rng.integers(-2, 3, size=(6, n)).astype(np.int64)
    assert run(a) == oracle.per_laplace(a)
    b = (rng.random((6, n)) < 0.5).astype(np.uint8)
    assert run(b) == oracle.per_laplace(b.astype(np.int64))


def esym_abs_sum_vec(a):
    """esym_abs_sum for larger m, vectorised over the sign vectors."""
    m, n = a.shape
    tot = 0.0
    step = 1 << 14
    for s0 in range(0, 1 << (m - 1), step):
        idx = np.arange(s0, min(1 << (m - 1), s0 + step))
        d = np.ones((len(idx), m))
        d[:, 1:] = 1 - 2 * ((idx[:, None] >> np.arange(m - 1)) & 1)
        c = np.abs(d @ a)
        e = np.zeros((len(idx), m + 1))
        e[:, 0] = 1.0
        for j in range(n):
            e[:, 1:] = e[:, 1:] + c[:, j:j + 1] * e[:, :-1]
        tot += e[:, m].sum()
    return tot / 2 ** (m - 1)


# exact-degree (banded) kernels run from m = 14 on
BAND_ORACLE = [(14, 14), (14, 15), (14, 30), (15, 48), (16, 17), (16, 40), (17, 23), (18, 18),
               (18, 36), (19, 20), (20, 33)]


@pytest.mark.parametrize("m,n", BAND_ORACLE)
def test_banded_against_oracle(m, n):
    a = workloads.uniform(m, n, 9500 + 64 * m + n)
    ref = oracle.per_laplace(a)
    want = ref.hi + ref.lo
    got = run(a)
    bound = 8 * n * U * esym_abs_sum_vec(a) + 4 * U * abs(want)
    assert abs(got - want) <= bound, (got, want, bound)
    z = workloads.complex_gauss(m, n, 9700 + 64 * m + n)
    refz = oracle.per_laplace(z)
    wz = complex(refz.re.hi + refz.re.lo, refz.im.hi + refz.im.lo)
    gz = run(z)
    bz = 16 * n * U * esym_abs_sum_vec(np.abs(z)) + 4 * U * abs(wz)
    assert abs(gz - wz) <= bz, (gz, wz, bz)


def _generic(a, monkeypatch):
    monkeypatch.setenv("PERM_ESYM_GENERIC", "1")
    try:
        return run(a)
    finally:
        monkeypatch.delenv("PERM_ESYM_GENERIC")


# every banded degree m with a few vector lengths each (short walks: m <= 24)
BAND_SWEEP = [(m, n) for m in range(14, 25) for n in sorted({m, m + 1, min(48, m + 7), 48})]


@pytest.mark.parametrize("m,n", BAND_SWEEP)
def test_banded_matches_generic(m, n, monkeypatch):
    """The banded recurrence skips only degrees that cannot reach e_m, so the
    two kernels evaluate the same terms; the sums differ by the rounding of
    their (differently planned) accumulations only."""
    a = workloads.uniform(m, n, 9900 + 64 * m + n)
    got, ref = run(a), _generic(a, monkeypatch)
    assert abs(got - ref) <= 1e-10 * abs(ref), (got, ref)
    z = workloads.complex_gauss(m, n, 9950 + 64 * m + n)
    gz, rz = run(z), _generic(z, monkeypatch)
    assert abs(gz - rz) <= 1e-10 * abs(rz), (gz, rz)


@pytest.mark.parametrize("m,n", [(26, 27), (28, 48), (30, 31), (32, 32), (32, 48)])
def test_banded_large_degrees_match_generic(m, n, monkeypatch):
    a = workloads.uniform(m, n, 9800 + 64 * m + n)
    got, ref = run(a), _generic(a, monkeypatch)
    assert abs(got - ref) <= 1e-10 * abs(ref), (got, ref)
