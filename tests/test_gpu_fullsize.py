"""Parity at the full workload sizes, in the launch configuration the
benchmark times (the same library calls).

The reference values come from tests/golden/reference_values.json, written by
tests/golden/make_golden.py with the CPU oracle only (exact integer DP, or
double-double Glynn / memoised expansion).  Where one permanent is the whole
output, properties that hold at any size complete the check: bitwise run-to-run
determinism, bitwise scaling / sign / conjugation symmetry, the Laplace row
expansion through 31 x 31 minors, and closed forms at the same size.
"""
import math

import numpy as np
import pytest

import workloads
from tests import closed_forms as cf
from tests.gpu_util import dev, run_algo, golden, ref_value, abs_ref

pytestmark = pytest.mark.gpu
CRIT = 1e-11


def rec(name):
    g = golden()
    if name not in g:
        pytest.skip(f"no reference value for {name} (run tests/golden/make_golden.py {name})")
    return g[name]


def fp_check(got, r, rel_bound):
    ref, pabs = ref_value(r), abs_ref(r)
    err = abs(complex(got) - complex(ref))
    assert err <= CRIT * pabs, (got, ref, err, pabs)
    assert err <= rel_bound * abs(ref), (got, ref, err / abs(ref))
    return err / abs(ref)


def test_u32_glynn_and_ryser():
    """Glynn keeps ~13 digits here; Ryser's inclusion-exclusion sum over 2^32
    column sets is worse conditioned (measured relative error ~1e-8).  Both meet
    the 1e-11 per(|A|) criterion by many orders of magnitude."""
    r = rec("u32")
    a = dev(workloads.config_matrix("u32"))
    g1 = run_algo("glynn", a)
    g2 = run_algo("glynn", a)
    assert g1 == g2                                  # bitwise reproducible
    fp_check(g1, r, 1e-11)
    fp_check(run_algo("ryser", a), r, 1e-6)


def test_u32_exact_symmetries():
    a_h = workloads.config_matrix("u32")
    base = run_algo("glynn", dev(a_h))
    # scaling by 2 is exact everywhere: result(2A) = 2^32 result(A)
    assert run_algo("glynn", dev(2.0 * a_h)) == base * 2.0 ** 32
    # negation commutes with rounding: result(-A) = (-1)^32 result(A)
    assert run_algo("glynn", dev(-a_h)) == base
    # negating one row flips the sign of per(A) exactly, but changes the
    # rounding of the column sums, so only to within the error bound
    neg_row = a_h.copy()
    neg_row[5] *= -1
    assert abs(run_algo("glynn", dev(neg_row)) + base) <= 1e-11 * abs(base)


def test_u32_laplace_expansion():
    """per(A) = sum_j a_0j per(A without row 0 and column j), every minor a
    31 x 31 Glynn evaluation on the GPU."""
    r = rec("u32")
    a_h = workloads.config_matrix("u32")
    total = 0.0
    for j in range(32):
        minor = np.ascontiguousarray(np.delete(a_h[1:], j, axis=1))
        total += a_h[0, j] * run_algo("glynn", dev(minor))
    fp_check(total, r, 1e-9)


def test_c32_complex_glynn():
    r = rec("c32")
    z = workloads.config_matrix("c32")
    got = run_algo("glynn", dev(z))
    fp_check(got, r, 1e-9)
    assert run_algo("glynn", dev(z)) == got
    # conjugation commutes with every rounding in the path (bitwise); a
    # multiplication by i does mathematically (i^32 = 1) but swaps real and
    # imaginary parts inside the fused complex products, so only to tolerance
    assert run_algo("glynn", dev(np.conj(z))) == got.conjugate()
    assert abs(run_algo("glynn", dev(1j * z)) - got) <= 1e-11 * abs(got)


def test_b28_exact_int128():
    r = rec("b28")
    want = ref_value(r)
    b = dev(workloads.config_matrix("b28"))
    assert run_algo("ryser", b) == want
    assert run_algo("glynn", b) == want
    # the binary64 path on the same 0/1 matrix
    f = run_algo("glynn", b, out="f64")
    assert abs(f - want) <= 1e-12 * want


def test_b30_exact_int128():
    """30 x 30, density 0.15, no zero row or column: a nonzero permanent,
    bit-exact through both formulas."""
    r = rec("b30")
    want = ref_value(r)
    assert want > 0
    b = dev(workloads.config_matrix("b30"))
    assert run_algo("ryser", b) == want
    assert run_algo("glynn", b) == want
    assert run_algo("ryser", dev(np.ascontiguousarray(workloads.config_matrix("b30").T))) == want


def test_b30z_zero_row():
    """The same recipe with seed 3030 has an all-zero row: per = 0 exactly,
    and the overflow pre-check takes its shortcut."""
    a = workloads.config_matrix("b30z")
    assert (a.sum(axis=1) == 0).any()
    assert ref_value(rec("b30z")) == 0
    assert run_algo("ryser", dev(a)) == 0
    assert run_algo("glynn", dev(a)) == 0


def test_b16x48_exact_rectangular_ryser():
    r = rec("b16x48")
    b = workloads.config_matrix("b16x48")
    assert run_algo("ryser", dev(b)) == ref_value(r)
    assert run_algo("ryser", dev(np.ascontiguousarray(b.T))) == ref_value(r)


def test_u20x40_rectangular():
    r = rec("u20x40")
    a = dev(workloads.config_matrix("u20x40"))
    # by-size Ryser weights reach C(39, 19) ~ 7e10 with alternating signs:
    # measured relative error ~1e-7, far inside the per(|A|) criterion
    rel_ryser = fp_check(run_algo("ryser", a), r, 1e-5)
    # the padded Glynn form (Eq. glynn_rectangle) with rows of ones is
    # ill-conditioned for m << n: it meets the per(|A|) criterion but keeps few
    # correct digits ...
    import paper_2510_03421_amd as pg
    g = run_algo("glynn", a, flags=pg._capi.PERM_FLAG_PAD_ONES)
    assert abs(g - ref_value(r)) <= CRIT * abs_ref(r)
    # ... padding rows of 2^e scaled to the data (the default) keep them
    g2 = run_algo("glynn", a)
    rel_glynn = fp_check(g2, r, 1e-9)
    assert rel_glynn < 1e-9 and rel_ryser < 1e-5


def test_u36_glynn_double_double():
    r = rec("u36")
    a = dev(workloads.config_matrix("u36"))
    import paper_2510_03421_amd as pg
    hi, lo = pg.glynn(a, out="dd").value()
    fp_check(hi + lo, r, 1e-10)


@pytest.mark.parametrize("n", [28, 32])
def test_closed_forms_at_full_size(n):
    # 0/1 graph counts through the exact integer paths at the benchmark sizes
    assert run_algo("ryser", dev(cf.derangement_matrix(n).astype(np.uint8))) == \
        cf.derangements(n)
    assert run_algo("ryser", dev(cf.tridiagonal_ones(n).astype(np.uint8))) == cf.fibonacci(n + 1)
    assert run_algo("glynn", dev(cf.hessenberg_ones(n).astype(np.uint8))) == 2 ** (n - 1)
    # binary64 Glynn and Ryser on the identity are exact
    assert run_algo("glynn", dev(np.eye(n))) == 1.0
    assert run_algo("ryser", dev(np.eye(n))) == 1.0


def test_limits():
    import torch

    import paper_2510_03421_amd as pg
    a = torch.zeros((49, 49), dtype=torch.float64, device="cuda")
    with pytest.raises(pg.PermError) as e:
        pg.glynn(a)
    assert e.value.status == -2
    b = torch.zeros((41, 41), dtype=torch.uint8, device="cuda")
    with pytest.raises(pg.PermError) as e:
        pg.ryser(b)
    assert e.value.status == -2


@pytest.mark.parametrize("n", [12, 16, 20])
def test_triangular_within_formula_bound(n):
    """per(T) = prod diag for a triangular T, and per(|T|) = |per(T)| is tiny
    next to the terms of either formula, so no binary64 evaluation of Glynn's
    or Ryser's sum can meet 1e-11 per(|A|) here; both are held to the bound the
    arithmetic gives, a few n u times the formula's absolute sum."""
    from tests.gpu_util import formula_abs_sums
    t = np.triu(workloads.uniform(n, n, 11)) + np.eye(n)
    exact = float(np.prod(np.diag(t)))
    ryser_abs, glynn_abs = formula_abs_sums(t)
    U = 2.0 ** -53
    assert abs(run_algo("glynn", dev(t)) - exact) <= 4 * n * U * glynn_abs + 4 * n * U * abs(exact)
    assert abs(run_algo("ryser", dev(t)) - exact) <= 4 * n * U * ryser_abs + 4 * n * U * abs(exact)


@pytest.mark.parametrize("n,p,seed", [(14, 0.15, 1), (18, 0.12, 2), (22, 0.2, 3), (24, 0.1, 4),
                                      (26, 0.15, 5), (20, 0.5, 6)])
def test_sparse_01_ryser_exact(n, p, seed):
    """Sparse 0/1 square matrices (the rows reordered by their counts of
    ones, whole waves of zero terms skipped) stay bit-exact."""
    import oracle
    a = workloads.bernoulli(n, n, p, 3300 + seed)
    want = oracle.per_laplace(a.astype(np.int64))
    assert run_algo("ryser", dev(a)) == want
    assert run_algo("ryser", dev(np.ascontiguousarray(a.T))) == want
    import paper_2510_03421_amd as pg
    assert pg.ryser(dev(a), flags=pg._capi.PERM_FLAG_WRAP).value() == want
