"""Property tests of the CPU oracle on random small matrices (Hypothesis):
the four evaluators agree exactly on integer matrices, and the permanent's
invariances hold -- row and column permutations, transposition (square),
row scaling, the Laplace expansion along a row, and per(-A) = (-1)^m per(A),
per(conj A) = conj per(A), per(iA) = i^m per(A) (Sec. 1.1 definitions)."""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle

settings.register_profile("oracle", max_examples=40, deadline=None, derandomize=True)
settings.load_profile("oracle")


@st.composite
def int_matrix(draw, max_n=6):
    n = draw(st.integers(1, max_n))
    m = draw(st.integers(1, n))
    vals = draw(st.lists(st.integers(-3, 3), min_size=m * n, max_size=m * n))
    return np.array(vals, dtype=np.int64).reshape(m, n)


def exact(x):
    """An oracle value as an exact Python int (integer input: int128 result;
    floating-point evaluators on small integers: double-double, exact here)."""
    if isinstance(x, int):
        return x
    return int(round(x.hi)) + int(round(x.lo))


@given(int_matrix())
def test_evaluators_agree_exactly(a):
    want = oracle.per_brute(a)
    assert oracle.per_laplace(a) == want
    f = a.astype(np.float64)
    for ev in (oracle.per_brute, oracle.per_laplace, oracle.per_glynn, oracle.per_ryser):
        assert exact(ev(f)) == want, ev.__name__


@given(int_matrix(), st.randoms(use_true_random=False))
def test_permutations_and_transpose(a, rnd):
    m, n = a.shape
    rows, cols = list(range(m)), list(range(n))
    rnd.shuffle(rows)
    rnd.shuffle(cols)
    want = oracle.per_brute(a)
    assert oracle.per_brute(np.ascontiguousarray(a[rows][:, cols])) == want
    assert oracle.per_brute(np.ascontiguousarray(a.T)) == want      # m > n reads A^T


@given(int_matrix(), st.integers(0, 5), st.integers(-4, 4))
def test_row_scaling_and_laplace(a, r, k):
    m, n = a.shape
    r %= m
    want = oracle.per_brute(a)
    b = a.copy()
    b[r] *= k
    assert oracle.per_brute(b) == k * want
    # expansion along row r: sum over columns j of a_rj per(A without row r, column j)
    if m > 1:
        total = 0
        for j in range(n):
            minor = np.delete(np.delete(a, r, axis=0), j, axis=1)
            total += int(a[r, j]) * oracle.per_brute(np.ascontiguousarray(minor))
        assert total == want
    else:
        assert int(a[0].sum()) == want


@given(int_matrix(max_n=5), int_matrix(max_n=5))
def test_complex_symmetries(re_, im_):
    m = min(re_.shape[0], im_.shape[0])
    n = min(re_.shape[1], im_.shape[1])
    if m > n:
        m = n
    z = re_[:m, :n].astype(np.float64) + 1j * im_[:m, :n].astype(np.float64)

    def val(x):
        v = oracle.per_brute(np.ascontiguousarray(x))
        return complex(exact(v.re), exact(v.im))

    p = val(z)
    assert val(-z) == (-1) ** m * p
    assert val(np.conj(z)) == p.conjugate()
    assert val(1j * z) == (1j) ** m * p
    assert complex(oracle.per_laplace(np.ascontiguousarray(z))) == p
