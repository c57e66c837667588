"""Square integer Ryser with the column window (perm_ryser on sparse input)
against the oracle, against the whole walk (PERM_RYSER_WINDOW=0), and on
the degenerate cases: a zero row (nothing left to walk), windows of one
column, signed entries (blocks whose window state has odd size are
subtracted)."""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def masks_of(a):
    return [int(sum(1 << j for j in np.flatnonzero(r))) for r in a]


def sparse(n, p, seed, signed=False):
    rng = np.random.default_rng(seed)
    a = (rng.random((n, n)) < p).astype(np.int64)
    if signed:
        a *= rng.choice([-3, -2, -1, 1, 2, 3], size=(n, n))
    # two very sparse rows, so that a window pays at every order here
    for i, k in ((0, 1), (1, 2)):
        a[i] = 0
        a[i, rng.choice(n, k, replace=False)] = 1 if not signed else -1
    return a


def with_mode(mode, fn):
    os.environ["PERM_RYSER_WINDOW"] = mode
    try:
        return fn()
    finally:
        del os.environ["PERM_RYSER_WINDOW"]


def whole_walk(fn):
    return with_mode("0", fn)


@pytest.mark.parametrize("n,p,signed", [(12, 0.3, False), (16, 0.2, True), (20, 0.25, False),
                                        (22, 0.25, True)])
def test_against_the_oracle(n, p, signed):
    import paper_2510_03421_amd as pg
    a = sparse(n, p, 7200 + n, signed)
    # at these orders the model keeps the whole walk: force the window
    assert pg.ryser_window_plan(masks_of(a), 1 << 18, force=True) is not None
    want = oracle.per_laplace(a)
    src = a if signed else a.astype(np.uint8)
    assert with_mode("2", lambda: pg.ryser(dev(src)).value()) == want
    assert whole_walk(lambda: pg.ryser(dev(src)).value()) == want
    assert pg.ryser(dev(src)).value() == want


@pytest.mark.parametrize("n,seed", [(28, 1), (30, 4), (32, 3)])
def test_window_equals_the_whole_walk(n, seed):
    import paper_2510_03421_amd as pg
    a = (np.random.default_rng(7300 + seed).random((n, n)) < 0.15).astype(np.uint8)
    assert pg.ryser_window_plan(masks_of(a), 1 << 18) is not None
    got = pg.ryser(dev(a)).value()
    assert got == whole_walk(lambda: pg.ryser(dev(a)).value())
    b = a.astype(np.int64) * np.random.default_rng(7400 + seed).choice([-1, 1], size=a.shape)
    assert pg.ryser(dev(b)).value() == whole_walk(lambda: pg.ryser(dev(b)).value())


def test_zero_row_and_auto():
    import paper_2510_03421_amd as pg
    a = (np.random.default_rng(7500).random((30, 30)) < 0.5).astype(np.uint8)
    a[17] = 0
    assert pg.ryser(dev(a)).value() == 0
    assert pg.ryser(dev(a.astype(np.int64)), out="i64").value() == 0
    b = workloads.config_matrix("b30")
    import json
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "reference_values.json")))["b30"]["value"]
    assert pg.auto(dev(b)).value() == int(gold)


def test_strided_input():
    """The window is chosen on the logical matrix: a strided view (lda 27)
    gives the same integer."""
    import paper_2510_03421_amd as pg
    import torch
    a = sparse(20, 0.2, 7600)
    want = oracle.per_laplace(a)
    big = torch.zeros(20, 27, dtype=torch.int64)
    big[:, :20] = torch.from_numpy(a)
    view = big.cuda()[:, :20]
    assert view.stride() == (27, 1)
    assert pg.ryser(view).value() == want


@pytest.mark.parametrize("n,p,seed", [(24, 0.15, 1), (28, 0.15, 2), (30, 0.15, 3)])
def test_floating_point_window(n, p, seed):
    """Floating-point square Ryser takes the window by itself from n = 30
    (complex 29) and at any n with PERM_FLAG_SPARSE: the skipped terms are
    exact zeros, so it agrees with the whole walk to rounding (and, at 24,
    with the oracle); real and complex."""
    import paper_2510_03421_amd as pg
    from paper_2510_03421_amd import _capi as C
    rng = np.random.default_rng(8100 + seed)
    pat = rng.random((n, n)) < p
    pat[np.arange(n), rng.permutation(n)] = True        # a perfect matching: per != 0
    a = np.where(pat, rng.uniform(-1, 1, size=(n, n)), 0.0)
    assert pg.ryser_window_plan(masks_of(a), 1 << 18) is not None
    fl = C.PERM_FLAG_SPARSE if n < 30 else 0
    got = pg.ryser(dev(a), out="dd", flags=fl).value()
    whole = whole_walk(lambda: pg.ryser(dev(a), out="dd", flags=fl).value())
    # per(|A|) <= prod_i sum_j |a_ij|: a certified scale for the criterion
    # where the oracle's per(|A|) is out of reach
    rows_bound = float(np.prod(np.abs(a).sum(axis=1)))
    if n <= 24:
        scale = float(oracle.per_laplace(np.abs(a)).hi)
        want = oracle.per_laplace(a)
        assert abs((got[0] + got[1]) - (want.hi + want.lo)) <= 1e-11 * scale
        assert abs((whole[0] + whole[1]) - (want.hi + want.lo)) <= 1e-11 * scale
    assert abs((got[0] + got[1]) - (whole[0] + whole[1])) <= 1e-11 * rows_bound
    assert got[0] != 0.0
    c = a * np.exp(1j * rng.uniform(0, 2 * np.pi, size=(n, n)))
    gc = pg.ryser(dev(c), flags=C.PERM_FLAG_SPARSE if n < 29 else 0).value()
    wc = whole_walk(lambda: pg.ryser(dev(c)).value())
    assert abs(gc - wc) <= 1e-11 * float(np.prod(np.abs(c).sum(axis=1)))
    assert gc != 0


def test_floating_point_window_forced_small():
    """The forced window at n = 14 on real input against the oracle."""
    import paper_2510_03421_amd as pg
    a = sparse(14, 0.25, 8200).astype(np.float64) * workloads.uniform(14, 14, 8201)
    want = oracle.per_laplace(a)
    scale = float(oracle.per_laplace(np.abs(a)).hi)
    got = with_mode("2", lambda: pg.ryser(dev(a), out="dd").value())
    assert abs((got[0] + got[1]) - (want.hi + want.lo)) <= 1e-11 * scale
