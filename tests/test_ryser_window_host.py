"""The square-Ryser column window (host planner, no device call).

A row whose nonzeros lie in a column set U has an empty sum over every
column subset that misses them, so its Ryser term (Sec. 1.2 Eq. ryser_square)
is zero.  perm_ryser_window_plan picks U and lists the states of U that the
walk still visits; these tests check the plan's contract on the CPU and,
on small matrices, that summing Eq. ryser_square over only the listed states
(with the walk's block structure and signs) gives the oracle's permanent."""
import numpy as np
import pytest

import oracle
import workloads

pg = pytest.importorskip("paper_2510_03421_amd")


def masks_of(a):
    return [int(sum(1 << j for j in np.flatnonzero(r))) for r in a]


def check_contract(a, plan):
    n = a.shape[0]
    fw, col = plan["fw"], [int(c) for c in plan["col_order"]]
    assert sorted(col) == list(range(n))
    win = col[n - fw:]
    assert win == sorted(win) and col[:n - fw] == sorted(col[:n - fw])
    assert plan["b"] >= 3 and plan["wlow"] >= 7 and plan["b"] + plan["wlow"] + fw == n
    states = [int(s) for s in plan["states"]]
    assert len(set(states)) == len(states) and all(0 <= s < (1 << fw) for s in states)
    inside = [r for r in masks_of(a) if all(((r >> j) & 1) == 0 or j in win for j in range(n))]
    listed = set(states)
    for v in range(1 << fw):
        cols = sum(1 << win[p] for p in range(fw) if (v >> p) & 1)
        if v not in listed:
            # every state left out empties some row inside the window
            assert any((cols & r) == 0 for r in inside), v


def window_sum(a, plan):
    """Eq. ryser_square summed over the plan's states only: every subset of
    the Gray bits under the window with each listed state on top, each term
    signed by the parity of its subset size."""
    n = a.shape[0]
    fw, b, wlow = plan["fw"], plan["b"], plan["wlow"]
    col = [int(c) for c in plan["col_order"]]
    A = a.astype(np.int64)[:, col]                    # Gray bit q -> column col[q]
    low = n - fw
    k = np.arange(1 << low, dtype=np.int64)
    g = k ^ (k >> 1)                                  # every subset of the low bits
    bits = ((g[:, None] >> np.arange(low)) & 1).astype(np.int64)
    base = bits @ A[:, :low].T                        # row sums over the low columns
    par = np.array([bin(int(x)).count("1") & 1 for x in g])
    total = 0
    for ws in plan["states"]:
        ws = int(ws)
        wcols = [low + p for p in range(fw) if (ws >> p) & 1]
        rs = base + A[:, wcols].sum(1)[None, :]
        prods = [int(np.prod([int(x) for x in r])) for r in rs]
        sgn = [(-1) ** (int(p) + len(wcols)) for p in par]
        total += sum(s * p for s, p in zip(sgn, prods))
    return (-1) ** n * total


def test_b30_pattern_gets_a_window():
    a = workloads.config_matrix("b30")
    plan = pg.ryser_window_plan(masks_of(a), 1 << 18)
    assert plan is not None
    check_contract(a, plan)
    # the sparsest rows of the 30 x 30, p = 0.15 workload leave well under
    # a fifth of the window's states
    assert len(plan["states"]) < 0.2 * (1 << plan["fw"])


def test_dense_pattern_keeps_the_whole_walk():
    assert pg.ryser_window_plan(masks_of(workloads.config_matrix("b28")), 1 << 18) is None
    assert pg.ryser_window_plan(masks_of(np.ones((30, 30), dtype=np.uint8)), 1 << 18) is None


def test_zero_row_leaves_nothing_to_walk():
    a = (np.random.default_rng(3).random((24, 24)) < 0.5).astype(np.uint8)
    a[5] = 0
    plan = pg.ryser_window_plan(masks_of(a), 1 << 18)
    assert plan is not None and len(plan["states"]) == 0
    check_contract(a, plan)


@pytest.mark.parametrize("seed", range(4))
def test_window_sum_equals_the_oracle(seed):
    """n = 14 with 256 lanes: windows of up to 4 columns; signed integers."""
    rng = np.random.default_rng(7100 + seed)
    n = 14
    a = (rng.random((n, n)) < 0.3) * rng.integers(-3, 4, size=(n, n))
    a[0] = 0
    a[0, rng.choice(n, 2, replace=False)] = rng.integers(1, 4, size=2)
    a[1] = 0
    a[1, rng.choice(n, 1)] = -2
    plan = pg.ryser_window_plan(masks_of(a), 256)
    assert plan is not None
    check_contract(a, plan)
    assert window_sum(a, plan) == oracle.per_laplace(a.astype(np.int64))


def test_small_or_invalid_inputs():
    assert pg.ryser_window_plan(masks_of(np.ones((9, 9))), 1 << 18) is None  # n < 10
    assert pg.ryser_window_plan([], 1 << 18) is None
    with pytest.raises(pg.PermError):
        pg.ryser_window_plan([1] * 65, 1 << 18)
