"""Host-side checks of algorithm selection (no GPU): the selector's features,
the size limits it respects, and that the threshold-table logic the fitting
tool uses makes exactly the library's choices."""
import ctypes
import math
import os
import tempfile

import numpy as np
import pytest

import paper_2510_03421_amd as pg
from paper_2510_03421_amd import _capi as C
from paper_2510_03421_amd import selector as S
from paper_2510_03421_amd import train_selector as TS
import torch


def lib_select(m, n, dt, density=-1.0):
    ch, src = ctypes.c_int(-1), ctypes.c_int(-1)
    rc = C.lib.perm_select(m, n, dt, density, ctypes.byref(ch), ctypes.byref(src))
    return rc, ch.value, src.value


def test_features():
    x = S.features(3, 5, torch.float64, 0.5)
    assert np.allclose(x, [math.log(3), math.log(5), 0.5, 0.0])
    assert np.array_equal(S.features(5, 3, torch.float64, 0.5), x)       # orientation
    assert S.features(4, 4, torch.complex128)[2:].tolist() == [1.0, 1.0]  # unknown density
    assert S.features(4, 4, torch.uint8, 0.3)[3] == 2.0
    assert S.features(4, 4, torch.int64, 0.3)[3] == 2.0


def test_size_limits_are_respected():
    pg.selector_load(None)
    try:
        # 0/1 input, 44 x 44: the integer Gray walk stops at 40, Ryser square too,
        # the definition has 44! maps: nothing can run it
        rc, _, _ = lib_select(44, 44, C.PERM_B8)
        assert rc == C.PERM_E_TOO_LARGE
        # 44 x 44 real: Glynn or Ryser (both <= 48)
        rc, ch, _ = lib_select(44, 44, C.PERM_F64)
        assert rc == 0 and ch in (C.PERM_ALGO_GLYNN, C.PERM_ALGO_RYSER)
        # 0/1 20 x 44: the table picks Ryser by size, and the e_m form (no
        # integer Glynn beyond 40 columns anyway) needs far fewer operations
        rc, ch, _ = lib_select(20, 44, C.PERM_B8)
        assert rc == 0 and ch == C.PERM_ALGO_GLYNN_ESYM
        # 30 x 49 real: only Ryser by size admits it (no Glynn or e_m beyond 48
        # columns, no sweep beyond 28 rows, too many maps for the definition)
        rc, ch, _ = lib_select(30, 49, C.PERM_F64)
        assert rc == 0 and ch == C.PERM_ALGO_RYSER
    finally:
        pg.selector_load(None)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_table_mirror_matches_the_library(seed):
    """train_selector.table_choice (used to fit p1..p8) against perm_select
    with the same table loaded, over every shape m <= n <= 48."""
    rng = np.random.default_rng(seed)
    p = np.zeros(9)
    p[1:] = [rng.uniform(-20, 20), rng.uniform(-2, 1), rng.uniform(-5, 30), rng.integers(0, 12),
             rng.uniform(-20, 20), rng.uniform(-1, 1), rng.uniform(-15, 15), rng.integers(2, 20)]
    d = tempfile.mkdtemp()
    path = os.path.join(d, "t.txt")
    with open(path, "w") as fh:
        fh.write("permgpu-selector 1\ntable " + " ".join(f"{v:.17g}" for v in p[1:]) + "\n")
    ms, ns = np.array([(m, n) for n in range(1, 49) for m in range(1, n + 1)]).T
    avail = np.ones((len(ms), 5), dtype=bool)
    for k, (m, n) in enumerate(zip(ms, ns)):
        avail[k, 0] = math.perm(int(n), int(m)) <= 2 ** 40
        avail[k, 1] = (m == n and n <= 48) or (m < n and m <= 40)   # square / by size
        avail[k, 2] = n <= 48
        avail[k, 3] = m <= n and m <= 32 and n <= 48                  # the e_m form
        avail[k, 4] = m <= 28                                         # the column sweep
    want = TS.table_choice(p, ms.astype(float), ns.astype(float), avail,
                           TS.log2_terms(ms, ns))
    pg.selector_load(path)
    try:
        got = np.array([TS.OUT_OF_ALGO[lib_select(int(m), int(n), C.PERM_F64)[1]]
                        for m, n in zip(ms, ns)])
    finally:
        pg.selector_load(pg.SELECTOR_WEIGHTS)
    assert np.array_equal(got, want), np.flatnonzero(got != want)[:10]


def test_weights_file_round_trip():
    rng = np.random.default_rng(4)
    params = rng.normal(size=S.NPARAMS).astype(np.float32)
    norm = np.array([1, 2, 0.5, 1, 0.5, 0.7, 0.3, 0.8], dtype=np.float32)
    d = tempfile.mkdtemp()
    path = os.path.join(d, "w.txt")
    S.save(path, params, norm, table=[0, -1, 5.5, 4, 1, 0, -0.62, 8])
    toks = open(path).read().split()
    assert toks[:2] == ["permgpu-selector", "2"]
    vals = np.array(toks[toks.index("mlp") + 1:], dtype=np.float32)
    assert np.array_equal(vals, params)                  # %.9g round-trips float32
    pg.selector_load(path)
    try:
        rc, ch, src = lib_select(20, 30, C.PERM_F64)
        assert rc == 0 and src == 1                      # the network decides
    finally:
        pg.selector_load(None)
    bad = os.path.join(d, "bad.txt")
    with open(bad, "w") as fh:
        fh.write("permgpu-selector 2\nmlp 1 2 3\n")
    with pytest.raises(pg.PermError):
        pg.selector_load(bad)


TIMINGS = os.path.join(os.path.dirname(pg.__file__), "data", "selector_timings_mi355x.csv")


def test_shipped_network_beats_the_table_on_held_out_timings():
    """On the 1000 held-out cases of the committed MI355X timings (5000 seeded
    cases, 80/20 split), the shipped network's choices (made by perm_select
    with its weights loaded) cost less time than the fitted table's, which
    cost less than always running Glynn.  Regret = t_chosen / t_best - 1
    against exhaustive timing of every algorithm."""
    d = TS.load_timings(TIMINGS)
    assert len(d["m"]) == 5000
    _, te = TS.split(len(d["m"]))
    ms = d["ms"][te]
    try:
        mlp = TS.regret(TS.library_choices(d, te, pg.SELECTOR_WEIGHTS), ms)
        table = TS.regret(TS.library_choices(d, te, None), ms)
    finally:
        pg.selector_load(pg.SELECTOR_WEIGHTS)
    avail = ~np.isnan(ms)
    glynn = TS.regret(np.where(avail[:, 2], 2, np.where(avail[:, 1], 1, 0)), ms)
    assert np.mean(mlp) < 0.05 and np.percentile(mlp, 95) < 0.2
    assert np.mean(mlp) < np.mean(table)
    assert np.mean(table) < np.mean(glynn)
    assert np.mean(mlp <= 1e-12) > 0.8          # the fastest algorithm in > 80% of cases
    # the network itself picks the e_m form where it is fastest
    choice = TS.library_choices(d, te, pg.SELECTOR_WEIGHTS)
    pg.selector_load(pg.SELECTOR_WEIGHTS)
    fastest = np.nanargmin(ms, axis=1)
    assert np.sum((choice == TS.ESYM) & (fastest == TS.ESYM)) > 0.5 * np.sum(fastest == TS.ESYM)


def test_committed_timings_are_consistent():
    d = TS.load_timings(TIMINGS)
    assert np.all(d["m"] <= d["n"]) and d["m"].min() >= 2 and d["n"].max() <= 48
    avail = ~np.isnan(d["ms"])
    assert np.all(avail.any(axis=1))
    assert np.all(d["ms"][avail] > 0)
    # availability is exactly the library's size limits (perm_select never
    # picks an algorithm without a timing)
    pg.selector_load(None)
    try:
        for i in range(0, 5000, 37):
            m, n = int(d["m"][i]), int(d["n"][i])
            dt = {"f64": C.PERM_F64, "c128": C.PERM_C128, "b8": C.PERM_B8}[d["dtype"][i]]
            rc, ch, _ = lib_select(m, n, dt, float(d["density"][i]))
            assert rc == 0 and avail[i, TS.OUT_OF_ALGO[ch]]
    finally:
        pg.selector_load(pg.SELECTOR_WEIGHTS)
