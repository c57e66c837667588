"""The paired real walk (two Gray blocks per lane at a time, one scalar row
load for both; used for real walks of 16..40 entries that fill the device)
against the oracle and against the single walk (PERM_ENGINE_PAIR=0): square
Glynn and Ryser, rectangular Glynn.  (Chunks of the 32 x 32 sum, which take
the paired walk too, are covered by test_gpu_chunks.py.)"""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def single(fn):
    os.environ["PERM_ENGINE_PAIR"] = "0"
    try:
        return fn()
    finally:
        del os.environ["PERM_ENGINE_PAIR"]


def dd(v):
    return v[0] + v[1]


@pytest.mark.parametrize("n,seed", [(23, 1), (24, 2), (26, 3)])
def test_square_glynn_against_the_oracle(n, seed):
    import paper_2510_03421_amd as pg
    a = workloads.uniform(n, n, 9700 + seed)
    want = oracle.per_glynn(a)
    scale = float(oracle.per_glynn(np.abs(a)).hi)
    got = dd(pg.glynn(dev(a), out="dd").value())
    ref = dd(single(lambda: pg.glynn(dev(a), out="dd").value()))
    assert abs(got - (want.hi + want.lo)) <= 1e-11 * scale
    assert abs(got - ref) <= 1e-13 * scale


def test_square_ryser_and_rectangular_glynn():
    import paper_2510_03421_amd as pg
    a = workloads.uniform(24, 24, 9710)
    want = oracle.per_glynn(a)
    scale = float(oracle.per_glynn(np.abs(a)).hi)
    got = dd(pg.ryser(dev(a), out="dd").value())
    assert abs(got - (want.hi + want.lo)) <= 1e-11 * scale
    # 22 x 26: padded Glynn over 26 columns (the paired walk) against the
    # e_m form, which sums the padding rows out, and against the single walk
    r = workloads.uniform(22, 26, 9711)
    g = dd(pg.glynn(dev(r), out="dd").value())
    e = pg.glynn_esym(dev(r)).value()
    gs = dd(single(lambda: pg.glynn(dev(r), out="dd").value()))
    rs = float(abs(pg.glynn_esym(dev(np.abs(r))).value()))
    assert abs(g - e) <= 1e-11 * rs
    assert abs(g - gs) <= 1e-13 * rs


def test_integer_and_complex_are_unchanged():
    """The paired walk is real only: 0/1 and complex inputs of the same
    orders give the same values with and without it."""
    import paper_2510_03421_amd as pg
    b = (np.random.default_rng(9720).random((24, 24)) < 0.5).astype(np.uint8)
    assert pg.ryser(dev(b)).value() == single(lambda: pg.ryser(dev(b)).value())
    c = workloads.uniform(24, 24, 9721) + 1j * workloads.uniform(24, 24, 9722)
    assert pg.glynn(dev(c)).value() == single(lambda: pg.glynn(dev(c)).value())
