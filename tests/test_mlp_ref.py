"""Pins of the selector network's CPU reference (oracle/mlp_ref.py): the
backpropagated gradient against central finite differences of the loss,
forward passes with closed-form outputs, and the Adam step's closed-form
first step (Kingma & Ba 2015, Algorithm 1) and schedule end points."""
import numpy as np
import pytest

from oracle import mlp_ref as R


def random_problem(seed, batch=40, nan_frac=0.2):
    rng = np.random.default_rng(seed)
    p = np.concatenate([rng.uniform(-1.2, 1.2, size=k) * (1.0 if k > 5 else 0.3)
                        for k in (256, 64, 4096, 64, 320, 5)])
    x = np.stack([np.log(rng.integers(2, 31, batch)), np.log(rng.integers(2, 49, batch)),
                  rng.uniform(0.1, 1.0, batch), rng.integers(0, 3, batch)], axis=1)
    norm = np.concatenate([x.mean(axis=0), x.std(axis=0) + 0.1])
    t = rng.normal(0, 3, size=(batch, 5))
    t[rng.random(size=t.shape) < nan_frac] = np.nan
    return p, norm, x, t


def test_layout_size():
    assert R.NPARAMS == 4805
    p = np.arange(R.NPARAMS, dtype=float)
    assert np.array_equal(R.pack(R.unpack(p)), p)
    w = R.unpack(p)
    assert w["W1"][1, 0] == 4 and w["b1"][0] == 256 and w["W2"][0, 1] == 321
    assert w["W3"][4, 63] == 4799 and w["b3"][4] == 4804


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_matches_finite_differences(seed):
    p, norm, x, t = random_problem(seed)
    scale = 1.0 / np.count_nonzero(~np.isnan(t))
    g = R.grad(p, norm, x, t, scale)
    rng = np.random.default_rng(100 + seed)
    # every block: W1, b1, W2, b2, W3, b3
    idx = np.concatenate([rng.integers(lo, hi, 12) for lo, hi in
                          ((0, 256), (256, 320), (320, 4416), (4416, 4480), (4480, 4800),
                           (4800, 4805))])
    num = R.numeric_grad(p, norm, x, t, scale, idx)
    assert np.allclose(g[idx], num, rtol=1e-5, atol=1e-8 * np.max(np.abs(g)))


def test_masked_targets_do_not_contribute():
    p, norm, x, t = random_problem(4)
    t[:, 1] = np.nan
    g = R.unpack(R.grad(p, norm, x, t, 0.5))
    assert np.all(g["W3"][1] == 0) and g["b3"][1] == 0
    t2 = t.copy()
    t2[:, 1] = 1e9  # any value: the column is masked in t
    assert R.loss(p, norm, x, t, 0.5) == pytest.approx(
        R.loss(p, norm, x, np.where(np.isnan(t), np.nan, t), 0.5))
    t_all = np.full_like(t, np.nan)
    assert R.loss(p, norm, x, t_all, 1.0) == 0.0
    assert np.all(R.grad(p, norm, x, t_all, 1.0) == 0)


def test_forward_closed_forms():
    w = {k: np.zeros(s) for k, s in R.LAYOUT}
    norm = np.array([0, 0, 0, 0, 1, 1, 1, 1.0])
    x = np.array([[0.3, -2.0, 0.5, 1.0]])
    w["b1"][:] = 1.0            # h1 = 1
    w["b2"][:] = 2.0            # h2 = 2
    w["W3"][:] = 1.0
    w["b3"][:] = [0.5, -1.0, 3.0, 0.0, -2.5]
    y, _ = R.forward(R.pack(w), norm, x)
    assert np.allclose(y, [[128.5, 127.0, 131.0, 128.0, 125.5]])
    w["b2"][:] = -1.0           # ReLU cuts every unit
    y, _ = R.forward(R.pack(w), norm, x)
    assert np.allclose(y, [[0.5, -1.0, 3.0, 0.0, -2.5]])
    # normalisation and both ReLUs: y_k = max(z_1, 0) with z_1 = (x_1 - mu) / sd
    w = {k: np.zeros(s) for k, s in R.LAYOUT}
    w["W1"][0, 1] = 1.0
    w["W2"][0, 0] = 1.0
    w["W3"][:, 0] = 1.0
    norm = np.array([0, -1.0, 0, 0, 1, 4.0, 1, 1])
    for x1, want in ((3.0, 1.0), (-5.0, 0.0)):
        y, _ = R.forward(R.pack(w), norm, np.array([[0, x1, 0, 0.0]]))
        assert np.allclose(y, want)


def test_adam_first_step_and_schedule():
    rng = np.random.default_rng(5)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    z = np.zeros(50)
    # step 1: bias-corrected moments are g and g^2, so the move is lr * g / (|g| + eps)
    p1, m1, v1 = R.adam(p, g, z, z, 1, 0.01, eps=0.0)
    assert np.allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    # cosine decay: full rate at the start, zero at the end
    pe, _, _ = R.adam(p, g, z, z, 10, 0.01, total_steps=10)
    assert np.array_equal(pe, p)
    ph, _, _ = R.adam(p, g, z, z, 5, 0.01, total_steps=10)
    pc, _, _ = R.adam(p, g, z, z, 5, 0.005)
    assert np.allclose(ph, pc, rtol=0, atol=1e-15)
