"""The selector network's GPU kernels against the float64 CPU reference
(forward, gradient, Adam), the captured training epoch against the same
steps run one by one, the timing entry point, and perm_auto's fallback."""
import math
import os
import tempfile

import numpy as np
import pytest

from oracle import mlp_ref as R

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def problem(seed, batch, nan_frac=0.2):
    rng = np.random.default_rng(seed)
    p = np.concatenate([rng.uniform(-1, 1, size=k) * math.sqrt(6.0 / f)
                        for k, f in ((256, 4), (64, 1e9), (4096, 64), (64, 1e9), (320, 64),
                                     (5, 1e9))]).astype(np.float32)
    p[256:320] = rng.uniform(-0.2, 0.2, 64)
    p[4416:4480] = rng.uniform(-0.2, 0.2, 64)
    x = np.stack([np.log(rng.integers(2, 31, batch)), np.log(rng.integers(2, 49, batch)),
                  rng.integers(1, 11, batch) / 10.0, rng.integers(0, 3, batch)],
                 axis=1).astype(np.float32)
    norm = np.array([2.6, 3.1, 0.55, 1.0, 0.65, 0.55, 0.29, 0.82], dtype=np.float32)
    t = rng.normal(0, 3, size=(batch, 5)).astype(np.float32)
    t[rng.random(size=t.shape) < nan_frac] = np.nan
    return p, norm, x, t


def cu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def abs_forward(p, norm, x):
    """Magnitude bound of every activation: the forward pass on |W|, |b|, |z|."""
    w = R.unpack(np.abs(p.astype(np.float64)))
    # |x - mean| can cancel: the rounding of z is relative to |x| + |mean|
    z = (np.abs(x.astype(np.float64)) + np.abs(norm[:4])) / norm[4:]
    h1 = z @ w["W1"].T + w["b1"]
    h2 = h1 @ w["W2"].T + w["b2"]
    return h2 @ w["W3"].T + w["b3"], h1, h2, z


@pytest.mark.parametrize("batch", [1, 300, 4000])
def test_forward_matches_reference(batch):
    from paper_2510_03421_amd import selector as S
    p, norm, x, _ = problem(batch, batch)
    y = S.mlp_forward(cu(p), cu(norm), cu(x)).cpu().numpy().astype(np.float64)
    ref, _ = R.forward(p, norm, x)
    yabs = abs_forward(p, norm, x)[0]
    # three layers of dot products of length <= 64 in FP32 (plus the input scaling)
    tol = 3 * 70 * U32 * yabs
    assert np.all(np.abs(y - ref) <= tol), np.max(np.abs(y - ref) / tol)


@pytest.mark.parametrize("batch,seed", [(1, 1), (37, 2), (300, 3), (4000, 4)])
def test_gradient_matches_reference(batch, seed):
    from paper_2510_03421_amd import selector as S
    p, norm, x, t = problem(seed, batch)
    # a ReLU whose input is within rounding of 0 may switch either way in FP32;
    # such a sample gets no targets, so it adds nothing to either gradient
    _, (_, a1, _, a2, _) = R.forward(p, norm, x)
    _, h1abs, h2abs, _ = abs_forward(p, norm, x)
    amb = np.any(np.abs(a1) <= 1e-5 * h1abs, axis=1) | np.any(np.abs(a2) <= 2e-5 * h2abs, axis=1)
    t[amb] = np.nan
    finite = int(np.count_nonzero(~np.isnan(t)))
    scale = 1.0 / max(finite, 1)
    g, loss = S.mlp_grad(cu(p), cu(norm), cu(x), cu(t), scale)
    g = g.cpu().numpy().astype(np.float64)
    loss = float(loss.cpu().numpy()[0])
    g_ref = R.grad(p, norm, x, t, scale)
    l_ref = R.loss(p, norm, x, t, scale)
    # magnitude of each gradient entry's terms: the backward pass on absolute
    # values (same ReLU masks), times the FP32 error of sums over the batch
    # and over 64 units, with the forward error carried along
    _, (z, a1, h1, a2, h2) = R.forward(p, norm, x)
    w = R.unpack(np.abs(p.astype(np.float64)))
    yabs = abs_forward(p, norm, x)[0]
    ok = ~np.isnan(t)
    y_ref, _ = R.forward(p, norm, x)
    dyabs = np.where(ok, 2 * scale * (np.abs(y_ref - np.where(ok, t, 0)) + 3 * 70 * U32 * yabs),
                     0)
    # an activation whose pre-activation cancels to a small value keeps the
    # forward error of its terms, not of its own size: carry that error into
    # the weight gradients that multiply it
    ga = {"W3": dyabs.T @ (np.abs(h2) + 140 * U32 * h2abs), "b3": dyabs.sum(0)}
    d2 = (dyabs @ w["W3"]) * (a2 > 0)
    ga["W2"], ga["b2"] = d2.T @ (np.abs(h1) + 70 * U32 * h1abs), d2.sum(0)
    d1 = (d2 @ w["W2"]) * (a1 > 0)
    ga["W1"], ga["b1"] = d1.T @ np.abs(z), d1.sum(0)
    gabs = R.pack(ga)
    tol = 4 * (batch + 200) * U32 * gabs + 1e-30
    bad = np.abs(g - g_ref) > tol
    assert not np.any(bad), (np.flatnonzero(bad)[:10], np.max(np.abs(g - g_ref) / tol))
    assert abs(loss - l_ref) <= 1e-4 * l_ref + 1e-30


def test_adam_matches_reference():
    import torch
    from paper_2510_03421_amd import selector as S
    rng = np.random.default_rng(9)
    p = rng.normal(size=R.NPARAMS).astype(np.float32)
    P, state = cu(p.copy()), torch.zeros(3 * R.NPARAMS, dtype=torch.float32, device="cuda")
    pr, m, v = p.astype(np.float64), np.zeros(R.NPARAMS), np.zeros(R.NPARAMS)
    for step in range(1, 6):
        g = (rng.normal(size=R.NPARAMS) * 10.0 ** rng.integers(-3, 3)).astype(np.float32)
        S.mlp_adam(P, cu(g), state, lr=1e-2, total_steps=8)
        pr, m, v = R.adam(pr, g, m, v, step, 1e-2, total_steps=8)
        got = P.cpu().numpy().astype(np.float64)
        assert np.allclose(got, pr, rtol=2e-6, atol=2e-6), np.max(np.abs(got - pr))
    steps = state[2 * R.NPARAMS:].cpu().view(torch.int32).numpy()
    assert np.all(steps == 5)


def test_training_graph_replays_match_eager_steps():
    """perm_selector_train replays one captured epoch; the same epochs run one
    by one through perm_mlp_grad / perm_mlp_adam give bitwise the same losses
    and parameters."""
    import torch
    from paper_2510_03421_amd import selector as S
    p0, _, x, t = problem(11, 500)
    epochs, lr = 7, 5e-3
    p_graph, norm, hist = S.train(x, t, epochs=epochs, lr=lr, params=p0)
    # again, with unrelated device work and synchronisation in between
    junk = torch.randn(1 << 20, device="cuda")
    junk.mul_(2.0).sum().item()
    torch.cuda.synchronize()
    p_graph2, norm2, hist2 = S.train(x, t, epochs=epochs, lr=lr, params=p0)
    assert np.array_equal(p_graph, p_graph2) and np.array_equal(hist, hist2)
    assert np.array_equal(norm, norm2)

    finite = int(np.count_nonzero(~np.isnan(t)))
    scale = float(np.float32(1.0) / np.float32(finite))
    P, N, X, T = cu(p0.copy()), cu(norm), cu(x), cu(t)
    state = torch.zeros(3 * R.NPARAMS, dtype=torch.float32, device="cuda")
    for e in range(epochs):
        g, loss = S.mlp_grad(P, N, X, T, scale)
        torch.cuda.synchronize()
        assert loss.cpu().numpy()[0] == hist[e], e
        S.mlp_adam(P, g, state, lr=lr, total_steps=epochs)
    assert np.array_equal(P.cpu().numpy(), p_graph)
    # and the loss history follows the CPU reference's trajectory (FP32)
    pr, m, v = p0.astype(np.float64), np.zeros(R.NPARAMS), np.zeros(R.NPARAMS)
    for e in range(epochs):
        assert abs(R.loss(pr, norm, x, t, scale) - hist[e]) <= 1e-3 * hist[e]
        pr, m, v = R.adam(pr, R.grad(pr, norm, x, t, scale), m, v, e + 1, lr,
                          total_steps=epochs)


def test_training_lowers_the_loss():
    from paper_2510_03421_amd import selector as S
    rng = np.random.default_rng(12)
    # a smooth target: log time of five made-up cost laws over the features
    m = rng.integers(2, 31, 2000)
    n = m + rng.integers(0, 19, 2000)
    x = np.stack([np.log(m), np.log(n), rng.integers(1, 11, 2000) / 10, rng.integers(0, 3, 2000)],
                 axis=1).astype(np.float32)
    t = np.stack([m * np.log(n) * 0.7 - 4, n * 0.69 - 12 + 0.2 * x[:, 3], (n - 1) * 0.69 - 12,
                  (m - 1) * 0.69 + np.log(n * m) - 14, m * 0.69 + np.log(n) - 13],
                 axis=1).astype(np.float32)
    _, _, hist = S.train(x, t, epochs=1500, lr=3e-3, seed=1)
    assert hist[-1] < 0.02 * hist[0], (hist[0], hist[-1])


def test_perm_time_cuts_work_and_restores_it():
    import paper_2510_03421_amd as pg
    from paper_2510_03421_amd import selector as S
    import workloads
    rng = np.random.default_rng(13)
    a = cu(rng.uniform(-1, 1, size=(34, 34)))
    before = pg.glynn(a, out="dd").value()
    t_small, f_small = S.time("glynn", a, fraction=1e-9, reps=1)
    t_full, f_full = S.time("glynn", a, fraction=1.0, reps=1)
    assert 0 < f_small < 1 and f_full == 1.0
    assert t_full > t_small
    after = pg.glynn(a, out="dd").value()
    assert after == before                       # truncation does not leak
    r = cu(rng.uniform(-1, 1, size=(16, 40)))
    _, fr = S.time("ryser", r, fraction=0.01, reps=1)
    assert 0 < fr < 0.2
    # the definition runs whole rounds of prefixes (a few per lane): the
    # fraction that ran is within a round of the one asked for
    c = cu(rng.uniform(-1, 1, size=(8, 12)))
    _, fc = S.time("combinatoric", c, fraction=0.5, reps=1)
    assert 0.3 <= fc <= 0.7, fc
    _, fc1 = S.time("combinatoric", c, fraction=1.0, reps=1)
    assert fc1 == 1.0
    for bad in (0.0, 1.5, -1.0):
        with pytest.raises(pg.PermError):
            S.time("glynn", a, fraction=bad)
    with pytest.raises(pg.PermError):
        S.time("combinatoric", a)                 # 34! maps: refused by size
    # the e_m form cuts its Gray blocks (when each lane walks several: 2^31
    # sign vectors here, at least two blocks per lane still run); the column
    # sweep always runs whole (its cost is bounded)
    _, fe = S.time("glynn_esym", cu(rng.uniform(-1, 1, size=(32, 48))), fraction=0.01, reps=1)
    assert 0 < fe <= 0.5
    e = cu(rng.uniform(-1, 1, size=(24, 40)))
    _, fs = S.time("column_sweep", e, fraction=0.3, reps=1)
    assert fs == 1.0


def test_auto_moves_on_when_glynn_refuses_an_integer_bound():
    """A 30 x 30 matrix of ones: per = 30! fits int128, Glynn's sum 2^29 30!
    does not, so a table that puts Glynn first must fall back."""
    import paper_2510_03421_amd as pg
    a = cu(np.ones((30, 30), dtype=np.uint8))
    d = tempfile.mkdtemp()
    path = os.path.join(d, "glynn_first.txt")
    with open(path, "w") as fh:
        # n > p8 = 0 always; p5 r + p6 n + p7 = 1 > 0: Glynn first
        fh.write("permgpu-selector 1\ntable 0 0 0 0 0 0 1 0\n")
    try:
        pg.selector_load(path)
        assert pg.select(30, 30, dtype=__import__("torch").uint8) == ("glynn", False)
        r = pg.auto(a)
        assert r.value() == math.factorial(30)
        assert pg.ALGORITHMS[r.algo] != "glynn"
    finally:
        pg.selector_load(pg.SELECTOR_WEIGHTS)


def test_training_on_stored_timings_beats_the_table():
    """The network trained here, on the GPU, from the committed MI355X timings
    (training split only) chooses better on the held-out split than the
    threshold table does."""
    import paper_2510_03421_amd as pg
    from paper_2510_03421_amd import selector as S, train_selector as TS
    d = TS.load_timings(os.path.join(os.path.dirname(pg.__file__), "data",
                                     "selector_timings_mi355x.csv"))
    tr, te = TS.split(len(d["m"]))
    params, norm, hist = S.train(TS.features(d, tr), np.log(d["ms"][tr]).astype(np.float32),
                                 epochs=3000, lr=3e-3, seed=1)
    # the measured times carry noise that no fit removes: the loss falls
    # by more than 10x, not to zero
    assert hist[-1] < 0.1 * hist[0]
    path = os.path.join(tempfile.mkdtemp(), "w.txt")
    S.save(path, params, norm)
    try:
        mlp = TS.regret(TS.library_choices(d, te, path), d["ms"][te])
        table = TS.regret(TS.library_choices(d, te, None), d["ms"][te])
    finally:
        pg.selector_load(pg.SELECTOR_WEIGHTS)
    assert np.mean(mlp) < np.mean(table), (np.mean(mlp), np.mean(table))


def test_host_choice_matches_the_gpu_forward_on_the_shipped_network():
    """perm_auto evaluates the shipped network on the host; on every stored
    selector case its choice equals the argmin, over the algorithms the case
    admits, of the GPU forward kernel's predictions (up to FP32 near-ties)."""
    import torch

    import paper_2510_03421_amd as pg
    from paper_2510_03421_amd import selector as S
    from paper_2510_03421_amd import train_selector as TS
    toks = open(pg.SELECTOR_WEIGHTS).read().split()
    norm = np.array(toks[toks.index("norm") + 1:toks.index("norm") + 9], dtype=np.float32)
    params = np.array(toks[toks.index("mlp") + 1:], dtype=np.float32)
    assert params.size == 4805
    d = TS.load_timings(os.path.join(os.path.dirname(pg.__file__), "data",
                                     "selector_timings_mi355x.csv"))
    tdt = {"f64": torch.float64, "c128": torch.complex128, "b8": torch.uint8}
    x = np.stack([S.features(int(m), int(n), tdt[dt], float(de))
                  for m, n, dt, de in zip(d["m"], d["n"], d["dtype"], d["density"])])
    y = S.mlp_forward(cu(params), cu(norm), cu(x.astype(np.float32))).cpu().numpy()
    y = y.astype(np.float64)
    avail = ~np.isnan(d["ms"])
    best = np.argmin(np.where(avail, y, np.inf), axis=1)
    pg.selector_load(pg.SELECTOR_WEIGHTS)
    order = list(S.ALGO_ORDER)
    near_ties = 0
    for i in range(len(best)):
        name, from_net = pg.select(int(d["m"][i]), int(d["n"][i]), tdt[d["dtype"][i]],
                                   float(d["density"][i]))
        assert from_net
        ch = order.index(name)
        if ch != best[i]:
            near_ties += 1
            assert abs(y[i, ch] - y[i, best[i]]) <= 1e-4 * (1.0 + abs(y[i, ch])), (i, y[i])
    assert near_ties <= 5
