"""Train the algorithm selector from measured timings and report its regret.

    python -m paper_2510_03421_amd.train_selector --timings timings.csv
           --out selector_weights.txt [--report report.json] [--epochs 8000]

Steps: an 80/20 seeded split of the timed cases; the network is trained on
the GPU (``perm_selector_train``: the library's own forward, gradient and
Adam kernels) on log run times in milliseconds; the threshold table of
Alg. 5's form is refitted on the same training cases; both go into the
weights file.  On the held-out cases every policy's choice comes from the
library itself (``perm_select`` with the weights loaded), and its regret is
t_chosen / t_best - 1, t_best being the fastest measured algorithm
(exhaustive timing).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile

import numpy as np
import torch

from . import _capi as C
from . import selector as S

DTYPES = {"f64": torch.float64, "c128": torch.complex128, "b8": torch.uint8}
COMB, RYSER, GLYNN, ESYM, SWEEP = 0, 1, 2, 3, 4   # network output indices (S.ALGO_ORDER)
OUT_OF_ALGO = {a: k for k, a in enumerate(S.ALGO_IDS)}


def load_timings(path: str) -> dict:
    """Columns of a timings CSV as numpy arrays; ms[:, a] is NaN where
    algorithm a refused the shape."""
    rows = [ln.rstrip("\n").split(",") for ln in open(path) if ln.strip()]
    head, rows = rows[0], rows[1:]
    col = {h: i for i, h in enumerate(head)}
    get = lambda r, h: r[col[h]]
    ms = np.array([[float(get(r, f"ms_{a}")) if f"ms_{a}" in col and get(r, f"ms_{a}") else np.nan
                    for a in S.ALGO_ORDER] for r in rows])
    return {
        "i": np.array([int(get(r, "i")) for r in rows]),
        "m": np.array([int(get(r, "m")) for r in rows]),
        "n": np.array([int(get(r, "n")) for r in rows]),
        "dtype": np.array([get(r, "dtype") for r in rows]),
        "density": np.array([float(get(r, "density")) for r in rows]),
        "ms": ms,
    }


def split(count: int, seed: int = 5001, train_frac: float = 0.8):
    perm = np.random.default_rng(seed).permutation(count)
    k = int(round(train_frac * count))
    return np.sort(perm[:k]), np.sort(perm[k:])


def features(d: dict, idx) -> np.ndarray:
    return np.stack([S.features(int(d["m"][i]), int(d["n"][i]), DTYPES[d["dtype"][i]],
                                float(d["density"][i])) for i in idx]).astype(np.float32)


def regret(choice: np.ndarray, ms: np.ndarray) -> np.ndarray:
    best = np.nanmin(ms, axis=1)
    t = ms[np.arange(len(choice)), choice]
    return t / best - 1.0


def summary(r: np.ndarray) -> dict:
    return {"mean": float(np.mean(r)), "median": float(np.median(r)),
            "p95": float(np.percentile(r, 95)), "max": float(np.max(r)),
            "optimal_frac": float(np.mean(r <= 1e-12))}


def library_choices(d: dict, idx, weights: str | None) -> np.ndarray:
    """perm_select's choice for each case with `weights` loaded (None: the
    built-in table)."""
    C.check(C.lib.perm_selector_load(weights.encode() if weights else None), "load")
    import ctypes
    out = np.empty(len(idx), dtype=np.int64)
    ch, src = ctypes.c_int(-1), ctypes.c_int(-1)
    for k, i in enumerate(idx):
        C.check(C.lib.perm_select(int(d["m"][i]), int(d["n"][i]),
                                  {"f64": C.PERM_F64, "c128": C.PERM_C128,
                                   "b8": C.PERM_B8}[d["dtype"][i]],
                                  float(d["density"][i]), ctypes.byref(ch), ctypes.byref(src)),
                "perm_select")
        out[k] = OUT_OF_ALGO[ch.value]
    return out


# ---- the threshold table (Alg. 5's form), for fitting ----
def log2_terms(m: np.ndarray, n: np.ndarray) -> np.ndarray:
    """log2 of the term counts per case of the five algorithms (combinatoric,
    Ryser, Glynn, the e_m form, the column sweep's state updates), as the
    library ranks them (log2_algo_terms)."""
    lc = np.array([sum(math.log2(nn - i) for i in range(mm)) for mm, nn in zip(m, n)])
    lr = np.array([float(nn) if mm == nn else
                   math.log2(sum(math.comb(int(nn), k) for k in range(int(mm) + 1)))
                   for mm, nn in zip(m, n)])
    le = m - 1.0
    ls = []
    for mm, nn in zip(m, n):
        mm, nn = int(mm), int(nn)
        tot = sum(math.comb(mm, k) * max(0, min(nn - mm + 1, k + 1, nn - (mm - k)))
                  for k in range(mm + 1))
        ls.append(math.log2(max(tot, 1)))
    return np.stack([lc, lr, n - 1.0, le, np.array(ls)], axis=1)


def log2_ops(m: np.ndarray, n: np.ndarray, terms: np.ndarray) -> np.ndarray:
    """log2 of the rough operation counts the library's table rule compares
    (terms times the work of one term)."""
    mm, nn = m.astype(float), n.astype(float)
    per = np.stack([np.maximum(mm, 1), 2 * mm, 2 * nn, nn * (np.minimum(mm, 32) + 1),
                    np.maximum(mm, 1)], axis=1)
    return terms + np.log2(per)


def table_choice(p: np.ndarray, m: np.ndarray, n: np.ndarray, avail: np.ndarray,
                 terms: np.ndarray) -> np.ndarray:
    """The library's table policy: Alg. 5's decision with values p[1..8]
    among the paper's three algorithms, the e_m form instead when its
    operation count is below half of that choice's, the rest by term count
    with the column sweep last; the first available algorithm."""
    r = m / n
    small = n <= p[8]
    comb_small = ((m == n) & (n <= p[4])) | (p[1] * r + p[2] * n + p[3] > 0)
    glynn_large = p[5] * r + p[6] * n + p[7] > 0
    pick = np.where(small, np.where(comb_small, COMB, GLYNN),
                    np.where(glynn_large, GLYNN, RYSER))
    rows = np.arange(len(pick))
    ops = log2_ops(m, n, terms)
    esym = avail[:, ESYM] & (ops[:, ESYM] + 1.0 < ops[rows, pick])
    pick = np.where(esym, ESYM, pick)
    key = terms.copy()
    key[rows, pick] = -1e300
    key[:, SWEEP] = 1e300
    key = np.where(avail, key, np.inf)
    return np.argmin(key, axis=1)


def fit_table(d: dict, idx, seed: int = 7, rounds: int = 6) -> np.ndarray:
    """Coordinate search over p1..p8 minimising mean training regret."""
    m, n, ms = d["m"][idx].astype(float), d["n"][idx].astype(float), d["ms"][idx]
    avail = ~np.isnan(ms)
    terms = log2_terms(d["m"][idx], d["n"][idx])
    grids = {1: np.linspace(-40, 40, 81), 2: np.linspace(-3, 1, 41), 3: np.linspace(-20, 40, 121),
             4: np.arange(0, 17), 5: np.linspace(-40, 40, 81), 6: np.linspace(-2, 2, 81),
             7: np.linspace(-30, 30, 121), 8: np.arange(2, 25)}
    p = np.array([0.0, 0.0, -1.0, 5.5, 4.0, 1.0, 0.0, -0.62, 8.0])
    cost = lambda q: float(np.mean(regret(table_choice(q, m, n, avail, terms), ms)))
    best = cost(p)
    rng = np.random.default_rng(seed)
    for _ in range(rounds):
        for j in rng.permutation(np.arange(1, 9)):
            for v in grids[int(j)]:
                q = p.copy()
                q[j] = v
                c = cost(q)
                if c < best - 1e-12:
                    best, p = c, q
    return p


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--timings", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--report", default=None)
    ap.add_argument("--epochs", type=int, default=8000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seeds", type=int, default=4)
    args = ap.parse_args(argv)

    d = load_timings(args.timings)
    tr, te = split(len(d["m"]))
    x_tr = features(d, tr)
    t_tr = np.log(d["ms"][tr]).astype(np.float32)  # NaN stays NaN
    ms_tr, ms_te = d["ms"][tr], d["ms"][te]

    table = fit_table(d, tr)
    tmp = tempfile.mkdtemp()
    best = None
    for sd in range(1, args.seeds + 1):
        params, norm, hist = S.train(x_tr, t_tr, epochs=args.epochs, lr=args.lr, seed=sd)
        path = os.path.join(tmp, f"w{sd}.txt")
        S.save(path, params, norm, table[1:])
        r = float(np.mean(regret(library_choices(d, tr, path), ms_tr)))
        print(f"train_selector: seed {sd} final loss {hist[-1]:.4g} train regret {r:.4g}",
              flush=True)
        if best is None or r < best[0]:
            best = (r, params, norm, hist, sd)
    _, params, norm, hist, sd = best
    S.save(args.out, params, norm, table[1:])

    table_only = os.path.join(tmp, "table.txt")
    with open(table_only, "w") as fh:
        fh.write("permgpu-selector 2\ntable " + " ".join(f"{v:.9g}" for v in table[1:]) + "\n")
    pol = {
        "mlp": library_choices(d, te, args.out),
        "table_fitted": library_choices(d, te, table_only),
        "table_builtin": library_choices(d, te, None),
    }
    avail = ~np.isnan(ms_te)
    glynn_first = np.where(avail[:, GLYNN], GLYNN, np.where(avail[:, RYSER], RYSER, COMB))
    pol["always_glynn"] = glynn_first
    # the paper's three algorithms only (no e_m form, no sweep): best of them
    three = np.where(avail[:, :3], ms_te[:, :3], np.inf)
    pol["best_of_three"] = np.argmin(three, axis=1)
    rep = {"cases": int(len(d["m"])), "train": int(len(tr)), "held_out": int(len(te)),
           "epochs": args.epochs, "lr": args.lr, "seed": sd,
           "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
           "table": [float(v) for v in table[1:]],
           "regret": {k: summary(regret(v, ms_te)) for k, v in pol.items()}}
    C.check(C.lib.perm_selector_load(None), "unload")
    print(json.dumps(rep, indent=1), flush=True)
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(rep, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
