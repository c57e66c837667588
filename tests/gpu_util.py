"""Helpers of the GPU tests: move seeded inputs to the device and call the
library through its Python binding (which calls the C ABI)."""
import json
import os

import numpy as np

ALGOS = ("glynn", "ryser", "combinatoric")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "reference_values.json")


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_algo(algo, t, out=None, flags=0):
    """Run one algorithm and return the value on the host (int, float, complex)."""
    import paper_2510_03421_amd as pg
    fn = {"glynn": pg.glynn, "ryser": pg.ryser, "combinatoric": pg.combinatoric,
          "auto": pg.auto}[algo]
    if algo == "combinatoric" and t.dim() == 2:
        m, n = sorted(t.shape)
        total = 1
        for i in range(m):
            total *= (n - i)
        if total > 2 ** 31:
            raise ValueError("too many maps for a test")
    return fn(t, out=out, flags=flags).value()


def golden():
    return json.load(open(GOLDEN))


def ref_value(rec):
    v = rec["value"]
    if isinstance(v, str):
        return int(v)
    if "hi" in v:
        return v["hi"] + v["lo"]
    return complex(v["re"]["hi"] + v["re"]["lo"], v["im"]["hi"] + v["im"]["lo"])


def abs_ref(rec):
    v = rec.get("per_abs")
    if v is None:
        return None
    if "hi" in v:
        return v["hi"] + v["lo"]
    return v["re"]["hi"] + v["re"]["lo"]


def formula_abs_sums(a):
    """Condition scales of the two formulas for a square real matrix (n <= 22):
    Ryser: sum over column sets S of |prod_i sum_{j in S} a_ij|;
    Glynn: 2^-(n-1) sum over sign vectors (delta_1 = +1) of |prod_j sum_i delta_i a_ij|.
    Each term is computed with a relative error of a few n u, so the error of a
    binary64 evaluation is bounded by a small multiple of n u times these."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    ryser = glynn = 0.0
    for s0 in range(0, 1 << n, 1 << 16):
        idx = np.arange(s0, min(1 << n, s0 + (1 << 16)))
        bits = ((idx[:, None] >> np.arange(n)) & 1).astype(np.float64)
        ryser += np.abs(np.prod(bits @ a.T, axis=1)).sum()
    for s0 in range(0, 1 << (n - 1), 1 << 16):
        idx = np.arange(s0, min(1 << (n - 1), s0 + (1 << 16)))
        d = np.ones((len(idx), n))
        d[:, 1:] = 1 - 2 * ((idx[:, None] >> np.arange(n - 1)) & 1)
        glynn += np.abs(np.prod(d @ a, axis=1)).sum() / 2.0 ** (n - 1)
    return ryser, glynn
