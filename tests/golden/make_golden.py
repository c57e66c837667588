"""Write tests/golden/reference_values.json: reference permanents of the
full-size seeded workloads, computed by the CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py [names...]
Each entry records the workload recipe (``workloads.CONFIGS``), the evaluator
used, the value (exact integer, or double-double hi/lo) and, for floating
point inputs, per(|A|) (the scale of the error criterion).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "reference_values.json")


def dd_json(v):
    if isinstance(v, oracle.DD):
        return {"hi": v.hi, "lo": v.lo}
    return {"re": {"hi": v.re.hi, "lo": v.re.lo}, "im": {"hi": v.im.hi, "lo": v.im.lo}}


def evaluate(name):
    a = workloads.config_matrix(name)
    m, n = a.shape
    rec = {"name": name, "recipe": workloads.CONFIGS[name], "m": m, "n": n}
    t = time.time()
    if a.dtype == np.uint8:
        rec["evaluator"] = "laplace"
        rec["value"] = str(oracle.per_laplace(a.astype(np.int64)))
    elif min(m, n) <= 24 or max(m, n) <= 28:
        rec["evaluator"] = "laplace"
        rec["value"] = dd_json(oracle.per_laplace(a))
        rec["per_abs"] = dd_json(oracle.per_laplace(np.abs(a)))
    else:
        rec["evaluator"] = "glynn"
        rec["value"] = dd_json(oracle.per_glynn(a))
        rec["per_abs"] = dd_json(oracle.per_glynn(np.abs(a)))
    rec["seconds"] = round(time.time() - t, 1)
    rec["threads"] = oracle.hardware_threads()
    return rec


def main(names):
    data = {}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    for name in names:
        print(f"{name} ...", flush=True)
        data[name] = evaluate(name)
        print(json.dumps(data[name]), flush=True)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:] or ["u12", "b16x48", "u20x40", "b28", "u32", "b30", "c32"])
