"""Write tests/golden/reference_values.json: reference permanents of the
full-size seeded workloads, computed by the CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py [names...]
Each entry records the workload recipe (``workloads.CONFIGS``), the evaluator
used, the value (exact integer, or double-double hi/lo) and, for floating
point inputs, per(|A|) (the scale of the error criterion).

``--second name...`` adds to existing entries the value of a second,
independent evaluator: for the Glynn-evaluated inputs (32x32 real and complex,
36x36 real) the double-double Ryser sum over column subsets (Sec. 1.2
Eq. ryser_square), which shares no seeding or update step with the Glynn walk
over row signs; the tests check that the two agree within their error bounds.
Set ``ORACLE_THREADS`` to limit the threads used.

``--batches`` writes tests/golden/batch_reference.json: the oracle's values of
the first matrices of the benchmark's batched workloads.
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


THREADS = int(os.environ.get("ORACLE_THREADS", "0"))


def evaluate_second(name, rec):
    """Add the double-double Ryser value of workload ``name`` to ``rec``."""
    a = workloads.config_matrix(name)
    t = time.time()
    rec["value_ryser"] = dd_json(oracle.per_ryser(a, nthreads=THREADS))
    rec["seconds_ryser"] = round(time.time() - t, 1)
    return rec


def _read():
    return json.load(open(OUT)) if os.path.exists(OUT) else {}


def main(names, second=False):
    for name in names:
        print(f"{name} ...", flush=True)
        rec = evaluate_second(name, _read()[name]) if second else evaluate(name)
        data = _read()  # re-read: another run may have added entries meanwhile
        data[name] = rec
        print(json.dumps(rec), flush=True)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)


BATCH_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_reference.json")


def batches(sample: int = 400):
    """Reference permanents of the first `sample` matrices of the benchmark's
    two batches: the 200,000 Haar submatrices (complex double-double Glynn)
    and the 20,000 0/1 matrices (exact, memoised expansion)."""
    out = {}
    b = workloads.boson_batch(200_000, 4, 20, N=64, seed_u=6400, seed_idx=6401)
    vals = []
    for i in range(sample):
        v = oracle.per_glynn(np.ascontiguousarray(b.matrix(i)))
        vals.append([v.re.hi, v.re.lo, v.im.hi, v.im.lo])
    out["boson_200000_c128_n4..20"] = {"recipe": "workloads.boson_batch(200000, 4, 20, N=64, "
                                       "seed_u=6400, seed_idx=6401)", "evaluator": "glynn",
                                       "first": sample, "values": vals}
    z = workloads.bernoulli_batch(20_000, 8, 24, 0.5, seed=6500)
    ints = [str(oracle.per_laplace(np.ascontiguousarray(z.matrix(i)).astype(np.int64)))
            for i in range(sample)]
    out["bernoulli_20000_b8_n8..24"] = {"recipe": "workloads.bernoulli_batch(20000, 8, 24, 0.5, "
                                        "seed=6500)", "evaluator": "laplace", "first": sample,
                                        "values": ints}
    with open(BATCH_OUT + ".tmp", "w") as fh:
        json.dump(out, fh)
    os.replace(BATCH_OUT + ".tmp", BATCH_OUT)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--second":
        main(args[1:] or ["u32", "c32", "u36"], second=True)
    elif args and args[0] == "--batches":
        batches()
    else:
        main(args or ["u12", "b16x48", "u20x40", "b28", "u32", "b30", "c32"])
