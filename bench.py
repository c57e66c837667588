"""Benchmark: Glynn's formula on the 32 x 32 float64 workload (entries
uniform on [-1, 1], seed 3201) -- the hot path's headline configuration.

One step = one perm_glynn call on a device-resident matrix: staging of the
update table, 2^31 Gray-code terms (closed-form re-seed per lane block, one
row update and one 32-factor product per term, compensated accumulation),
the deterministic reduction and the final scaling.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 32
SEED = 3201
TERMS = 2 ** (N - 1)
OPS_PER_TERM = 2 * N          # N adds (update) + (N-1) multiplies + 1 add (accumulate)
# FP64 vector issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# = 39.32e12 lane-operations/s (an FMA counts 2 flops, giving the published
# 78.6 TFLOP/s; an add or a multiply counts one).
PEAK_FP64_OPS = 256 * 4 * 16 * 2.4e9


def cpu_baseline(a, budget_s: float = 15.0):
    """The oracle's double-double Glynn evaluator timed on a bounded sample of
    the same workload: the first K Gray-code terms of the 32 x 32 matrix."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else \
        oracle.hardware_threads()
    k = 1 << 20
    t0 = time.perf_counter()
    oracle.per_glynn(a, nthreads=threads, k0=0, k1=k, partial=True)
    dt = time.perf_counter() - t0
    rate = k / max(dt, 1e-9)
    k = int(min(TERMS, max(1 << 20, rate * budget_s)))
    k = 1 << max(20, k.bit_length() - 1)
    t0 = time.perf_counter()
    oracle.per_glynn(a, nthreads=threads, k0=0, k1=k, partial=True)
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "terms/s", "cores": threads, "kind": "oracle",
            "sample": f"first {k} of the 2^31 Gray-code terms of the same 32x32 matrix "
                      f"(double-double Glynn evaluator, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this library computes one permanent per GPU call and is "
              "measured on a single GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_03421_amd as pg
    import workloads

    a_host = workloads.uniform(N, N, SEED)
    a = torch.from_numpy(a_host).cuda()
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    from paper_2510_03421_amd import _capi as C
    stream = torch.cuda.current_stream().cuda_stream

    def step():
        C.check(C.lib.perm_glynn(N, N, C.PERM_F64, a.data_ptr(), N, C.PERM_OUT_DD,
                                 out.data_ptr(), 0, stream), "perm_glynn")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K steps, synchronised on both sides
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps

    # kernel durations with HIP events recorded by the library on this stream
    pg.profile_enable(True)
    kms = []
    for _ in range(args.steps):
        step()
        kms.append(pg.profile_last_ms())
    pg.profile_enable(False)
    kernel_ms = float(np.mean(kms))

    hi, lo = out.cpu().tolist()
    result = hi + lo
    ref = None
    gold = os.path.join(ROOT, "tests", "golden", "reference_values.json")
    err = {}
    if os.path.exists(gold):
        rec = json.load(open(gold)).get("u32")
        if rec:
            ref = rec["value"]["hi"] + rec["value"]["lo"]
            pabs = rec["per_abs"]["hi"]
            d = abs(result - ref)
            err = {"abs_err": d, "rel_err": d / abs(ref), "err_over_per_abs": d / pabs,
                   "criterion_1e-11_per_abs": bool(d <= 1e-11 * pabs)}

    achieved = TERMS * OPS_PER_TERM / (kernel_ms * 1e-3) / 1e12
    peak = PEAK_FP64_OPS / 1e12
    line = {
        "metric": "Gray-code terms/s (n=32 Glynn, FP64)",
        "value": TERMS / (ms_per_step * 1e-3),
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "glynn_32x32_f64_uniform[-1,1]", "m": N, "n": N, "seed": SEED,
                   "terms": TERMS, "algorithm": "glynn", "output": "double-double"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel_ms": kernel_ms,
                     "note": "FP64 add/mul lane-ops (1 each) of the Gray-walk engine kernel: "
                             "64 per term x 2^31 terms; peak = FP64 VALU issue rate "
                             "(78.6 TFLOP/s counts an FMA as 2)"},
        "fp64_frac_of_78.6": achieved * 1e12 / 78.6e12,
        "result": result,
        "error_vs_oracle": err,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(a_host)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
