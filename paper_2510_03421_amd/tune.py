"""Timing generator for the algorithm selector: times every algorithm the
library offers on seeded (m, n, density, dtype) cases on the current GPU and
writes one CSV row per case.

    python -m paper_2510_03421_amd.tune --out timings.csv [--cases 5000]
           [--start 0] [--stop 5000]

A run that would take long is timed on cut-down fractions of its work
(``perm_time``) and extrapolated linearly to the whole: t(f) = a + b f,
where a holds the fixed costs (planning, staging, reduction, launch latency)
and b the time of the whole walk.  Integer (0/1) cases are
timed with PERM_FLAG_WRAP, so that no data-dependent overflow refusal hides a
run time; an algorithm whose size limits refuse the shape gets an empty cell.
Rows are appended as they are measured, so an interrupted run can continue
with --start.
"""
from __future__ import annotations

import argparse
import os
import sys
import time as _time

import numpy as np
import torch

from . import _capi as C
from . import selector as S

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)
import workloads  # noqa: E402  (seeded case recipes)

HEADER = "i,m,n,dtype,density,seed," + ",".join(
    f"{k}_{a}" for k in ("ms", "frac", "s") for a in S.ALGO_ORDER)
TORCH_DT = {"f64": torch.float64, "c128": torch.complex128, "b8": torch.uint8}
SLOPE_MS = 3.0       # the cut-down run used for the slope adds at least this much
FULL_MS = 25.0       # whole runs shorter than this are timed again with more repetitions


def time_algo(algo: str, a: torch.Tensor, flags: int):
    """(estimated full ms, fraction of the slope run) or (None, None) if the
    algorithm refuses the shape.

    t0 is the time of the smallest cut-down run (fraction r0: fixed costs and
    the least work the cut allows).  A second run at r0 + e, with e sized
    from the first guess t0 / r0 of the whole run's time and corrected by the
    measured ratio until the run adds about max(SLOPE_MS, t0 / 4), gives the
    slope; the full time is t0 + (1 - r0) (t - t0) / (r - r0)."""
    try:
        t0, r0 = S.time(algo, a, fraction=1e-12, reps=1, flags=flags)
    except C.PermError as e:
        if e.status in (C.PERM_E_TOO_LARGE, C.PERM_E_UNSUPPORTED):
            return None, None
        raise
    if t0 < FULL_MS:
        t0, r0 = S.time(algo, a, fraction=1e-12, reps=2, flags=flags)
    if r0 >= 1.0:
        return t0, 1.0
    target = max(SLOPE_MS, 0.25 * t0)
    e = min(1.0, max(1e-9, target * r0 / max(t0, 1e-3)))
    t, r = t0, r0
    for _ in range(12):
        t, r = S.time(algo, a, fraction=min(1.0, r0 + e), reps=1, flags=flags)
        if r >= 1.0 or (r > r0 and t - t0 >= 0.5 * target):
            break
        grow = 8.0 if t - t0 <= 0.05 * target or r <= r0 else min(8.0, 1.5 * target / (t - t0))
        e = min(1.0, e * max(grow, 1.5))
    if r >= 1.0:
        if t < FULL_MS:
            t, _ = S.time(algo, a, fraction=1.0, reps=3, flags=flags)
        return t, 1.0
    return t0 + (1.0 - r0) * (t - t0) / (r - r0), r


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--cases", type=int, default=5000)
    ap.add_argument("--seed", type=int, default=5000)
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--stop", type=int, default=None)
    args = ap.parse_args(argv)
    cases = workloads.selector_cases(args.cases, seed=args.seed)
    stop = args.cases if args.stop is None else min(args.stop, args.cases)
    new = not os.path.exists(args.out) or os.path.getsize(args.out) == 0
    dev = torch.device("cuda", torch.cuda.current_device())
    t_start = _time.time()
    with open(args.out, "a") as fh:
        if new:
            fh.write(HEADER + "\n")
        for i in range(args.start, stop):
            c = cases[i]
            a = workloads.case_matrix(c)
            density = float(np.count_nonzero(a)) / a.size
            at = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
            flags = C.PERM_FLAG_WRAP if c["dtype"] == "b8" else 0
            ms, fr, spent = [], [], []
            for algo in S.ALGO_ORDER:
                t_a = _time.time()
                t, f = time_algo(algo, at, flags)
                spent.append(f"{_time.time() - t_a:.3g}")
                ms.append("" if t is None else f"{t:.6g}")
                fr.append("" if f is None else f"{f:.6g}")
            fh.write(f"{i},{c['m']},{c['n']},{c['dtype']},{density:.6g},{c['seed']},"
                     + ",".join(ms + fr + spent) + "\n")
            fh.flush()
            if (i + 1) % 50 == 0 or i + 1 == stop:
                print(f"tune: case {i + 1}/{stop} done, {(_time.time() - t_start):.0f} s",
                      flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
