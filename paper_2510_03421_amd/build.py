"""Build ``libpermgpu.so`` (the HIP library behind ``include/perm.h``) for gfx950.

Each source under ``csrc/`` is compiled by hipcc in parallel and the objects
are linked into one shared library next to this file.  Runs without a GPU.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libpermgpu.so")
OBJDIR = os.path.join(ROOT, "_build", "permgpu")

ARCH = os.environ.get("PERM_GFX", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    # packed FP32 instructions are not used anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
]

def _sources():
    # the slowest translation units first, so the pool finishes early
    order = ["esym_int", "ryser_rect", "gray_int", "esym_cplx", "gray_cplx", "batched_cplx",
             "batched_real", "gray_real"]
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    key = lambda f: (next((i for i, p in enumerate(order) if f.startswith(p)), len(order)), f)
    return sorted(srcs, key=key)


def _band_units():
    """The banded e_m objects: esym_band.inc compiled once per X(kind, m_lo,
    m_hi) entry of esym_band_ranges.h."""
    import re
    text = open(os.path.join(CSRC, "esym_band_ranges.h")).read()
    units = []
    for k, lo, hi in re.findall(r"X\((\d+),\s*(\d+),\s*(\d+)\)", text):
        units.append((f"esym_band_{k}_{lo}", "esym_band.inc",
                      ["-x", "hip", f"-DESYM_KIND={k}", f"-DESYM_M_LO={lo}", f"-DESYM_M_HI={hi}"]))
    # complex (slower) first
    return sorted(units, key=lambda u: u[2][2] != "-DESYM_KIND=1")


def _walk_units():
    """The staged batch walk objects: batched_walk.inc compiled once per
    X(kind, esym, nv_lo, nv_hi) entry of batched_walk_units.h."""
    import re
    text = open(os.path.join(CSRC, "batched_walk_units.h")).read()
    units = []
    for k, e, lo, hi in re.findall(r"X\((\d+),\s*(\d+),\s*(\d+),\s*(\d+)\)", text):
        units.append((f"batched_walk_{k}{e}_{lo}_{hi}", "batched_walk.inc",
                      ["-x", "hip", f"-DBW_KIND={k}", f"-DBW_ESYM={e}", f"-DBW_NV_LO={lo}",
                       f"-DBW_NV_HI={hi}"]))
    # the exact-integer e_m units (slowest) first
    return sorted(units, key=lambda u: not (u[2][2] == "-DBW_KIND=2" and u[2][3] == "-DBW_ESYM=1"))


SOURCES = _sources()
EXTRA = {f: ["-x", "hip"] for f in SOURCES if f.endswith(".cpp")}
# (object name, source file, extra flags): banded units first, then one object per source
UNITS = _walk_units() + _band_units() + [(os.path.splitext(f)[0], f, EXTRA.get(f, [])) for f in SOURCES]


def _compile(unit, verbose: bool) -> str:
    name, src, extra = unit
    obj = os.path.join(OBJDIR, name + ".o")
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines()
            if "packed-fp32-ops" not in ln and ln.strip()]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {name} ({src}):\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    if verbose:
        print(f"  {name}: {time.time() - t0:.1f}s", flush=True)
    return obj


def _includes(path: str, seen: set) -> set:
    """Local files `path` includes, recursively (quoted #include only)."""
    import re
    for inc in re.findall(r'^\s*#\s*include\s+"([^"]+)"', open(path).read(), flags=re.M):
        dep = os.path.normpath(os.path.join(os.path.dirname(path), inc))
        if os.path.exists(dep) and dep not in seen:
            seen.add(dep)
            _includes(dep, seen)
    return seen


def _stale(unit) -> bool:
    name, src, _ = unit
    obj = os.path.join(OBJDIR, name + ".o")
    if not os.path.exists(obj):
        return True
    path = os.path.join(CSRC, src)
    deps = [path] + sorted(_includes(path, set()))
    return max(os.path.getmtime(d) for d in deps) > os.path.getmtime(obj)


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every unit (or, with ``incremental``, only those older than
    their inputs) and link ``libpermgpu.so``."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or max(1, min(len(UNITS), os.cpu_count() or 1))
    todo = [u for u in UNITS if not incremental or _stale(u)]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda u: _compile(u, verbose), todo))
    objs = [os.path.join(OBJDIR, u[0] + ".o") for u in UNITS]
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    t = time.time()
    build(verbose="-v" in sys.argv, incremental="-i" in sys.argv)
    print(f"built {OUT} in {time.time() - t:.1f}s")
