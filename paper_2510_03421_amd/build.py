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


SOURCES = _sources()
EXTRA = {f: ["-x", "hip"] for f in SOURCES if f.endswith(".cpp")}


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines()
            if "packed-fp32-ops" not in ln and ln.strip()]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    if verbose:
        print(f"  {src}: {time.time() - t0:.1f}s", flush=True)
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


def _stale(src: str) -> bool:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    if not os.path.exists(obj):
        return True
    path = os.path.join(CSRC, src)
    deps = [path] + sorted(_includes(path, set()))
    return max(os.path.getmtime(d) for d in deps) > os.path.getmtime(obj)


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every source (or, with ``incremental``, only those older than
    their inputs) and link ``libpermgpu.so``."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1))
    todo = [s for s in SOURCES if not incremental or _stale(s)]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda s: _compile(s, verbose), todo))
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
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
