"""Exact matrix permanents on AMD MI355X (gfx950).

Thin Python layer over the C ABI of ``libpermgpu.so`` (``include/perm.h``):
it maps torch tensors to (pointer, shape, leading dimension, dtype) and
passes torch's current HIP stream.  All computation happens in the HIP
library; there is no CPU fallback.

    >>> import torch, paper_2510_03421_amd as pg
    >>> a = torch.tensor([[1, 2, 3], [4, 5, 6], [7, 8, 9]], device="cuda")
    >>> pg.value(pg.glynn(a))
    450
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import _capi as C
from ._capi import PermError

__all__ = ["glynn", "glynn_esym", "ryser", "combinatoric", "column_sweep", "auto", "value", "PermError", "BatchPlan",
           "glynn_batched", "ryser_batched", "auto_batched", "gray_chunk", "select", "selector_load", "ALGORITHMS", "version",
           "profile_enable", "profile_last_ms", "profile_durations_ms", "workspace_release"]

ALGORITHMS = {C.PERM_ALGO_COMBINATORIC: "combinatoric", C.PERM_ALGO_RYSER: "ryser",
              C.PERM_ALGO_GLYNN: "glynn", C.PERM_ALGO_GLYNN_ESYM: "glynn_esym",
              C.PERM_ALGO_SWEEP: "column_sweep"}
_ALGO_ID = {v: k for k, v in ALGORITHMS.items()}
_ALGO_ID["auto"] = C.PERM_ALGO_AUTO

_DT = {torch.float64: C.PERM_F64, torch.complex128: C.PERM_C128, torch.int64: C.PERM_I64,
       torch.uint8: C.PERM_B8, torch.bool: C.PERM_B8}
_OUT = {"f64": C.PERM_OUT_F64, "c128": C.PERM_OUT_C128, "i64": C.PERM_OUT_I64,
        "i128": C.PERM_OUT_I128, "dd": C.PERM_OUT_DD, "cdd": C.PERM_OUT_CDD}
_DEFAULT_OUT = {C.PERM_F64: "f64", C.PERM_C128: "c128", C.PERM_I64: "i128", C.PERM_B8: "i128"}
# output buffer: (torch dtype, element count)
_OUTBUF = {"f64": (torch.float64, 1), "c128": (torch.float64, 2), "i64": (torch.int64, 1),
           "i128": (torch.int64, 2), "dd": (torch.float64, 2), "cdd": (torch.float64, 4)}


def version() -> int:
    return int(C.lib.perm_version())


def workspace_release() -> None:
    """Free the library's cached device tables and trim the stream-ordered pool."""
    C.check(C.lib.perm_workspace_release(), "perm_workspace_release")


def profile_enable(on: bool = True) -> None:
    """Record HIP events around the main kernel of every later call."""
    C.check(C.lib.perm_profile_enable(1 if on else 0), "perm_profile_enable")


def profile_last_ms() -> float:
    """Duration of the main kernel of this thread's last call (waits for it)."""
    ms = ctypes.c_double(0.0)
    C.check(C.lib.perm_profile_last(ctypes.byref(ms)), "perm_profile_last")
    return ms.value


def profile_durations_ms() -> list:
    """Main-kernel durations of every call since profile_enable(True), in
    call order (waits for them)."""
    count = ctypes.c_int(0)
    C.check(C.lib.perm_profile_durations(None, 0, ctypes.byref(count)), "perm_profile_durations")
    buf = (ctypes.c_double * max(1, count.value))()
    C.check(C.lib.perm_profile_durations(buf, count.value, ctypes.byref(count)),
            "perm_profile_durations")
    return list(buf[:count.value])


def _matrix(a: torch.Tensor):
    if not isinstance(a, torch.Tensor) or a.dim() != 2:
        raise TypeError("expected a 2-D torch tensor")
    if a.device.type != "cuda":
        raise ValueError("the matrix must be on a HIP device")
    if a.dtype not in _DT:
        raise TypeError(f"unsupported dtype {a.dtype}")
    if a.dtype == torch.bool:
        a = a.to(torch.uint8)
    if a.shape[0] > 0 and a.shape[1] > 0 and (a.stride(1) != 1 or a.stride(0) < a.shape[1]):
        a = a.contiguous()
    lda = a.stride(0) if a.shape[0] > 0 and a.shape[1] > 0 else max(1, a.shape[1])
    return a, _DT[a.dtype], lda


def _out_for(dt: int, out: str | None, device) -> tuple[torch.Tensor, str]:
    out = out or _DEFAULT_OUT[dt]
    if out not in _OUT:
        raise ValueError(f"unknown output type {out!r}")
    tdt, cnt = _OUTBUF[out]
    return torch.empty(cnt, dtype=tdt, device=device), out


def _stream(a: torch.Tensor) -> int:
    return torch.cuda.current_stream(a.device).cuda_stream


class Result:
    """A device-resident permanent and its output type; ``value()`` syncs."""

    __slots__ = ("buf", "kind", "algo")

    def __init__(self, buf: torch.Tensor, kind: str, algo: int | None = None):
        self.buf, self.kind, self.algo = buf, kind, algo

    def value(self):
        return value(self)


def _run(fn, a, out, flags):
    a, dt, lda = _matrix(a)
    buf, kind = _out_for(dt, out, a.device)
    m, n = a.shape
    with torch.cuda.device(a.device):
        C.check(fn(m, n, dt, a.data_ptr(), lda, _OUT[kind], buf.data_ptr(), flags,
                   _stream(a)), fn.__name__)
    return Result(buf, kind)


def glynn(a: torch.Tensor, out: str | None = None, flags: int = 0) -> Result:
    """Glynn's formula (square; rectangular via padding rows of 2^e scaled to
    the data, or of ones with flags=PERM_FLAG_PAD_ONES)."""
    return _run(C.lib.perm_glynn, a, out, flags)


def ryser(a: torch.Tensor, out: str | None = None, flags: int = 0) -> Result:
    """Ryser's formula (square; rectangular by subset size).  Square sparse
    input skips the column subsets that leave a row empty (a column window;
    floating point from n = 30, complex 29, or at any n with
    flags=PERM_FLAG_SPARSE)."""
    return _run(C.lib.perm_ryser, a, out, flags)


def glynn_esym(a: torch.Tensor, out: str | None = None, flags: int = 0) -> Result:
    """Rectangular Glynn with the padding rows summed out: a sum over the signs
    of the m rows of e_m of the column sums (floating-point outputs)."""
    return _run(C.lib.perm_glynn_esym, a, out, flags)


def gray_chunk(a: torch.Tensor, algo: str, chunk_log2: int, chunk: int, out: str | None = None,
               flags: int = 0) -> Result:
    """One chunk of the Glynn or square Ryser sum (perm_gray_chunk): the Gray
    indices [chunk 2^chunk_log2, (chunk+1) 2^chunk_log2), scaled so that the
    values of all chunks add up to the permanent."""
    a, dt, lda = _matrix(a)
    buf, kind = _out_for(dt, out, a.device)
    m, n = a.shape
    with torch.cuda.device(a.device):
        C.check(C.lib.perm_gray_chunk(_ALGO_ID[algo], m, n, dt, a.data_ptr(), lda, _OUT[kind],
                                      buf.data_ptr(), flags, int(chunk_log2), int(chunk), _stream(a)),
                "perm_gray_chunk")
    return Result(buf, kind)


def column_sweep(a: torch.Tensor, out: str | None = None, flags: int = 0) -> Result:
    """The definition regrouped column by column over the 2^m row subsets
    (perm_column_sweep): no subtraction of computed values."""
    return _run(C.lib.perm_column_sweep, a, out, flags)


def combinatoric(a: torch.Tensor, out: str | None = None, flags: int = 0) -> Result:
    """The definition: one product per injective row -> column map."""
    return _run(C.lib.perm_combinatoric, a, out, flags)


def auto(a: torch.Tensor, out: str | None = None, flags: int = 0,
         density: float = -1.0) -> Result:
    """Algorithm chosen by the selector (learned, else threshold table)."""
    a, dt, lda = _matrix(a)
    buf, kind = _out_for(dt, out, a.device)
    m, n = a.shape
    chosen = ctypes.c_int(-1)
    with torch.cuda.device(a.device):
        C.check(C.lib.perm_auto(m, n, dt, a.data_ptr(), lda, _OUT[kind], buf.data_ptr(), flags,
                                _stream(a), float(density), ctypes.byref(chosen)), "perm_auto")
    return Result(buf, kind, chosen.value)


def select(m: int, n: int, dtype: torch.dtype = torch.float64, density: float = -1.0):
    """(algorithm name, decided-by-learned-selector) that ``auto`` would use."""
    chosen, src = ctypes.c_int(-1), ctypes.c_int(-1)
    C.check(C.lib.perm_select(m, n, _DT[dtype], float(density), ctypes.byref(chosen),
                              ctypes.byref(src)), "perm_select")
    return ALGORITHMS[chosen.value], bool(src.value)


def ryser_window_plan(row_masks, lanes_max: int, force: bool = False):
    """The column window square ``ryser`` walks for an n x n matrix
    with nonzero pattern ``row_masks`` (n ints, bit j of row i = a_ij != 0):
    None for the whole walk, else a dict with fw, b, wlow, col_order and
    states (host only).  ``force``: any window that prunes (what
    PERM_RYSER_WINDOW=2 makes perm_ryser use)."""
    import numpy as np
    rm = np.ascontiguousarray(np.asarray(row_masks, dtype=np.uint64))
    n = rm.size
    fw, b, wlow = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    ns = ctypes.c_uint64(0)
    col = np.zeros(max(n, 1), dtype=np.int32)
    cap = 1 << 16
    st = np.zeros(cap, dtype=np.uint32)
    rc = C.lib.perm_ryser_window_plan(n, rm.ctypes.data, int(lanes_max), int(force),
                                      ctypes.byref(fw),
                                      ctypes.byref(b), ctypes.byref(wlow), ctypes.byref(ns),
                                      col.ctypes.data, st.ctypes.data, cap)
    if rc < 0:
        C.check(rc, "perm_ryser_window_plan")
    if rc == 0:
        return None
    return {"fw": fw.value, "b": b.value, "wlow": wlow.value, "col_order": col[:n].copy(),
            "states": st[:ns.value].copy()}


def selector_load(path: str | None) -> None:
    C.check(C.lib.perm_selector_load(path.encode() if path else None), "perm_selector_load")


# Selector weights trained on MI355X timings ship beside the library; perm_auto
# uses them from import on (selector_load(None) returns to the table).
SELECTOR_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.txt")
if os.path.exists(SELECTOR_WEIGHTS):
    C.check(C.lib.perm_selector_load(SELECTOR_WEIGHTS.encode()), "perm_selector_load")


def value(r: Result):
    """Copy a result to the host: int (exact), float, or complex.  For "dd" /
    "cdd" outputs returns (hi, lo) / ((re.hi, re.lo), (im.hi, im.lo))."""
    v = r.buf.cpu()
    k = r.kind
    if k == "f64":
        return float(v[0])
    if k == "c128":
        return complex(float(v[0]), float(v[1]))
    if k == "i64":
        return int(v[0])
    if k == "i128":
        lo, hi = int(v[0]) & (2 ** 64 - 1), int(v[1])
        return (hi << 64) | lo
    if k == "dd":
        return (float(v[0]), float(v[1]))
    return ((float(v[0]), float(v[1])), (float(v[2]), float(v[3])))


class BatchPlan:
    """A planned batch of square or rectangular matrices in one device buffer
    (see perm_batch_plan_create).  ``run`` replays a captured hipGraph."""

    def __init__(self, m, n, offset, ld, dtype: torch.dtype, out: str | None = None,
                 algo: str = "glynn", flags: int = 0, autotune: bool = False):
        import numpy as np
        self.m = np.ascontiguousarray(m, dtype=np.int32)
        self.n = np.ascontiguousarray(n, dtype=np.int32)
        self.offset = np.ascontiguousarray(offset, dtype=np.int64)
        self.ld = np.ascontiguousarray(ld, dtype=np.int64)
        self.count = int(self.n.shape[0])
        self.dt = _DT[dtype]
        self.kind = out or _DEFAULT_OUT[self.dt]
        self._h = ctypes.c_void_p()
        C.check(C.lib.perm_batch_plan_create(
            self.count, self.m.ctypes.data, self.n.ctypes.data, self.offset.ctypes.data,
            self.ld.ctypes.data, self.dt, _OUT[self.kind], _ALGO_ID[algo],
            flags | (C.PERM_BATCH_AUTOTUNE if autotune else 0),
            ctypes.byref(self._h)), "perm_batch_plan_create")

    def packing(self, n: int) -> int:
        """Matrices per wave used for order n (0: chunked kernel or absent)."""
        return int(C.lib.perm_batch_plan_packing(self._h, int(n)))

    def new_output(self, device="cuda") -> torch.Tensor:
        tdt, cnt = _OUTBUF[self.kind]
        return torch.empty(self.count * cnt, dtype=tdt, device=device)

    def run(self, data: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        C.check(C.lib.perm_batch_plan_run(self._h, data.data_ptr(), out.data_ptr(),
                                          _stream(data)), "perm_batch_plan_run")
        return out

    def close(self):
        if self._h:
            C.lib.perm_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batched_once(fn, data: torch.Tensor, m, n, offset, ld, out, flags) -> torch.Tensor:
    import numpy as np
    m = np.ascontiguousarray(m, dtype=np.int32)
    n = np.ascontiguousarray(n, dtype=np.int32)
    offset = np.ascontiguousarray(offset, dtype=np.int64)
    ld = np.ascontiguousarray(ld, dtype=np.int64)
    if data.dtype == torch.bool:
        data = data.to(torch.uint8)
    dt = _DT[data.dtype]
    kind = out or _DEFAULT_OUT[dt]
    tdt, cnt = _OUTBUF[kind]
    res = torch.empty(len(n) * cnt, dtype=tdt, device=data.device)
    C.check(fn(len(n), m.ctypes.data, n.ctypes.data, offset.ctypes.data, ld.ctypes.data, dt,
               data.data_ptr(), _OUT[kind], res.data_ptr(), flags, _stream(data)), fn.__name__)
    return res


def glynn_batched(data: torch.Tensor, m, n, offset, ld, out: str | None = None,
                  flags: int = 0) -> torch.Tensor:
    """One-shot batched Glynn (no graph capture): square matrices by Glynn's
    formula, rectangular ones by the e_m form (rows of ones with
    flags=PERM_FLAG_PAD_ONES)."""
    return _batched_once(C.lib.perm_glynn_batched, data, m, n, offset, ld, out, flags)


def ryser_batched(data: torch.Tensor, m, n, offset, ld, out: str | None = None,
                  flags: int = 0) -> torch.Tensor:
    """One-shot batched Ryser (square matrices)."""
    return _batched_once(C.lib.perm_ryser_batched, data, m, n, offset, ld, out, flags)


def auto_batched(data: torch.Tensor, m, n, offset, ld, out: str | None = None,
                 flags: int = 0) -> torch.Tensor:
    """One-shot batch with the sum chosen per matrix (perm_auto_batched)."""
    return _batched_once(C.lib.perm_auto_batched, data, m, n, offset, ld, out, flags)
