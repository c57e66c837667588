"""Reference permanents -- TEST INFRASTRUCTURE ONLY.

Plain CPU evaluators of the matrix permanent (Masschelein, Richer & Ayers,
Sec. 1.1 Eq. permanent_definition / Eq. rectangular_permanent_definition).
Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never calls it, and it
never calls the HIP library.

Evaluators (all in ``perm_oracle.c``):

* ``per_brute``   -- the definition: one product per injective row->column map.
* ``per_laplace`` -- the same sum grouped by distributivity (memoised Laplace
  expansion over column sets or row sets).
* ``per_glynn``   -- Eq. glynn / Eq. glynn_rectangle in double-double, Gray order.
* ``per_ryser``   -- Eq. ryser_square / Eq. ryser_rectangle (over column
  subsets) in double-double, Gray order.

Integer inputs are evaluated modulo 2^128 and returned as the signed Python
``int`` of that residue; real inputs return :class:`DD`; complex inputs
return :class:`CDD`.
"""
from __future__ import annotations

import ctypes
import os
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

__all__ = ["DD", "CDD", "per_brute", "per_laplace", "per_glynn", "per_ryser",
           "hardware_threads", "lib_path", "load"]


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Load ``liboracle.so`` (built by ``oracle/build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32, i64, p = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    u64 = ctypes.c_uint64
    for name in ("oracle_brute_i64", "oracle_brute_f64", "oracle_brute_c128"):
        getattr(lib, name).argtypes = [i32, i32, p, i64, i32, p]
        getattr(lib, name).restype = i32
    for name in ("oracle_laplace_i64", "oracle_laplace_f64", "oracle_laplace_c128"):
        getattr(lib, name).argtypes = [i32, i32, p, i64, i32, i32, p]
        getattr(lib, name).restype = i32
    for name in ("oracle_glynn_f64", "oracle_glynn_c128"):
        getattr(lib, name).argtypes = [i32, i32, p, i64, i32, u64, u64, i32, p]
        getattr(lib, name).restype = i32
    for name in ("oracle_ryser_f64", "oracle_ryser_c128"):
        getattr(lib, name).argtypes = [i32, i32, p, i64, i32, p]
        getattr(lib, name).restype = i32
    lib.oracle_hardware_threads.argtypes = []
    lib.oracle_hardware_threads.restype = i32
    _lib = lib
    return lib


def hardware_threads() -> int:
    return int(load().oracle_hardware_threads())


class DD:
    """A double-double value hi + lo."""

    __slots__ = ("hi", "lo")

    def __init__(self, hi: float, lo: float = 0.0):
        self.hi = float(hi)
        self.lo = float(lo)

    def __float__(self) -> float:
        return self.hi + self.lo

    def frac(self) -> Fraction:
        return Fraction(self.hi) + Fraction(self.lo)

    def __repr__(self) -> str:
        return f"DD({self.hi!r}, {self.lo!r})"


class CDD:
    """A complex double-double value."""

    __slots__ = ("re", "im")

    def __init__(self, re: DD, im: DD):
        self.re, self.im = re, im

    def __complex__(self) -> complex:
        return complex(float(self.re), float(self.im))

    def frac(self):
        return self.re.frac(), self.im.frac()

    def __repr__(self) -> str:
        return f"CDD({self.re!r}, {self.im!r})"


def _kind(a: np.ndarray) -> str:
    if np.iscomplexobj(a):
        return "c128"
    if a.dtype.kind in "biu":
        return "i64"
    if a.dtype.kind == "f":
        return "f64"
    raise TypeError(f"unsupported dtype {a.dtype}")


def _prep(a):
    a = np.asarray(a)
    if a.ndim != 2:
        raise ValueError("expected a 2-D matrix")
    kind = _kind(a)
    dt = {"i64": np.int64, "f64": np.float64, "c128": np.complex128}[kind]
    a = np.ascontiguousarray(a, dtype=dt)
    return a, kind


def _signed128(lo: int, hi: int) -> int:
    v = (hi << 64) | lo
    return v - (1 << 128) if v >> 127 else v


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def _decode(kind: str, out):
    if kind == "i64":
        return _signed128(int(out[0]), int(out[1]))
    if kind == "f64":
        return DD(out[0], out[1])
    return CDD(DD(out[0], out[1]), DD(out[2], out[3]))


def _outbuf(kind: str):
    if kind == "i64":
        return np.zeros(2, dtype=np.uint64)
    return np.zeros(2 if kind == "f64" else 4, dtype=np.float64)


def per_brute(a, nthreads: int = 0):
    """The definition, every injective map (Sec. 1.1).  Cost m * n!/(n-m)!."""
    a, kind = _prep(a)
    m, n = a.shape
    out = _outbuf(kind)
    fn = getattr(load(), f"oracle_brute_{kind}")
    _check(fn(m, n, a.ctypes.data, max(n, 1), nthreads, out.ctypes.data), "brute")
    return _decode(kind, out)


def per_laplace(a, nthreads: int = 0, form: int = 0):
    """Memoised Laplace expansion; ``form`` 1 = over column sets, 2 = over row
    sets, 0 = choose.  Memory 2^min-side entries (limit 2^30)."""
    a, kind = _prep(a)
    m, n = a.shape
    out = _outbuf(kind)
    fn = getattr(load(), f"oracle_laplace_{kind}")
    _check(fn(m, n, a.ctypes.data, max(n, 1), nthreads, form, out.ctypes.data), "laplace")
    return _decode(kind, out)


def per_glynn(a, nthreads: int = 0, k0: int = 0, k1: int = 0, partial: bool = False):
    """Eq. glynn / Eq. glynn_rectangle in double-double over the Gray indices
    [k0, k1) (k1 = 0: all 2^(n-1)).  ``partial`` returns the raw signed sum."""
    a, kind = _prep(a)
    if kind == "i64":
        a, kind = a.astype(np.float64), "f64"
    m, n = a.shape
    out = _outbuf(kind)
    fn = getattr(load(), f"oracle_glynn_{kind}")
    _check(fn(m, n, a.ctypes.data, max(n, 1), nthreads, k0, k1, int(partial),
              out.ctypes.data), "glynn")
    return _decode(kind, out)


def per_ryser(a, nthreads: int = 0):
    """Eq. ryser_square / Eq. ryser_rectangle in double-double, Gray order over
    all 2^n column subsets."""
    a, kind = _prep(a)
    if kind == "i64":
        a, kind = a.astype(np.float64), "f64"
    m, n = a.shape
    out = _outbuf(kind)
    fn = getattr(load(), f"oracle_ryser_{kind}")
    _check(fn(m, n, a.ctypes.data, max(n, 1), nthreads, out.ctypes.data), "ryser")
    return _decode(kind, out)
