"""Algorithm selection: timing, the selector network's GPU primitives and its
training, over the C ABI of ``libpermgpu.so`` (argument marshalling only).

The network maps the features of a problem (log m, log n, density, dtype id;
see ``features``) to predicted log run times of five algorithms, in the order
of ``ALGO_ORDER``: combinatoric, Ryser, Glynn, the e_m form (rectangular
shapes), the column sweep.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _capi as C
from . import _DT, _OUT, _DEFAULT_OUT, _matrix, _stream, _ALGO_ID

NPARAMS = C.PERM_MLP_PARAMS
ALGO_ORDER = ("combinatoric", "ryser", "glynn", "glynn_esym", "column_sweep")
NOUT = len(ALGO_ORDER)
# perm_algo value of each network output
ALGO_IDS = (C.PERM_ALGO_COMBINATORIC, C.PERM_ALGO_RYSER, C.PERM_ALGO_GLYNN,
            C.PERM_ALGO_GLYNN_ESYM, C.PERM_ALGO_SWEEP)


def features(m: int, n: int, dtype: torch.dtype, density: float = -1.0) -> np.ndarray:
    """The selector's input features of a problem (float32[4])."""
    x = np.zeros(4, dtype=np.float32)
    C.check(C.lib.perm_selector_features(m, n, _DT[dtype], float(density), x.ctypes.data),
            "perm_selector_features")
    return x


def time(algo: str, a: torch.Tensor, fraction: float = 1.0, reps: int = 3,
         out: str | None = None, flags: int = 0) -> tuple[float, float]:
    """(median wall ms, fraction of the work run) of ``algo`` on the device
    matrix ``a`` with its main kernel cut to about ``fraction`` of its work.
    Raises PermError if the algorithm refuses the shape."""
    a, dt, lda = _matrix(a)
    kind = out or _DEFAULT_OUT[dt]
    m, n = a.shape
    ms, ran = ctypes.c_double(0.0), ctypes.c_double(0.0)
    with torch.cuda.device(a.device):
        C.check(C.lib.perm_time(_ALGO_ID[algo], m, n, dt, a.data_ptr(), lda, _OUT[kind], flags,
                                float(fraction), int(reps), _stream(a), ctypes.byref(ms),
                                ctypes.byref(ran)), "perm_time")
    return ms.value, ran.value


def _dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor on a HIP device")
    return t


def mlp_forward(params: torch.Tensor, norm: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Network outputs y[batch][NOUT] for features x[batch][4] (device float32)."""
    _dev(params, "params"), _dev(norm, "norm"), _dev(x, "x")
    y = torch.empty(x.shape[0], NOUT, dtype=torch.float32, device=x.device)
    C.check(C.lib.perm_mlp_forward(params.data_ptr(), norm.data_ptr(), x.data_ptr(),
                                   x.shape[0], y.data_ptr(), _stream(x)), "perm_mlp_forward")
    return y


def mlp_grad(params, norm, x, t, scale: float):
    """(gradient[NPARAMS], loss[1]) of scale * sum over finite t of (y - t)^2."""
    for v, nme in ((params, "params"), (norm, "norm"), (x, "x"), (t, "t")):
        _dev(v, nme)
    g = torch.empty(NPARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    C.check(C.lib.perm_mlp_grad(params.data_ptr(), norm.data_ptr(), x.data_ptr(), t.data_ptr(),
                                x.shape[0], float(scale), g.data_ptr(), loss.data_ptr(),
                                _stream(x)), "perm_mlp_grad")
    return g, loss


def mlp_adam(params, grad, state, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
             total_steps: int = 0) -> None:
    """One Adam step in place; ``state`` is float32[3 * NPARAMS], zero at first."""
    for v, nme in ((params, "params"), (grad, "grad")):
        _dev(v, nme)
    if state.numel() != 3 * NPARAMS or not state.is_contiguous():
        raise ValueError("state must hold 3 * NPARAMS contiguous 32-bit words")
    C.check(C.lib.perm_mlp_adam(params.data_ptr(), grad.data_ptr(), state.data_ptr(), float(lr),
                                float(beta1), float(beta2), float(eps), int(total_steps),
                                _stream(params)), "perm_mlp_adam")


def train(x: np.ndarray, t: np.ndarray, epochs: int, lr: float = 3e-3, seed: int = 1,
          params: np.ndarray | None = None):
    """Full-batch training on the GPU (perm_selector_train).  x: float32[N][4]
    features, t: float32[N][NOUT] log times (NaN = unavailable).  Starts from
    ``params`` if given, else from the seeded initialisation.  Returns
    (params, norm, loss history)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    if x.ndim != 2 or x.shape[1] != 4 or t.shape != (x.shape[0], NOUT):
        raise ValueError(f"x must be [N][4] and t [N][{NOUT}]")
    init = params is None
    p = np.zeros(NPARAMS, dtype=np.float32) if init else \
        np.array(params, dtype=np.float32, copy=True)
    norm = np.zeros(8, dtype=np.float32)
    hist = np.zeros(epochs, dtype=np.float32)
    C.check(C.lib.perm_selector_train(x.shape[0], x.ctypes.data, t.ctypes.data, int(epochs),
                                      float(lr), int(seed), 1 if init else 0, p.ctypes.data,
                                      norm.ctypes.data, hist.ctypes.data,
                                      torch.cuda.current_stream().cuda_stream),
            "perm_selector_train")
    return p, norm, hist


def save(path: str, params: np.ndarray, norm: np.ndarray, table=None) -> None:
    """Write a weights file for ``selector_load`` (table = p1..p8 or None)."""
    p = np.ascontiguousarray(params, dtype=np.float32)
    nm = np.ascontiguousarray(norm, dtype=np.float32)
    tb = None if table is None else np.ascontiguousarray(table, dtype=np.float64)
    if p.size != NPARAMS or nm.size != 8 or (tb is not None and tb.size != 8):
        raise ValueError("params must have NPARAMS entries, norm 8, table 8")
    C.check(C.lib.perm_selector_save(path.encode(), p.ctypes.data, nm.ctypes.data,
                                     None if tb is None else tb.ctypes.data),
            "perm_selector_save")


def log_ms(ms: float) -> float:
    """The network's target scale: natural log of milliseconds."""
    return math.log(ms)
