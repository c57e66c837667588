"""Error paths of the C ABI on the host: argument errors are reported before
any device call (on any machine), and on a machine without a GPU every entry
point fails with PERM_E_HIP; in both cases the output is left untouched."""
import ctypes

import numpy as np
import pytest

from paper_2510_03421_amd import _capi as C


def no_device():
    import torch
    return torch.cuda.device_count() == 0


ENTRY = ("perm_glynn", "perm_ryser", "perm_combinatoric", "perm_glynn_esym", "perm_column_sweep",
         "perm_glynn_noalloc")


def call(name, m, n, dt, a, lda, ot, out, flags=0):
    return getattr(C.lib, name)(m, n, dt, a, lda, ot, out, flags, None)


@pytest.mark.parametrize("name", ENTRY)
def test_argument_errors_write_nothing(name):
    a = np.ones((4, 4))
    out = np.full(4, 7.0)
    p, o = a.ctypes.data, out.ctypes.data
    cases = [
        (4, 4, C.PERM_F64, None, 4, C.PERM_OUT_F64, o),        # null input
        (4, 4, C.PERM_F64, p, 3, C.PERM_OUT_F64, o),           # lda < n
        (4, 4, C.PERM_F64, p, 4, C.PERM_OUT_F64, None),        # null output
        (-1, 4, C.PERM_F64, p, 4, C.PERM_OUT_F64, o),          # negative size
        (4, 4, 9, p, 4, C.PERM_OUT_F64, o),                    # unknown input type
        (4, 4, C.PERM_F64, p, 4, 17, o),                       # unknown output type
        (4, 4, C.PERM_F64, p, 4, C.PERM_OUT_I128, o),          # integer output of real input
        (4, 4, C.PERM_C128, p, 4, C.PERM_OUT_F64, o),          # real output of complex input
    ]
    for m, n, dt, ptr, lda, ot, optr in cases:
        assert call(name, m, n, dt, ptr, lda, ot, optr) == C.PERM_E_INVALID, (m, n, dt, lda, ot)
    assert np.all(out == 7.0)


@pytest.mark.skipif(not no_device(), reason="runs the calls on host buffers: only without a GPU")
def test_without_a_device_every_entry_point_fails_cleanly():
    a = np.ones((4, 6))
    b = np.ones((4, 6), dtype=np.uint8)
    out = np.full(4, 7.0)
    o = out.ctypes.data
    for name in ENTRY:
        assert call(name, 4, 6, C.PERM_F64, a.ctypes.data, 6, C.PERM_OUT_F64, o) == C.PERM_E_HIP
        # the allocation-free variant serves floating-point outputs only
        want = C.PERM_E_UNSUPPORTED if name == "perm_glynn_noalloc" else C.PERM_E_HIP
        assert call(name, 4, 6, C.PERM_B8, b.ctypes.data, 6, C.PERM_OUT_I128, o) == want
    ch = ctypes.c_int(-1)
    assert C.lib.perm_auto(4, 6, C.PERM_F64, a.ctypes.data, 6, C.PERM_OUT_F64, o, 0, None, -1.0,
                           ctypes.byref(ch)) == C.PERM_E_HIP
    assert ch.value == -1
    h = ctypes.c_void_p()
    m, n = np.array([3], np.int32), np.array([3], np.int32)
    off, ld = np.zeros(1, np.int64), np.array([3], np.int64)
    assert C.lib.perm_batch_plan_create(1, m.ctypes.data, n.ctypes.data, off.ctypes.data,
                                        ld.ctypes.data, C.PERM_F64, C.PERM_OUT_F64,
                                        C.PERM_ALGO_GLYNN, 0, ctypes.byref(h)) == C.PERM_E_HIP
    assert h.value is None
    assert C.lib.perm_workspace_release() == C.PERM_E_HIP
    assert np.all(out == 7.0)
    # an empty matrix still needs the device (the value 1 is written there)
    assert call("perm_glynn", 0, 5, C.PERM_F64, None, 5, C.PERM_OUT_F64, o) == C.PERM_E_HIP
    assert np.all(out == 7.0)
