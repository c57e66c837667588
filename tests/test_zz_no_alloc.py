"""perm_glynn_noalloc (scratch in a fixed device array, no allocation in the
call) against perm_glynn through the C ABI: the same kernels and plan, so the
results must agree bitwise, and both meet the accuracy criterion against the
oracle.  Two calls in a row, the second on a smaller input, check that the
array's leftover contents from the first call do not leak into the second."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


def _call(fn, a, out_kind):
    import torch

    from paper_2510_03421_amd import _capi as C
    t = dev(a)
    m, n = a.shape
    dt = {np.dtype(np.float64): C.PERM_F64, np.dtype(np.complex128): C.PERM_C128,
          np.dtype(np.uint8): C.PERM_B8, np.dtype(np.int64): C.PERM_I64}[a.dtype]
    ot = {"f64": C.PERM_OUT_F64, "dd": C.PERM_OUT_DD, "c128": C.PERM_OUT_C128,
          "cdd": C.PERM_OUT_CDD, "i128": C.PERM_OUT_I128}[out_kind]
    words = {"f64": 1, "dd": 2, "c128": 2, "cdd": 4, "i128": 2}[out_kind]
    out = torch.full((words,), float("nan"), dtype=torch.float64, device="cuda")
    rc = fn(m, n, dt, t.data_ptr(), n, ot, out.data_ptr(), 0,
            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return rc, out.cpu().numpy()


def _both(a, out_kind):
    from paper_2510_03421_amd import _capi as C
    rc1, want = _call(C.lib.perm_glynn, a, out_kind)
    rc2, got = _call(C.lib.perm_glynn_noalloc, a, out_kind)
    assert rc1 == 0 and rc2 == 0, (rc1, rc2)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (got, want)
    return got


@pytest.mark.parametrize("shapes", [[(20, 20), (12, 12)], [(24, 24), (6, 9)], [(10, 30), (3, 3)]])
def test_matches_perm_glynn_on_two_calls(shapes):
    for k, (m, n) in enumerate(shapes):
        a = workloads.uniform(m, n, 12000 + 100 * k + m + n)
        got = _both(a, "dd")
        ref = oracle.per_laplace(a)
        pabs = oracle.per_laplace(np.abs(a))
        assert abs((got[0] + got[1]) - (ref.hi + ref.lo)) <= 1e-11 * pabs.hi
        z = workloads.complex_gauss(m, n, 12500 + 100 * k + m + n)
        gz = _both(z, "cdd")
        rz = oracle.per_laplace(z)
        pz = oracle.per_laplace(np.abs(z))
        err = abs(complex(gz[0] + gz[1], gz[2] + gz[3]) -
                  complex(rz.re.hi + rz.re.lo, rz.im.hi + rz.im.lo))
        assert err <= 1e-11 * pz.hi


def test_headline_size_then_smaller():
    """The 32 x 32 workload (the largest scratch of the test), then a 5 x 5."""
    big = workloads.config_matrix("u32")
    _both(big, "dd")
    small = workloads.uniform(5, 5, 12901)
    got = _both(small, "f64")
    assert abs(got[0] - float(oracle.per_brute(small))) <= 1e-11 * float(oracle.per_brute(np.abs(small)))


def test_refusals_and_empty_matrix():
    from paper_2510_03421_amd import _capi as C
    # integer outputs need the allocating pre-check
    rc, _ = _call(C.lib.perm_glynn_noalloc, np.ones((4, 4), dtype=np.uint8), "i128")
    assert rc == C.PERM_E_UNSUPPORTED
    # above the size limit of every path
    rc, _ = _call(C.lib.perm_glynn_noalloc, np.ones((2, 65)), "f64")
    assert rc == C.PERM_E_TOO_LARGE
    rc, out = _call(C.lib.perm_glynn_noalloc, np.zeros((0, 3)), "f64")
    assert rc == 0 and out[0] == 1.0
