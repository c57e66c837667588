"""Batched Glynn (one plan, per-order persistent kernels, one graph launch)
against the CPU oracle and against the single-matrix path."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import golden, ref_value

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def pack(mats, dtype):
    """Pack a list of 2-D arrays into one buffer (row-major, ld = n)."""
    m = np.array([a.shape[0] for a in mats], dtype=np.int32)
    n = np.array([a.shape[1] for a in mats], dtype=np.int32)
    off = np.zeros(len(mats), dtype=np.int64)
    tot = 0
    for i, a in enumerate(mats):
        off[i] = tot
        tot += a.size
    data = np.zeros(max(tot, 1), dtype=dtype)
    for i, a in enumerate(mats):
        data[off[i]:off[i] + a.size] = a.reshape(-1)
    return data, m, n, off, n.astype(np.int64)


def to_values(out, kind, count):
    v = out.cpu().numpy()
    if kind == "f64":
        return v
    if kind == "c128":
        return v[0::2] + 1j * v[1::2]
    if kind == "dd":
        return v[0::2] + v[1::2]
    return (v[0::4] + v[1::4]) + 1j * (v[2::4] + v[3::4])


@pytest.mark.parametrize("cplx", [False, True])
def test_random_shapes_against_oracle(cplx):
    import torch

    import paper_2510_03421_amd as pg
    rng = np.random.default_rng(11 + cplx)
    mats = []
    for k in range(60):
        n = int(rng.integers(1, 10))
        m = int(rng.integers(0, n + 1)) if k % 3 == 0 else n   # some rectangular, some m = 0
        mats.append(workloads.complex_gauss(m, n, 500 + k) if cplx else
                    workloads.uniform(m, n, 500 + k))
    dt = np.complex128 if cplx else np.float64
    data, m, n, off, ld = pack(mats, dt)
    t = torch.from_numpy(data).cuda()
    plan = pg.BatchPlan(m, n, off, ld, t.dtype, out="cdd" if cplx else "dd")
    out = plan.new_output()
    plan.run(t, out)
    got = to_values(out, plan.kind, len(mats))
    for i, a in enumerate(mats):
        ref = complex(oracle.per_brute(a)) if a.shape[0] else 1.0
        scale = float(oracle.per_brute(np.abs(a))) if a.shape[0] else 1.0
        # rectangular matrices go through the e_m form (padding summed out)
        assert abs(got[i] - ref) <= 1e-11 * scale + 1e-300, (i, a.shape, got[i], ref)
    plan.close()


def test_graph_replays_are_identical_and_match_single_calls():
    import torch

    import paper_2510_03421_amd as pg
    b = workloads.boson_batch(600, 4, 16, N=32, seed_u=77, seed_idx=78)
    t = torch.from_numpy(b.data).cuda()
    plan = pg.BatchPlan(b.m, b.n, b.offset, b.ld, t.dtype, out="c128")
    out = plan.new_output()
    plan.run(t, out)
    torch.cuda.synchronize()
    first = out.clone()
    for r in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        out.zero_()
        plan.run(t, out)
        torch.cuda.synchronize()
        assert torch.equal(out, first), r
        del junk
    vals = to_values(first, "c128", b.count)
    for i in range(0, b.count, 7):
        single = pg.glynn(torch.from_numpy(np.ascontiguousarray(b.matrix(i))).cuda()).value()
        assert abs(vals[i] - single) <= 1e-12 * (1 + abs(single))
        assert abs(vals[i]) <= 1 + 1e-9          # submatrix of a unitary: |per| <= 1
    plan.close()


def test_boson_sample_against_oracle():
    import torch

    import paper_2510_03421_amd as pg
    b = workloads.boson_batch(300, 4, 12, N=64, seed_u=6400, seed_idx=6401)
    t = torch.from_numpy(b.data).cuda()
    out = pg.glynn_batched(t, b.m, b.n, b.offset, b.ld, out="cdd")
    vals = to_values(out, "cdd", b.count)
    for i in range(0, b.count, 3):
        a = b.matrix(i)
        ref = complex(oracle.per_laplace(np.ascontiguousarray(a)))
        scale = float(oracle.per_laplace(np.abs(a)))
        assert abs(vals[i] - ref) <= 1e-13 * scale + 1e-300, (i, vals[i], ref)


@pytest.mark.parametrize("cplx", [False, True])
def test_packed_orders_strided_rectangular_and_partial_waves(cplx):
    """Orders 10..14 (several matrices per wave): 5 matrices of each order, so
    the last wave of every order is partly empty; rows m < n padded with ones;
    every matrix stored with a leading dimension n + 3 inside one buffer."""
    import torch

    import paper_2510_03421_amd as pg
    mats, ms, ns, offs, lds = [], [], [], [], []
    buf = []
    off = 0
    for n in range(10, 15):
        for k, m in enumerate((n, n - 2, 1, n, n - 5)):
            a = (workloads.complex_gauss(m, n, 3000 + 10 * n + k) if cplx else
                 workloads.uniform(m, n, 3000 + 10 * n + k))
            ld = n + 3
            block = np.zeros((m, ld), dtype=a.dtype)
            block[:, :n] = a
            mats.append(a)
            ms.append(m); ns.append(n); offs.append(off); lds.append(ld)
            buf.append(block.reshape(-1))
            off += block.size
    data = np.concatenate(buf)
    t = torch.from_numpy(data).cuda()
    plan = pg.BatchPlan(np.array(ms, np.int32), np.array(ns, np.int32), np.array(offs, np.int64),
                        np.array(lds, np.int64), t.dtype, out="cdd" if cplx else "dd")
    out = plan.new_output()
    plan.run(t, out)
    got = to_values(out, plan.kind, len(mats))
    for i, a in enumerate(mats):
        ref = complex(oracle.per_laplace(a))
        scale = float(oracle.per_laplace(np.abs(a)))
        # rectangular ones go through the e_m form
        assert abs(got[i] - ref) <= 1e-11 * scale, (i, a.shape, got[i], ref)
    plan.close()


@pytest.mark.parametrize("cplx", [False, True])
def test_autotuned_packing(cplx):
    """PERM_BATCH_AUTOTUNE: every small order gets an admissible matrices-per-
    wave count, the values agree with the oracle and with the rule-packed plan,
    and later runs replay the tuned graph bitwise."""
    import torch

    import paper_2510_03421_amd as pg
    C = 2 if cplx else 1
    mats = []
    for n in list(range(2, 15)) + [16, 18]:
        for k in range(9):
            mats.append(workloads.complex_gauss(n, n, 7000 + 20 * n + k) if cplx else
                        workloads.uniform(n, n, 7000 + 20 * n + k))
    data, m, n, off, ld = pack(mats, np.complex128 if cplx else np.float64)
    t = torch.from_numpy(data).cuda()
    kind = "cdd" if cplx else "dd"
    tuned = pg.BatchPlan(m, n, off, ld, t.dtype, out=kind, autotune=True)
    rule = pg.BatchPlan(m, n, off, ld, t.dtype, out=kind)
    out_t, out_r = tuned.new_output(), rule.new_output()
    tuned.run(t, out_t)
    rule.run(t, out_r)
    got_t = to_values(out_t, kind, len(mats))
    got_r = to_values(out_r, kind, len(mats))
    for order in range(2, 15):
        P = tuned.packing(order)
        assert P >= 1 and P & (P - 1) == 0 and 64 // P <= 2 ** (order - 1), (order, P)
        assert P * (order * order + order) * C * 8 <= 32768, (order, P)
        assert rule.packing(order) >= 1
    assert tuned.packing(16) == 0 and tuned.packing(18) == 0 and tuned.packing(15) == 0
    for i, a in enumerate(mats):
        ref = complex(oracle.per_laplace(a))
        scale = float(oracle.per_laplace(np.abs(a)))
        assert abs(got_t[i] - ref) <= 1e-11 * scale, (i, a.shape, got_t[i], ref)
        assert abs(got_t[i] - got_r[i]) <= 1e-12 * scale, (i, a.shape)
    first = out_t.clone()
    tuned.run(t, out_t)
    torch.cuda.synchronize()
    assert torch.equal(first, out_t)
    tuned.close()
    rule.close()


@pytest.mark.parametrize("cplx", [False, True])
def test_wide_rectangular_batches_e_m_and_ones_padding(cplx):
    """Rectangular matrices with m << n (n >= 15): the batch evaluates them by
    the e_m form (the padding rows summed out), which meets the 1e-11 per(|A|)
    criterion at every shape and keeps far more digits than the printed rows
    of ones (PERM_FLAG_PAD_ONES, as accurate as a single padded call)."""
    import torch

    import paper_2510_03421_amd as pg
    from paper_2510_03421_amd import _capi as C
    shapes = [(3, 20), (5, 24), (2, 26), (8, 28), (6, 16), (16, 16), (4, 32)]
    mats = [(workloads.complex_gauss(m, n, 7500 + n) if cplx else workloads.uniform(m, n, 7500 + n))
            for m, n in shapes]
    data, m, n, off, ld = pack(mats, np.complex128 if cplx else np.float64)
    t = torch.from_numpy(data).cuda()
    kind = "cdd" if cplx else "dd"
    plan = pg.BatchPlan(m, n, off, ld, t.dtype, out=kind)
    ones = pg.BatchPlan(m, n, off, ld, t.dtype, out=kind, flags=C.PERM_FLAG_PAD_ONES)
    out, out1 = plan.new_output(), ones.new_output()
    plan.run(t, out)
    ones.run(t, out1)
    got, got1 = to_values(out, kind, len(mats)), to_values(out1, kind, len(mats))

    def single(fn, a, flags):
        v = fn(torch.from_numpy(a).cuda(), out=kind, flags=flags).value()
        return complex(v[0] + v[1]) if not cplx else complex(v[0][0] + v[0][1], v[1][0] + v[1][1])

    rel_s, rel_1 = [], []
    for i, a in enumerate(mats):
        ref = complex(oracle.per_laplace(a))
        pabs = float(oracle.per_laplace(np.abs(a)))
        e_s, e_1 = abs(got[i] - ref), abs(got1[i] - ref)
        assert e_s <= 1e-11 * pabs, (a.shape, got[i], ref)            # every shape
        assert e_s <= 1e-12 * abs(ref), (a.shape, e_s / abs(ref))
        if a.shape[0] < a.shape[1]:
            # the same e_m sum as a single perm_glynn_esym call
            assert e_s <= 10 * abs(single(pg.glynn_esym, a, 0) - ref) + 1e-13 * abs(ref)
        # rows of ones: as accurate as a single padded call
        assert e_1 <= 10 * abs(single(pg.glynn, a, C.PERM_FLAG_PAD_ONES) - ref) + 1e-13 * pabs
        if a.shape[0] < a.shape[1]:
            rel_s.append(e_s / abs(ref))
            rel_1.append(e_1 / abs(ref))
    assert max(rel_s) < 1e-12 and sum(rel_s) < 1e-3 * sum(rel_1), (rel_s, rel_1)
    plan.close()
    ones.close()


def test_large_orders_use_many_chunks():
    import torch

    import paper_2510_03421_amd as pg
    # up to the batched limit n = 32; the last matrix is the 32 x 32 workload
    mats = [workloads.uniform(n, n, 900 + n) for n in (17, 20, 22, 24, 28)]
    mats.append(workloads.config_matrix("u32"))
    data, m, n, off, ld = pack(mats, np.float64)
    t = torch.from_numpy(data).cuda()
    plan = pg.BatchPlan(m, n, off, ld, t.dtype, out="dd")
    out = plan.new_output()
    plan.run(t, out)
    got = to_values(out, "dd", len(mats))
    for i, a in enumerate(mats):
        single = pg.glynn(torch.from_numpy(a).cuda(), out="dd").value()
        assert abs(got[i] - (single[0] + single[1])) <= 1e-12 * abs(single[0])
    rec = golden()["u32"]
    assert abs(got[-1] - ref_value(rec)) <= 1e-11 * abs(ref_value(rec))
    plan.close()


def test_empty_batch_and_errors():
    import torch

    import paper_2510_03421_amd as pg
    e = np.zeros(0, dtype=np.int32)
    plan = pg.BatchPlan(e, e, e.astype(np.int64), e.astype(np.int64), torch.float64)
    out = plan.new_output()
    plan.run(torch.zeros(1, dtype=torch.float64, device="cuda"), out)
    plan.close()
    one = np.array([3], dtype=np.int32)
    with pytest.raises(pg.PermError) as ex:        # m > n
        pg.BatchPlan(np.array([4], np.int32), one, np.zeros(1, np.int64), np.array([4]),
                     torch.float64)
    assert ex.value.status == -5
    with pytest.raises(pg.PermError) as ex:        # n > 32
        pg.BatchPlan(np.array([33], np.int32), np.array([33], np.int32), np.zeros(1, np.int64),
                     np.array([33]), torch.float64)
    assert ex.value.status == -2
    with pytest.raises(pg.PermError) as ex:        # Ryser batches take square matrices
        pg.BatchPlan(np.array([2], np.int32), one, np.zeros(1, np.int64), np.array([3]),
                     torch.int64, algo="ryser")
    assert ex.value.status == -5
    with pytest.raises(pg.PermError) as ex:        # a flag batches do not take
        pg.BatchPlan(one, one, np.zeros(1, np.int64), np.array([3]), torch.float64, flags=0x8)
    assert ex.value.status == -1
    with pytest.raises(pg.PermError) as ex:        # no batched definition
        pg.BatchPlan(one, one, np.zeros(1, np.int64), np.array([3]), torch.float64,
                     algo="combinatoric")
    assert ex.value.status == -5
