"""Plans with FP32 transforms (ERI4_PREC_FP32) against the oracle and against
the FP64 path.

The FP32 transforms round both matrix operands to FP32 (unit roundoff
u = 2^-24) and accumulate in FP32, so the error of an integral is bounded by a
few u times the sum of the magnitudes of the terms it adds, not by the integral
itself.  The check here allows TOL32 = 2e-5 (about 340 u) of each quartet's
largest integral: room for the length of the sums and for the cancellation
between terms that the FP64 results show on these inputs.  This is a bound on
FP32 arithmetic, not the 1e-10 absolute target of a mixed-precision scheme
that recovers FP64 accuracy; the benchmark reports how far FP32 is from it.
"""
import numpy as np
import pytest

import oracle
from paper_2307_03452_amd import eri4, inputs

pytestmark = pytest.mark.gpu
TOL32 = 2e-5
ZERO_SCALE = 1e-250


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    eri4.init()
    return _t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(torch, b, precision):
    p = eri4.Plan(b.lq, b.nprim, b.kmax, precision=precision)
    out = p.execute(dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs))
    torch.cuda.synchronize()
    return p, out.cpu().numpy()


def single_class(b):
    """A one-class batch as a plan input (per-quartet l array)."""
    b.lq = np.tile(np.array(b.ls, np.int32), (b.nq, 1))
    return b


def check_oracle(b, off, g_flat, idx):
    by_cls = {}
    for q in idx:
        by_cls.setdefault(tuple(int(x) for x in b.lq[q]), []).append(q)
    worst = 0.0
    for ls, qs in by_cls.items():
        s = inputs.subset(b, qs)
        o = oracle.eri_md4(ls, s.centers, s.exps, s.coefs, s.nprim)
        for i, q in enumerate(qs):
            g = g_flat[off[q]:off[q] + o[i].size].reshape(o[i].shape)
            scale = max(np.abs(o[i]).max(), ZERO_SCALE)
            assert np.isfinite(g).all(), q
            rel = np.abs(g - o[i]).max() / scale
            assert rel <= TOL32, (q, ls, rel, scale)
            worst = max(worst, rel)
    return worst


def test_fp32_plan_low_l_against_oracle(torch):
    b = inputs.uneven_batch(nq=80, seed=31, lvals=(0, 1, 2, 3), kmax=3)
    p, g = run(torch, b, "fp32")
    worst = check_oracle(b, p.offsets(), g, range(b.nq))
    assert worst > 0.0  # FP32 arithmetic is in use (not bitwise the FP64 result)


def test_fp32_plan_high_l_contracted_against_oracle(torch):
    b = inputs.uneven_batch(nq=24, seed=32, lvals=(4, 5, 6), kmax=2)
    p, g = run(torch, b, "fp32")
    check_oracle(b, p.offsets(), g, range(b.nq))


def test_fp32_plan_l7_against_oracle(torch):
    b = single_class(inputs.class_batch((7, 6, 7, 5), 4, 1, seed=33, exp_range=(0.05, 200.0)))
    p, g = run(torch, b, "fp32")
    check_oracle(b, p.offsets(), g, range(b.nq))


def test_fp32_plan_iiii_k1_against_fp64_path(torch):
    """Every quartet of the (ii|ii) K=1 workload: FP32 transforms against the
    FP64 plan (which matches the oracle to 1e-12), component by component."""
    b = single_class(inputs.iiii(1, nq=512))
    p64, g64 = run(torch, b, "fp64")
    p32, g32 = run(torch, b, "fp32")
    assert np.array_equal(p64.offsets(), p32.offsets())
    ref = g64.reshape(b.nq, -1)
    d = np.abs(g32.reshape(b.nq, -1) - ref).max(axis=1)
    scale = np.maximum(np.abs(ref).max(axis=1), ZERO_SCALE)
    bad = np.flatnonzero(d > TOL32 * scale)
    assert bad.size == 0, [(int(q), float(d[q] / scale[q]), float(scale[q])) for q in bad[:5]]


def test_fp32_plan_is_deterministic(torch):
    b = inputs.uneven_batch(nq=40, seed=34, lvals=(4, 5), kmax=3)
    _, g1 = run(torch, b, "fp32")
    _, g2 = run(torch, b, "fp32")
    assert np.array_equal(g1, g2)
