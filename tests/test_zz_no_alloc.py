"""eri4_batch_coulomb_static (no device allocation, static scratch) against
eri4_batch_coulomb (caller's workspace), through the C ABI.

Both run the same kernels on the same quartets, so their J blocks must agree
bit for bit; the static call also runs its quartets in passes of a different
size than the workspace call, which must not change any quartet's result.
Two calls in a row, the second smaller, check that the scratch the first call
left behind does not leak into the second.
"""
import numpy as np
import pytest

from paper_2307_03452_amd import eri4, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a ROCm device"
    eri4.init()
    return _t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _both(torch, b, D, seed_out):
    d = lambda a: dev(torch, a)
    C, E, Co, N, Dd = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim), d(D)
    ref = eri4.batch_coulomb(b.ls, C, E, Co, N, Dd)
    shape = (b.nq, inputs.ncart(b.ls[0]), inputs.ncart(b.ls[1]))
    # the output starts as garbage: every element must be written
    out = torch.from_numpy(np.random.default_rng(seed_out).uniform(-1e3, 1e3, shape)).cuda()
    eri4.batch_coulomb_static(b.ls, C, E, Co, N, Dd, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_static_scratch_matches_workspace_call_twice(torch):
    assert eri4.static_scratch_bytes() == 32 << 20
    # first call: (ii|ii) K=5 per shell, 400 quartets -> more than one pass of
    # the 32 MiB scratch (92.8 KB of densities per quartet)
    b1 = inputs.class_batch((6, 6, 6, 6), 400, 5, seed=1401, exp_range=(0.05, 200.0))
    b1 = inputs.subset(b1, range(400))
    D1 = inputs.ket_densities(b1, seed=1402)
    ref1, got1 = _both(torch, b1, D1, 1403)
    assert np.isfinite(got1).all()
    assert np.array_equal(ref1, got1)
    # second call, smaller: (gg|hg) with mixed contraction lengths, 7 quartets
    b2 = inputs.class_batch((4, 4, 5, 4), 7, (1, 3), seed=1404, exp_range=(0.05, 200.0), kmax=3)
    D2 = inputs.ket_densities(b2, seed=1405)
    ref2, got2 = _both(torch, b2, D2, 1406)
    assert np.isfinite(got2).all()
    assert np.array_equal(ref2, got2)


def test_static_call_rejects_bad_arguments_without_enqueueing(torch):
    L = eri4.lib()
    b = inputs.class_batch((4, 4, 4, 4), 2, 1, seed=1407)
    d = lambda a: dev(torch, a)
    C, E, Co, N = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim)
    D = d(inputs.ket_densities(b, seed=1408))
    out = torch.zeros(2, 15, 15, dtype=torch.float64, device="cuda")
    p = lambda t: t.data_ptr()
    # l beyond the tables, a NULL buffer, kmax out of range
    assert L.eri4_batch_coulomb_static(8, 4, 4, 4, 2, p(C), p(E), p(Co), p(N), 1, p(D), p(out), None) == 2
    assert L.eri4_batch_coulomb_static(4, 4, 4, 4, 2, p(C), p(E), p(Co), p(N), 1, None, p(out), None) == 1
    assert L.eri4_batch_coulomb_static(4, 4, 4, 4, 2, p(C), p(E), p(Co), p(N), 0, p(D), p(out), None) == 1
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 0.0).all()
