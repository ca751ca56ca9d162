"""Coulomb contraction without forming (ab|cd) (eri4_batch_coulomb) against the
oracle: its Cartesian integrals contracted with the density, J_ab = sum_cd
(ab|cd) D_cd.  Tolerance: 1e-12 times the quartet's largest
sum_cd |(ab|cd)| |D_cd|, the scale the contraction rounds at."""
import numpy as np
import pytest

import oracle
from paper_2307_03452_amd import eri4, inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    eri4.init()
    return _t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(torch, b, D, work=None):
    out = eri4.batch_coulomb(b.ls, dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs),
                             dev(torch, b.nprim), dev(torch, D), work=work)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(g, I, D):
    ref = np.einsum("qabcd,qcd->qab", I, D)
    bound = np.einsum("qabcd,qcd->qab", np.abs(I), np.abs(D))
    assert g.shape == ref.shape
    for q in range(ref.shape[0]):
        scale = max(bound[q].max(), 1e-250)
        assert np.isfinite(g[q]).all(), q
        assert np.abs(g[q] - ref[q]).max() <= TOL * scale, (q, np.abs(g[q] - ref[q]).max() / scale)


@pytest.mark.parametrize("ls,K,nq", [((0, 0, 0, 0), 2, 5), ((1, 0, 2, 1), (1, 3), 6), ((2, 2, 2, 2), 2, 4),
                                     ((3, 1, 2, 3), 1, 4), ((4, 4, 4, 4), 1, 3), ((5, 4, 6, 3), 2, 2),
                                     ((6, 6, 6, 6), 1, 2), ((6, 6, 6, 6), 2, 1), ((7, 7, 7, 7), 1, 1),
                                     ((6, 7, 6, 7), 1, 1)])
def test_against_oracle(torch, ls, K, nq):
    b = inputs.class_batch(ls, nq, K, seed=500 + 3 * sum(ls) + (K if isinstance(K, int) else 9),
                           exp_range=(0.05, 200.0))
    D = inputs.ket_densities(b, seed=77)
    I = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
    check(run(torch, b, D), I, D)


def test_matches_contracting_the_librarys_own_integrals_at_full_size(torch):
    """(ii|ii), K=1, the 512-quartet benchmark batch: J from eri4_batch_coulomb
    equals the contraction of eri4_batch's integrals (checked against the
    oracle elsewhere) on every quartet."""
    b = inputs.iiii(K=1)
    D = inputs.ket_densities(b, seed=78)
    C, E, Co, N = dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs), dev(torch, b.nprim)
    g = eri4.batch_coulomb(b.ls, C, E, Co, N, dev(torch, D))
    I = eri4.batch(b.ls, C, E, Co, N)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    for q0 in range(0, b.nq, 64):
        check(g[q0:q0 + 64], I[q0:q0 + 64].cpu().numpy(), D[q0:q0 + 64])


def test_passes_through_a_small_workspace_give_the_same_result(torch):
    ls = (4, 5, 5, 4)
    b = inputs.class_batch(ls, 5, (1, 2), seed=551, exp_range=(0.05, 200.0))
    D = inputs.ket_densities(b, seed=79)
    one = run(torch, b, D)
    w = torch.empty(eri4.coulomb_work_size(ls, b.kmax, 2), dtype=torch.float64, device="cuda")
    assert np.array_equal(run(torch, b, D, work=w), one)


def test_bad_contraction_length_gives_nan_and_others_are_untouched(torch):
    ls = (2, 1, 2, 2)
    b = inputs.class_batch(ls, 3, 2, seed=552)
    D = inputs.ket_densities(b, seed=80)
    I = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
    bad = b.nprim.copy()
    bad[1, 3] = 0
    out = eri4.batch_coulomb(ls, dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs), dev(torch, bad),
                             dev(torch, D))
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    assert np.isnan(out[1]).all()
    check(out[[0, 2]], I[[0, 2]], D[[0, 2]])


def _list_densities(ket, seed):
    rng = np.random.default_rng(seed)
    return [rng.uniform(-1.0, 1.0, size=(inputs.ncart(int(ket.l[j, 0])), inputs.ncart(int(ket.l[j, 1]))))
            for j in range(ket.n)]


def test_coulomb_pair_plan_against_oracle(torch):
    """J_i = sum_j sum_cd (ab|cd)_ij D_j over a 4-entry bra list and a 5-entry
    ket list with l in {2, 3, 4} and contraction lengths 1..2."""
    bra = inputs.pair_list(4, 61, lvals=(2, 3, 4), kmax=2)
    ket = inputs.pair_list(5, 62, lvals=(2, 3, 4), kmax=2)
    Ds = _list_densities(ket, 63)
    p = eri4.CoulombPlan(bra.l, bra.nprim, ket.l, ket.nprim, 2)
    d = lambda a: dev(torch, a)
    kd = d(np.concatenate([x.ravel() for x in Ds]))
    args = (d(bra.centers), d(bra.exps), d(bra.coefs), d(ket.centers), d(ket.exps), d(ket.coefs), kd)
    g = p.execute(*args)
    g2 = p.execute(*args)
    torch.cuda.synchronize()
    g, g2 = g.cpu().numpy(), g2.cpu().numpy()
    assert np.array_equal(g, g2)  # fixed summation order
    off = p.offsets()
    b = inputs.expand_pairs(bra, ket)
    for i in range(bra.n):
        na, nb = inputs.ncart(int(bra.l[i, 0])), inputs.ncart(int(bra.l[i, 1]))
        ref = np.zeros((na, nb))
        bound = np.zeros((na, nb))
        for j in range(ket.n):
            q = i * ket.n + j
            s = inputs.subset(b, [q])
            I = oracle.eri_md4(tuple(int(x) for x in b.lq[q]), s.centers, s.exps, s.coefs, s.nprim)[0]
            ref += np.einsum("abcd,cd->ab", I, Ds[j])
            bound += np.einsum("abcd,cd->ab", np.abs(I), np.abs(Ds[j]))
        got = g[off[i]:off[i] + na * nb].reshape(na, nb)
        assert np.abs(got - ref).max() <= TOL * bound.max(), (i, np.abs(got - ref).max() / bound.max())


def test_coulomb_pair_plan_rejects_other_executes_and_small_workspaces(torch):
    bra, ket = inputs.pair_list(2, 64, kmax=1), inputs.pair_list(2, 65, kmax=1)
    p = eri4.CoulombPlan(bra.l, bra.nprim, ket.l, ket.nprim, 1)
    d = lambda a: dev(torch, a)
    kd = d(np.concatenate([x.ravel() for x in _list_densities(ket, 66)]))
    args = (d(bra.centers), d(bra.exps), d(bra.coefs), d(ket.centers), d(ket.exps), d(ket.coefs))
    with pytest.raises(eri4.Eri4Error, match="workspace"):
        p.execute(*args, kd, work=torch.empty(p.work_size - 1, dtype=torch.float64, device="cuda"))
    L = eri4.lib()
    out = torch.zeros(4096, dtype=torch.float64, device="cuda")
    ptr = lambda t: t.data_ptr()
    assert L.eri4_plan_execute_pairs(p._h, *(ptr(a) for a in args), None, 0, ptr(out), None) == 1
    assert b"Coulomb" in L.eri4_last_error()


def test_coulomb_pair_plan_with_an_empty_ket_list_gives_zeros(torch):
    """J_i over an empty ket list is an empty sum: execute zeroes the output
    (which starts as garbage here) instead of leaving it untouched."""
    bra = inputs.pair_list(3, 67, kmax=2)
    z = lambda *shape: torch.zeros(*shape, dtype=torch.float64, device="cuda")
    p = eri4.CoulombPlan(bra.l, bra.nprim, np.zeros((0, 2), np.int32), np.zeros((0, 2), np.int32), 2)
    assert p.output_size == sum(inputs.ncart(int(a)) * inputs.ncart(int(b)) for a, b in bra.l)
    out = torch.full((p.output_size,), float("nan"), dtype=torch.float64, device="cuda")
    d = lambda a: dev(torch, a)
    p.execute(d(bra.centers), d(bra.exps), d(bra.coefs), z(0, 2, 3), z(0, 2, 2), z(0, 2, 2), z(1), out=out)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 0.0).all()


def test_coulomb_wrappers_reject_short_buffers_and_bad_shapes(torch):
    b = inputs.class_batch((4, 4, 4, 4), 2, 1, seed=68)
    d = lambda a: dev(torch, a)
    C, E, Co, N = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim)
    D = d(inputs.ket_densities(b, seed=69))
    with pytest.raises(ValueError, match="density"):
        eri4.batch_coulomb(b.ls, C, E, Co, N, D[:1].contiguous())
    with pytest.raises(ValueError, match="output"):
        eri4.batch_coulomb(b.ls, C, E, Co, N, D, out=torch.empty(10, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="nprim"):
        eri4.batch_coulomb(b.ls, C, E, Co, N[:1].contiguous(), D)
    bra, ket = inputs.pair_list(2, 70, kmax=1), inputs.pair_list(2, 71, kmax=1)
    p = eri4.CoulombPlan(bra.l, bra.nprim, ket.l, ket.nprim, 1)
    args = (d(bra.centers), d(bra.exps), d(bra.coefs), d(ket.centers), d(ket.exps), d(ket.coefs))
    with pytest.raises(ValueError, match="ket density"):
        p.execute(*args, torch.zeros(3, dtype=torch.float64, device="cuda"))
    kd = torch.zeros(p.ket_dens_size, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="output"):
        p.execute(*args, kd, out=torch.zeros(p.output_size - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="pair lists"):
        p.execute(args[0][:1].contiguous(), *args[1:], kd)


def test_solid_batch_and_coulomb_plan_replay_in_a_hip_graph(torch):
    """eri4_batch_solid and a Coulomb pair-list plan captured in one HIP graph
    (no allocation, no memset nodes) give the eager results on every replay,
    with unrelated eager work between replays."""
    ls = (4, 4, 5, 4)
    b = inputs.class_batch(ls, 3, 2, seed=571, exp_range=(0.05, 200.0))
    C, E, Co, N = dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs), dev(torch, b.nprim)
    work = torch.empty(eri4.solid_work_size(ls, 2, 3), dtype=torch.float64, device="cuda")
    eager_s = eri4.batch_solid(ls, C, E, Co, N, work=work).clone()
    bra, ket = inputs.pair_list(3, 572, lvals=(2, 4), kmax=2), inputs.pair_list(3, 573, lvals=(3, 4), kmax=2)
    Ds = _list_densities(ket, 574)
    p = eri4.CoulombPlan(bra.l, bra.nprim, ket.l, ket.nprim, 2)
    d = lambda a: dev(torch, a)
    args = (d(bra.centers), d(bra.exps), d(bra.coefs), d(ket.centers), d(ket.exps), d(ket.coefs),
            d(np.concatenate([x.ravel() for x in Ds])))
    cwork = torch.empty(p.work_size, dtype=torch.float64, device="cuda")
    eager_c = p.execute(*args, work=cwork).clone()
    torch.cuda.synchronize()
    out_s = torch.zeros_like(eager_s)
    out_c = torch.zeros_like(eager_c)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        eri4.batch_solid(ls, C, E, Co, N, work=work, out=out_s, stream=s)
        p.execute(*args, out=out_c, work=cwork, stream=s)
    for rep in range(3):
        out_s.zero_()
        out_c.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_s, eager_s), rep
        assert torch.equal(out_c, eager_c), rep
        eri4.batch(ls, C[:1].contiguous(), E[:1].contiguous(), Co[:1].contiguous(), N[:1].contiguous())
        torch.cuda.synchronize()
