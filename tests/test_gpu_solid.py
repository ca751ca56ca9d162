"""Solid-harmonic output (eri4_batch_solid) against the oracle: its Cartesian
integrals transformed by its own coefficient table.

Tolerance: TOL times the quartet's largest sum_k |C x C x C x C|[m, k] |cart[k]|
(cart: its Cartesian integrals), with TOL = 1e-12 for classes whose shells all
have l <= 3 and 1e-14 above.  For l <= 3 the scale is close to the Cartesian
maximum, so the bar is the Cartesian parity bar (1e-12 of the block's largest
integral): what shows there is both FP64 codes' own rounding of the Cartesian
integrals, measured up to 2.4e-14 on single-class batches and 1.04e-13 on one
(ss|pp) quartet of a mixed plan batch with contraction lengths up to 3 (for
l <= 1 the transform is a scaling of the Cartesian integrals, so that error is
the Cartesian one).  For l >= 4 the measured worst is 1.4e-16 (the scale is
far above the integrals' size), a factor 70 below the bar.  Solid functions of distant shells have no low
multipoles, so their integrals can be orders of magnitude (4e7 seen here)
below the Cartesian ones they combine, and the coefficients grow with l (row
1-norms up to 47 for l = 6); every FP64 route through Hermite or Cartesian
intermediates (the oracle's as well as the library's) rounds at that scale,
which is the forward error bound of the transform divided by the unit
roundoff.  At l <= 1 it is the Cartesian maximum."""
import numpy as np
import pytest

import oracle
from oracle import solid
from paper_2307_03452_amd import eri4, inputs

pytestmark = pytest.mark.gpu
ZERO_SCALE = 1e-250


def tol(ls):
    return 1e-12 if max(ls) <= 3 else 1e-14


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    eri4.init()
    return _t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(torch, b, work=None):
    out = eri4.batch_solid(b.ls, dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs),
                           dev(torch, b.nprim), work=work)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_solid(b):
    """(solid integrals, Cartesian integrals) of the oracle (scalar MD)."""
    cart = oracle.eri_md4(b.ls, b.centers, b.exps, b.coefs, b.nprim)
    return solid.cart_to_solid(cart, b.ls), cart


def check(g, ref, cart, ls):
    assert g.shape == ref.shape
    bound = solid.cart_to_solid(np.abs(cart), ls, absolute=True)
    for q in range(ref.shape[0]):
        scale = max(bound[q].max(), ZERO_SCALE)
        assert np.isfinite(g[q]).all(), q
        assert np.abs(g[q] - ref[q]).max() <= tol(ls) * scale, (q, np.abs(g[q] - ref[q]).max() / scale)


LOW = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 0, 1, 1), (2, 1, 0, 2), (1, 2, 2, 1), (2, 2, 2, 2), (3, 0, 2, 1),
       (3, 3, 2, 2), (1, 3, 3, 3), (3, 3, 3, 3)]


@pytest.mark.parametrize("ls", LOW)
def test_low_l_classes_against_oracle(torch, ls):
    b = inputs.class_batch(ls, 9, (1, 3), seed=300 + sum(ls) * 7 + ls[0], exp_range=(0.05, 50.0))
    check(run(torch, b), *oracle_solid(b), b.ls)


@pytest.mark.parametrize("ls,K,nq", [((4, 4, 4, 4), 1, 3), ((5, 4, 4, 5), 2, 2), ((4, 6, 5, 4), 1, 2),
                                     ((6, 6, 6, 6), 1, 2), ((6, 6, 6, 6), 2, 1), ((7, 7, 7, 7), 1, 1),
                                     ((6, 7, 6, 7), 1, 1)])
def test_high_l_classes_against_oracle(torch, ls, K, nq):
    b = inputs.class_batch(ls, nq, K, seed=400 + 3 * sum(ls) + K, exp_range=(0.05, 200.0))
    check(run(torch, b), *oracle_solid(b), b.ls)


def test_passes_through_a_small_workspace_give_the_same_integrals(torch):
    """A workspace holding 2 quartets runs 7 quartets in 4 passes, bit for bit
    as one pass."""
    ls = (4, 5, 4, 4)
    b = inputs.class_batch(ls, 7, (1, 2), seed=451, exp_range=(0.05, 200.0))
    one = run(torch, b)
    w = torch.empty(eri4.solid_work_size(ls, b.kmax, 2) + 5, dtype=torch.float64, device="cuda")
    assert np.array_equal(run(torch, b, work=w), one)


def test_solid_equals_transformed_cartesian_at_full_size(torch):
    """(ii|ii), K=1, 512 quartets (the benchmark batch): the solid integrals
    equal the oracle's transform of the library's Cartesian integrals on every
    quartet (a property at any size; the Cartesian path is checked against the
    oracle elsewhere)."""
    b = inputs.iiii(K=1)
    C, E, Co, N = dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs), dev(torch, b.nprim)
    g = eri4.batch_solid(b.ls, C, E, Co, N)
    cart = eri4.batch(b.ls, C, E, Co, N)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    cart = cart.cpu().numpy()
    for q0 in range(0, b.nq, 64):
        check(g[q0:q0 + 64], solid.cart_to_solid(cart[q0:q0 + 64], b.ls), cart[q0:q0 + 64], b.ls)


def test_bad_contraction_length_gives_nan_and_others_are_untouched(torch):
    ls = (2, 2, 1, 1)
    b = inputs.class_batch(ls, 4, 2, seed=452)
    ref, cart = oracle_solid(b)
    bad = b.nprim.copy()
    bad[2, 1] = 3  # above kmax = 2
    out = eri4.batch_solid(ls, dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs), dev(torch, bad))
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    assert np.isnan(out[2]).all()
    check(out[[0, 1, 3]], ref[[0, 1, 3]], cart[[0, 1, 3]], ls)


def plan_blocks(torch, b, plan=None, work=None):
    """Run b through a solid quartet plan; the blocks per quartet (host)."""
    p = plan or eri4.SolidPlan(b.lq, b.nprim, b.kmax)
    out = p.execute(dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs), work=work)
    torch.cuda.synchronize()
    flat = out.cpu().numpy()
    off = p.offsets()
    blocks = []
    for q in range(b.nq):
        s = [2 * int(x) + 1 for x in b.lq[q]]
        blocks.append(flat[off[q]:off[q] + int(np.prod(s))].reshape(s))
    return blocks


def check_plan(torch, b, blocks):
    """Each quartet's block against the oracle's transform of its Cartesian
    integrals, quartets grouped by class."""
    by_cls = {}
    for q in range(b.nq):
        by_cls.setdefault(tuple(int(x) for x in b.lq[q]), []).append(q)
    for ls, qs in by_cls.items():
        s = inputs.subset(b, qs)
        s = inputs.Batch(ls, s.centers, s.exps, s.coefs, s.nprim, s.lq)
        ref, cart = oracle_solid(s)
        check(np.stack([blocks[q] for q in qs]), ref, cart, ls)


def test_solid_plan_low_l_mixed_against_oracle(torch):
    """Quartet plan over solid harmonics: 60 quartets of classes in {0..3}^4
    with contraction lengths 1..3 per shell, one persistent launch."""
    b = inputs.uneven_batch(nq=60, seed=461, lvals=(0, 1, 2, 3), kmax=3, exp_range=(0.05, 50.0))
    check_plan(torch, b, plan_blocks(torch, b))


def test_solid_plan_high_l_mixed_against_oracle(torch):
    """12 quartets of classes in {4,5,6}^4 plus one (77|77), lengths 1..2 per
    shell."""
    b = inputs.uneven_batch(nq=12, seed=462, lvals=(4, 5, 6), kmax=2)
    k = inputs.class_batch((7, 7, 7, 7), 1, 1, seed=463, exp_range=(0.05, 200.0), kmax=2)
    b = inputs.Batch(None, np.concatenate([b.centers, k.centers]), np.concatenate([b.exps, k.exps]),
                     np.concatenate([b.coefs, k.coefs]), np.concatenate([b.nprim, k.nprim]),
                     np.concatenate([b.lq, np.full((1, 4), 7, np.int32)]))
    check_plan(torch, b, plan_blocks(torch, b))


def test_solid_plan_equals_batch_solid_per_class(torch):
    """The plan's blocks equal eri4_batch_solid's on the same quartets, class
    by class (the same transforms over the same H matrices; 1e-15 of the
    transform bound allows for a different tile height)."""
    b = inputs.uneven_batch(nq=40, seed=464, lvals=(2, 4, 5), kmax=3)
    blocks = plan_blocks(torch, b)
    by_cls = {}
    for q in range(b.nq):
        by_cls.setdefault(tuple(int(x) for x in b.lq[q]), []).append(q)
    for ls, qs in by_cls.items():
        s = inputs.subset(b, qs)
        s = inputs.Batch(ls, s.centers, s.exps, s.coefs, s.nprim, s.lq)
        g = run(torch, s)
        cart = oracle.eri_md4(ls, s.centers, s.exps, s.coefs, s.nprim)
        bound = solid.cart_to_solid(np.abs(cart), ls, absolute=True)
        for i, q in enumerate(qs):
            scale = max(bound[i].max(), ZERO_SCALE)
            assert np.abs(blocks[q] - g[i]).max() <= 1e-15 * scale, (ls, q)


def test_solid_plan_with_tile_table_and_reuse(torch):
    """The tuned tile table gives the same integrals (to the oracle's bar);
    a second execute with a caller workspace repeats the first bit for bit."""
    b = inputs.uneven_batch(nq=24, seed=465, lvals=(4, 5), kmax=2)
    p = eri4.SolidPlan(b.lq, b.nprim, b.kmax, tune_file=eri4.TUNE_FILE)
    first = plan_blocks(torch, b, plan=p)
    check_plan(torch, b, first)
    w = torch.full((p.work_size + 3,), float("nan"), dtype=torch.float64, device="cuda")
    again = plan_blocks(torch, b, plan=p, work=w)
    for x, y in zip(first, again):
        assert np.array_equal(x, y)


def test_solid_plan_argument_errors(torch):
    b = inputs.uneven_batch(nq=3, seed=466, lvals=(1, 2), kmax=2)
    p = eri4.SolidPlan(b.lq, b.nprim, b.kmax)
    C, E, Co = dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs)
    out = torch.empty(p.output_size, dtype=torch.float64, device="cuda")
    w = torch.empty(max(1, p.work_size), dtype=torch.float64, device="cuda")
    # the Cartesian execute refuses a solid plan, and a short workspace is refused
    with pytest.raises(eri4.Eri4Error, match="eri4_plan_execute_solid"):
        eri4._check(eri4.lib().eri4_plan_execute(p._h, eri4._ptr(C, "float64"), eri4._ptr(E, "float64"),
                                                    eri4._ptr(Co, "float64"), eri4._ptr(out, "float64"), None))
    with pytest.raises(eri4.Eri4Error, match="workspace"):
        eri4._check(eri4.lib().eri4_plan_execute_solid(p._h, eri4._ptr(C, "float64"), eri4._ptr(E, "float64"),
                                                          eri4._ptr(Co, "float64"), eri4._ptr(w, "float64"),
                                                          p.work_size - 1, eri4._ptr(out, "float64"), None))
    cart = eri4.Plan(b.lq, b.nprim, b.kmax)
    with pytest.raises(eri4.Eri4Error, match="Cartesian plan"):
        eri4._check(eri4.lib().eri4_plan_execute_solid(cart._h, eri4._ptr(C, "float64"), eri4._ptr(E, "float64"),
                                                          eri4._ptr(Co, "float64"), eri4._ptr(w, "float64"),
                                                          w.numel(), eri4._ptr(out, "float64"), None))
    with pytest.raises(eri4.Eri4Error, match="unknown|is for|arch|open"):
        eri4.SolidPlan(b.lq, b.nprim, b.kmax, tune_file="/nonexistent/tile_table.txt")


def test_solid_plan_and_coulomb_batch_replay_in_a_hip_graph(torch):
    """A solid quartet plan (H build plus persistent kernel) and the J-engine
    Coulomb batch captured in one HIP graph (no allocation, no memset nodes)
    give the eager results on every replay, with eager work in between."""
    b = inputs.uneven_batch(nq=10, seed=467, lvals=(3, 4, 5), kmax=2)
    p = eri4.SolidPlan(b.lq, b.nprim, b.kmax, tune_file=eri4.TUNE_FILE)
    C, E, Co = dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs)
    work = torch.empty(max(1, p.work_size), dtype=torch.float64, device="cuda")
    eager_s = p.execute(C, E, Co, work=work).clone()
    ls = (5, 4, 4, 5)
    c = inputs.class_batch(ls, 4, 2, seed=468, exp_range=(0.05, 200.0))
    D = dev(torch, inputs.ket_densities(c, seed=469))
    cC, cE, cCo, cN = dev(torch, c.centers), dev(torch, c.exps), dev(torch, c.coefs), dev(torch, c.nprim)
    cwork = torch.empty(eri4.coulomb_work_size(ls, 2, 4), dtype=torch.float64, device="cuda")
    eager_c = eri4.batch_coulomb(ls, cC, cE, cCo, cN, D, work=cwork).clone()
    torch.cuda.synchronize()
    out_s = torch.zeros_like(eager_s)
    out_c = torch.zeros_like(eager_c)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        p.execute(C, E, Co, out=out_s, work=work, stream=s)
        eri4.batch_coulomb(ls, cC, cE, cCo, cN, D, work=cwork, out=out_c, stream=s)
    for rep in range(3):
        out_s.zero_()
        out_c.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_s, eager_s), rep
        assert torch.equal(out_c, eager_c), rep
        eri4.batch(ls, cC[:1].contiguous(), cE[:1].contiguous(), cCo[:1].contiguous(), cN[:1].contiguous())
        torch.cuda.synchronize()


def test_solid_plan_on_a_stream_sample_against_oracle(torch):
    """The quartet plan over solid harmonics with the tuned tile table on 48
    quartets of the l = 4..7, K = 3 stream batch (the benchmark's solid plan
    leg): every quartet of classes with total l <= 18 against the oracle, and
    the rest against the oracle's transform of the library's own Cartesian
    integrals from the Cartesian plan (checked against the oracle elsewhere)."""
    b = inputs.stream_batch(48, 1006)
    p = eri4.SolidPlan(b.lq, b.nprim, b.kmax, tune_file=eri4.TUNE_FILE)
    blocks = plan_blocks(torch, b, plan=p)
    cp = eri4.Plan(b.lq, b.nprim, b.kmax, tune_file=eri4.TUNE_FILE)
    cart = cp.execute(dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs))
    torch.cuda.synchronize()
    cart = cart.cpu().numpy()
    coff = cp.offsets()
    small = [q for q in range(b.nq) if int(b.lq[q].sum()) <= 18]
    assert small, "sample has no small classes"
    sub = inputs.subset(b, small)
    check_plan(torch, sub, [blocks[q] for q in small])
    for q in range(b.nq):
        ls = tuple(int(x) for x in b.lq[q])
        n = [(l + 1) * (l + 2) // 2 for l in ls]
        c = cart[coff[q]:coff[q] + int(np.prod(n))].reshape([1] + n)
        check(blocks[q][None], solid.cart_to_solid(c, ls), c, ls)
