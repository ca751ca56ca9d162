"""Solid-harmonic output (eri4_batch_solid) against the oracle: its Cartesian
integrals transformed by its own coefficient table.

Tolerance: TOL times the quartet's largest sum_k |C x C x C x C|[m, k] |cart[k]|
(cart: its Cartesian integrals), with TOL = 1e-13 for classes whose shells all
have l <= 3 and 1e-14 above.  Measured worst ratios: 2.4e-14 for the l <= 3
classes (there the scale is close to the Cartesian maximum and both FP64 codes'
own rounding, about 1e-14 of it, shows) and 1.4e-16 for l >= 4 (the scale is
far above the integrals' size), so the bounds leave a factor of 4 and 70.  Solid functions of distant shells have no low
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
    return 1e-13 if max(ls) <= 3 else 1e-14


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
