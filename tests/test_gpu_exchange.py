"""Exchange-type contraction without forming (ab|cd) (eri4_batch_exchange)
against the oracle: its Cartesian integrals contracted with the density,
K_ac = sum_bd (ab|cd) D_bd.  Tolerance: 1e-12 times the quartet's largest
sum_bd |(ab|cd)| |D_bd|, the scale the contraction rounds at."""
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
    out = eri4.batch_exchange(b.ls, dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs),
                              dev(torch, b.nprim), dev(torch, D), work=work)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(g, I, D):
    ref = np.einsum("qabcd,qbd->qac", I, D)
    bound = np.einsum("qabcd,qbd->qac", np.abs(I), np.abs(D))
    assert g.shape == ref.shape
    for q in range(ref.shape[0]):
        scale = max(bound[q].max(), 1e-250)
        assert np.isfinite(g[q]).all(), q
        assert np.abs(g[q] - ref[q]).max() <= TOL * scale, (q, np.abs(g[q] - ref[q]).max() / scale)


# classes cover every tile height and R layout the library picks (16-, 32- and
# 64-row tiles; box, two boxes, slab), rows per b of 16, 32 and 48, and column
# blocks of c from 1 to 3
@pytest.mark.parametrize("ls,K,nq", [((0, 0, 0, 0), 2, 5), ((1, 0, 2, 1), (1, 3), 6), ((2, 2, 2, 2), 2, 4),
                                     ((3, 1, 2, 3), 1, 4), ((4, 4, 4, 4), 1, 3), ((4, 4, 4, 4), 3, 2),
                                     ((5, 4, 6, 3), 2, 2), ((4, 6, 5, 6), 1, 2), ((6, 6, 6, 6), 1, 2),
                                     ((6, 6, 6, 6), 2, 1), ((7, 7, 7, 7), 1, 1), ((6, 7, 6, 7), 1, 1),
                                     ((7, 5, 7, 2), 2, 2)])
def test_against_oracle(torch, ls, K, nq):
    b = inputs.class_batch(ls, nq, K, seed=800 + 3 * sum(ls) + (K if isinstance(K, int) else 9),
                           exp_range=(0.05, 200.0))
    D = inputs.exchange_densities(b, seed=81)
    I = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
    check(run(torch, b, D), I, D)


def test_matches_contracting_the_librarys_own_integrals_at_full_size(torch):
    """(ii|ii), K=1, the 512-quartet benchmark batch: K from eri4_batch_exchange
    against the contraction of eri4_batch's integrals (checked against the
    oracle elsewhere) on every quartet, and the oracle on two of them."""
    b = inputs.iiii(K=1)
    D = inputs.exchange_densities(b, seed=82)
    g = run(torch, b, D)
    d = lambda a: dev(torch, a)
    I = eri4.batch(b.ls, d(b.centers), d(b.exps), d(b.coefs), d(b.nprim))
    torch.cuda.synchronize()
    Dt = d(D)
    for q0 in range(0, b.nq, 64):
        Ib = I[q0:q0 + 64]
        ref = torch.einsum("qabcd,qbd->qac", Ib, Dt[q0:q0 + 64]).cpu().numpy()
        bound = torch.einsum("qabcd,qbd->qac", Ib.abs(), Dt[q0:q0 + 64].abs()).cpu().numpy()
        for i in range(ref.shape[0]):
            assert np.abs(g[q0 + i] - ref[i]).max() <= TOL * bound[i].max(), q0 + i
    s = inputs.subset(b, [0, 511])
    check(g[[0, 511]], oracle.eri_md4(b.ls, s.centers, s.exps, s.coefs, s.nprim), D[[0, 511]])


def test_passes_through_a_small_workspace_give_the_same_result(torch):
    b = inputs.class_batch((5, 4, 5, 4), 9, 2, seed=83, exp_range=(0.05, 200.0))
    D = inputs.exchange_densities(b, seed=84)
    full = run(torch, b, D)
    w = torch.empty(eri4.exchange_work_size(b.ls, b.kmax, 2), dtype=torch.float64, device="cuda")
    assert np.array_equal(full, run(torch, b, D, work=w))
    with pytest.raises(eri4.Eri4Error, match="workspace"):
        run(torch, b, D, work=torch.empty(10, dtype=torch.float64, device="cuda"))


def test_bad_contraction_length_gives_nan_and_others_are_untouched(torch):
    b = inputs.class_batch((4, 4, 4, 4), 3, 1, seed=85, kmax=2)
    b.nprim[1, 0] = 3  # > kmax
    D = inputs.exchange_densities(b, seed=86)
    g = run(torch, b, D)
    assert np.isnan(g[1]).all()
    assert np.isfinite(g[0]).all() and np.isfinite(g[2]).all()
    s = inputs.subset(b, [0, 2])
    check(g[[0, 2]], oracle.eri_md4(b.ls, s.centers, s.exps, s.coefs, s.nprim), D[[0, 2]])
