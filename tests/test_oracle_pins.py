"""Pins of the CPU oracle to facts other than itself (no GPU needed).

Each test checks the oracle against something the paper or the mathematics
fixes independently of the oracle's own code: a high-precision quadrature of
the Boys integral, closed values, a brute-force 6-d quadrature of the Coulomb
integral, a second independent recurrence, exact symmetries and bounds, and the
sizes the paper prints.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import bruteforce_eri as bf
from paper_2307_03452_amd import inputs, metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one(ls, rng, K=1, spread=1.5, zlo=0.4, zhi=2.0, nq=1):
    c = rng.uniform(0, spread, (nq, 4, 3))
    e = rng.uniform(zlo, zhi, (nq, 4, K))
    co = rng.uniform(0.2, 1.0, (nq, 4, K)) if K > 1 else np.ones((nq, 4, 1))
    n = np.full((nq, 4), K, np.int32)
    return c, e, co, n


# ---------------------------------------------------------------- Boys (eq. boys)

def test_boys_against_high_precision_quadrature():
    """eq. (boys) by mpmath: the lower incomplete gamma form (substituting
    u = T y^2) at 40 digits, and a direct quadrature of the integral."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    for T in (0.0, 1e-6, 0.3, 2.5, 11.7, 29.0, 49.99, 50.01, 77.0, 150.0, 1234.5):
        F = oracle.boys(28, T)
        for m in (0, 1, 4, 9, 16, 24, 28):
            if T > 0:
                g = mpmath.gammainc(m + 0.5, 0, T) / (2 * mpmath.mpf(T) ** (m + 0.5))
            else:
                g = mpmath.mpf(1) / (2 * m + 1)
            assert abs(F[m] - float(g)) <= 2.5e-16 * float(g), (T, m)
            if T > 200:
                continue  # direct quadrature of the sharp peak is less accurate than F itself
            # the integrand peaks at y = sqrt(m/T); many panels around it
            top = min(1.0, 12.0 * math.sqrt((m + 1) / T)) if T > 0 else 1.0
            pts = mpmath.linspace(0, top, 60) + ([1] if top < 1 else [])
            ref = mpmath.quad(lambda y: y ** (2 * m) * mpmath.exp(-T * y * y), pts, method="gauss-legendre")
            assert abs(F[m] - float(ref)) <= 1e-14 * float(ref), (T, m, F[m], ref)


def test_boys_at_zero_is_one_over_2m_plus_1():
    F = oracle.boys(32, 0.0)
    for m in range(33):
        assert F[m] == 1.0 / (2 * m + 1)


def test_boys_f0_is_error_function():
    for T in (1e-3, 0.7, 3.3, 20.0, 49.0, 51.0, 400.0):
        ref = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
        assert abs(oracle.boys(0, T)[0] - ref) <= 4e-16 * ref


def test_boys_downward_relation_holds_across_branch_switch():
    for T in (45.0, 50.0, 55.0, 120.0):
        F = oracle.boys(30, T)
        for m in range(30):
            lhs = (2 * T * F[m + 1] + math.exp(-T)) / (2 * m + 1)
            assert abs(lhs - F[m]) <= 1e-15 * F[m]


# ------------------------------------------- Hermite expansion (eq. cart2herm-2)

def test_etab_reproduces_cartesian_product_pointwise():
    """x_A^a x_B^b exp(-za x_A^2 - zb x_B^2) = K sum_t E^t_ab Lambda_t(x), with
    Lambda_t = (d/dP)^t exp(-zp (x-P)^2) = zp^{t/2} H_t(sqrt(zp)(x-P)) exp(..)."""
    rng = np.random.default_rng(3)
    from numpy.polynomial.hermite import hermval
    for la, lb in ((0, 0), (1, 0), (0, 2), (3, 2), (6, 6), (7, 5)):
        za, zb = rng.uniform(0.2, 3.0, 2)
        A, B = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
        E = oracle.md4_etab(la, lb, za, zb, A, B)
        zp = za + zb
        for i in range(3):
            P = (za * A[i] + zb * B[i]) / zp
            K = math.exp(-za * zb / zp * (A[i] - B[i]) ** 2)
            for x in rng.uniform(-2, 2, 5):
                y = math.sqrt(zp) * (x - P)
                g = math.exp(-y * y)
                for a in range(la + 1):
                    for b in range(lb + 1):
                        lhs = (x - A[i]) ** a * (x - B[i]) ** b * math.exp(-za * (x - A[i]) ** 2 - zb * (x - B[i]) ** 2)
                        rhs = 0.0
                        for t in range(a + b + 1):
                            c = np.zeros(t + 1)
                            c[t] = 1.0
                            rhs += E[i, a, b, t] * zp ** (t / 2) * hermval(y, c) * g
                        scale = max(1.0, abs(lhs)) * (1 + max(abs(x - A[i]), abs(x - B[i]))) ** (a + b)
                        assert abs(lhs - K * rhs) <= 1e-12 * scale, (la, lb, a, b, x)


def test_etab_zero_beyond_a_plus_b():
    E = oracle.md4_etab(5, 4, 0.7, 1.3, np.array([0.1, 0.2, 0.3]), np.array([1.0, -0.5, 0.0]))
    for a in range(6):
        for b in range(5):
            assert np.all(E[:, a, b, a + b + 1:] == 0.0)


def test_etab_overlap_by_gauss_hermite():
    """E^0_ab sqrt(pi/zp) K_x is the 1-d overlap, exact by Gauss-Hermite."""
    xg, wg = np.polynomial.hermite.hermgauss(20)
    rng = np.random.default_rng(4)
    for la, lb in ((2, 3), (6, 6), (7, 7)):
        za, zb = rng.uniform(0.1, 4.0, 2)
        A, B = rng.uniform(-2, 2, 3), rng.uniform(-2, 2, 3)
        E = oracle.md4_etab(la, lb, za, zb, A, B)
        zp = za + zb
        for i in range(3):
            P = (za * A[i] + zb * B[i]) / zp
            K = math.exp(-za * zb / zp * (A[i] - B[i]) ** 2)
            x = P + xg / math.sqrt(zp)
            for a in range(la + 1):
                for b in range(lb + 1):
                    S = np.sum(wg * (x - A[i]) ** a * (x - B[i]) ** b) / math.sqrt(zp)
                    assert abs(S - E[i, a, b, 0] * math.sqrt(math.pi / zp)) <= 1e-12 * (1 + abs(S))


# ---------------------------------------------------------- full integrals

@pytest.mark.parametrize("ls", [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1),
                                (1, 1, 1, 1), (2, 1, 0, 2), (2, 2, 2, 2), (3, 2, 1, 3), (4, 4, 4, 4),
                                (5, 3, 4, 2)])
def test_md4_against_bruteforce_quadrature(ls):
    rng = np.random.default_rng(100 + sum(ls))
    c, e, co, n = one(ls, rng)
    md = oracle.eri_md4(ls, c, e, co, n)[0]
    ref = bf.primitive_eri(ls, *c[0], *e[0, :, 0])
    assert np.abs(md - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.slow
def test_md4_against_bruteforce_quadrature_iiii():
    rng = np.random.default_rng(66)
    ls = (6, 6, 6, 6)
    c, e, co, n = one(ls, rng)
    md = oracle.eri_md4(ls, c, e, co, n)[0]
    ref = bf.primitive_eri(ls, *c[0], *e[0, :, 0])
    assert np.abs(md - ref).max() <= 1e-12 * np.abs(ref).max()


def test_md4_against_obara_saika_all_low_classes_contracted():
    rng = np.random.default_rng(7)
    for la in range(3):
        for lb in range(3):
            for lc in range(3):
                for ld in range(3):
                    ls = (la, lb, lc, ld)
                    c, e, co, n = one(ls, rng, K=2, spread=3.0, zlo=0.1, zhi=10.0, nq=2)
                    md = oracle.eri_md4(ls, c, e, co, n)
                    os_ = oracle.eri_os(ls, c, e, co, n)
                    for q in range(2):
                        # The horizontal recurrence loses a few digits when |A-B| is
                        # large next to the integrals' size; where the two differ by
                        # more than 1e-13 the brute-force quadrature sides with MD.
                        assert np.abs(md[q] - os_[q]).max() <= 2e-12 * np.abs(os_[q]).max(), ls


def test_md4_against_obara_saika_high_l_samples():
    """Compact geometry: there the horizontal recurrence keeps its accuracy
    (with distant, tight shells it loses digits; the quadrature test below
    covers that regime)."""
    for i, ls in enumerate(((4, 4, 4, 4), (5, 4, 6, 3), (6, 6, 5, 5), (7, 4, 4, 7))):
        b = inputs.class_batch(ls, 1, 1, seed=40 + i, exp_range=(0.3, 3.0), box=1.0)
        md = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
        os_ = oracle.eri_os(ls, b.centers, b.exps, b.coefs, b.nprim)
        assert np.abs(md - os_).max() <= 1e-12 * np.abs(os_).max(), ls


@pytest.mark.parametrize("ls,seed", [((4, 4, 4, 4), 41), ((4, 4, 4, 4), 42), ((6, 5, 6, 4), 41)])
def test_md4_against_bruteforce_in_workload_regime(ls, seed):
    """Exponents log-uniform in [0.05, 50] over a 3-Bohr cube (T up to ~10)."""
    b = inputs.class_batch(ls, 1, 1, seed=seed, exp_range=(0.05, 50.0), box=3.0)
    md = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)[0]
    ref = b.coefs[0, :, 0].prod() * bf.primitive_eri(ls, *b.centers[0], *b.exps[0, :, 0])
    assert np.abs(md - ref).max() <= 1e-13 * np.abs(ref).max()


def test_ssss_point_charge_limit():
    """Far-apart distributions interact like point charges S_ab S_cd / R."""
    ls = (0, 0, 0, 0)
    A = np.array([0.0, 0.0, 0.0]); B = np.array([0.3, -0.2, 0.1])
    C = np.array([40.0, 35.0, -30.0]); D = C + np.array([-0.2, 0.1, 0.25])
    za, zb, zc, zd = 1.1, 0.9, 1.7, 0.6
    c = np.array([[A, B, C, D]])
    e = np.array([[[za], [zb], [zc], [zd]]])
    v = oracle.eri_md4(ls, c, e, np.ones((1, 4, 1)), np.ones((1, 4), np.int32))[0, 0, 0, 0, 0]
    p, q = za + zb, zc + zd
    Sab = (math.pi / p) ** 1.5 * math.exp(-za * zb / p * np.sum((A - B) ** 2))
    Scd = (math.pi / q) ** 1.5 * math.exp(-zc * zd / q * np.sum((C - D) ** 2))
    R = np.linalg.norm((za * A + zb * B) / p - (zc * C + zd * D) / q)
    assert abs(v - Sab * Scd / R) <= 1e-13 * abs(v)


def _cart(l):
    return [(ax, ay, l - ax - ay) for ax in range(l, -1, -1) for ay in range(l - ax, -1, -1)]


@pytest.mark.parametrize("ls", [(4, 3, 2, 1), (4, 4, 4, 4), (6, 5, 4, 6)])
def test_eightfold_permutational_symmetry(ls):
    la, lb, lc, ld = ls
    b = inputs.class_batch(ls, 1, 2, seed=11 + la, exp_range=(0.05, 50.0), box=4.0)
    C, E, Co, N = b.centers, b.exps, b.coefs, b.nprim
    ref = oracle.eri_md4(ls, C, E, Co, N)[0]
    scale = np.abs(ref).max()
    perms = {  # shell order, and axes of ref to move
        (1, 0, 2, 3): (1, 0, 2, 3),
        (0, 1, 3, 2): (0, 1, 3, 2),
        (2, 3, 0, 1): (2, 3, 0, 1),
        (3, 2, 1, 0): (3, 2, 1, 0),
    }
    for order, axes in perms.items():
        ls2 = tuple(ls[i] for i in order)
        v = oracle.eri_md4(ls2, C[:, order], E[:, order], Co[:, order], N[:, order])[0]
        assert np.abs(v - np.transpose(ref, axes)).max() <= 1e-13 * scale, order


def test_translation_invariance():
    ls = (5, 4, 4, 5)
    b = inputs.class_batch(ls, 1, 2, seed=21, box=4.0)
    ref = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)[0]
    shifted = b.centers + np.array([3.25, -7.5, 1.125])
    v = oracle.eri_md4(ls, shifted, b.exps, b.coefs, b.nprim)[0]
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(ref).max()


def test_axis_swap_permutes_components():
    ls = (4, 2, 3, 4)
    b = inputs.class_batch(ls, 1, 1, seed=22, box=4.0)
    ref = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)[0]
    sw = b.centers[:, :, [1, 0, 2]].copy()
    v = oracle.eri_md4(ls, sw, b.exps, b.coefs, b.nprim)[0]
    idx = []
    for l in ls:
        c = _cart(l)
        pos = {t: i for i, t in enumerate(c)}
        idx.append([pos[(t[1], t[0], t[2])] for t in c])
    perm = ref[np.ix_(*idx)]
    assert np.abs(v - perm).max() <= 1e-13 * np.abs(ref).max()


def test_reflection_sign():
    ls = (5, 3, 4, 4)
    b = inputs.class_batch(ls, 1, 1, seed=23, box=4.0)
    ref = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)[0]
    fl = b.centers.copy()
    fl[:, :, 0] *= -1.0
    v = oracle.eri_md4(ls, fl, b.exps, b.coefs, b.nprim)[0]
    sg = [np.array([(-1.0) ** t[0] for t in _cart(l)]) for l in ls]
    sign = np.einsum("a,b,c,d->abcd", *sg)
    assert np.abs(v - sign * ref).max() <= 1e-13 * np.abs(ref).max()


def test_schwarz_bound_and_positive_diagonal():
    rng = np.random.default_rng(9)
    for ls in ((4, 4, 4, 4), (5, 6, 4, 5)):
        la, lb, lc, ld = ls
        b = inputs.class_batch(ls, 3, 2, seed=int(rng.integers(1 << 30)), box=4.0)
        abcd = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
        cab = b.centers[:, [0, 1, 0, 1]]
        ccd = b.centers[:, [2, 3, 2, 3]]
        abab = oracle.eri_md4((la, lb, la, lb), cab, b.exps[:, [0, 1, 0, 1]], b.coefs[:, [0, 1, 0, 1]], b.nprim[:, [0, 1, 0, 1]])
        cdcd = oracle.eri_md4((lc, ld, lc, ld), ccd, b.exps[:, [2, 3, 2, 3]], b.coefs[:, [2, 3, 2, 3]], b.nprim[:, [2, 3, 2, 3]])
        nab, ncd = metrics.npair(la, lb), metrics.npair(lc, ld)
        for q in range(3):
            M1 = abab[q].reshape(nab, nab)
            M2 = cdcd[q].reshape(ncd, ncd)
            assert np.allclose(M1, M1.T, rtol=0, atol=1e-13 * np.abs(M1).max())
            assert np.linalg.eigvalsh(0.5 * (M1 + M1.T)).min() >= -1e-12 * np.abs(M1).max()
            d1, d2 = np.diag(M1), np.diag(M2)
            bound = np.sqrt(np.outer(d1, d2))
            X = abcd[q].reshape(nab, ncd)
            assert np.all(np.abs(X) <= bound * (1 + 1e-12) + 1e-300)


def test_unit_normalisation_of_generated_shells():
    """The x^l component of each generated contracted shell has unit norm:
    its (ss|ss)-like self overlap computed independently by Gauss-Hermite."""
    b = inputs.class_batch((4, 6, 5, 7), 2, 3, seed=5)
    xg, wg = np.polynomial.hermite.hermgauss(30)
    for q in range(2):
        for s, l in enumerate((4, 6, 5, 7)):
            z = b.exps[q, s, :3]
            c = b.coefs[q, s, :3]
            tot = 0.0
            for i in range(3):
                for j in range(3):
                    zz = z[i] + z[j]
                    x = xg / math.sqrt(zz)
                    sx = np.sum(wg * x ** (2 * l)) / math.sqrt(zz)
                    tot += c[i] * c[j] * sx * (math.pi / zz)
            assert abs(tot - 1.0) <= 1e-13


# ------------------------------------------------ sizes printed in the paper

def test_paper_printed_sizes():
    g = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    ff = metrics.footprint(3, 3, 3, 3, solid=True)
    assert ff["N_p"] == g["ff_N_p"]
    assert ff["N_r"] == g["ff_N_r"]
    assert ff["pq_bytes"] == g["ff_pq_bytes"]
    assert ff["R_bytes"] == g["ff_R_bytes"]
    assert ff["H_bra_elems"] == g["ff_H_elems_solid"]
    assert ff["H_bra_bytes"] == g["ff_H_bytes_solid"]
    ii = metrics.footprint(6, 6, 6, 6, solid=True)
    assert round(ii["R_bytes"] / 1000) == g["ii_R_kB"]
    assert round(ii["pq_bytes"] / 1e6, 2) == g["ii_pq_MB"]
    assert round(ii["H_bra_bytes"] / 1000) == g["ii_H_kB_solid"]
    assert round(metrics.arithmetic_intensity(6, 6, 6, 6), 1) == g["ai_ii_solid"]
    assert round(metrics.arithmetic_intensity(3, 3, 3, 3), 1) == g["ai_ff_solid"]
