"""Pins of the oracle's Cartesian-to-solid transform against facts that do not
depend on how it was written: the textbook p and d functions, harmonicity
(zero Laplacian) and orthonormality of every function in exact arithmetic, and
the covariance of whole integral blocks under rotations of the geometry."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import solid
from paper_2307_03452_amd import inputs


def test_p_and_d_functions_are_the_textbook_ones():
    assert np.array_equal(solid.solid_matrix(0), [[1.0]])
    # p: (y, z, x) for m = -1, 0, 1
    assert np.array_equal(solid.solid_matrix(1), [[0, 1, 0], [0, 0, 1], [1, 0, 0]])
    # d over (xx, xy, xz, yy, yz, zz): sqrt3 xy, sqrt3 yz, zz - (xx + yy)/2, sqrt3 xz, sqrt3/2 (xx - yy)
    s3 = math.sqrt(3.0)
    want = [[0, s3, 0, 0, 0, 0], [0, 0, 0, 0, s3, 0], [-0.5, 0, 0, -0.5, 0, 1], [0, 0, s3, 0, 0, 0],
            [s3 / 2, 0, 0, -s3 / 2, 0, 0]]
    assert np.allclose(solid.solid_matrix(2), want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("l", range(8))
def test_every_function_is_harmonic(l):
    """The Laplacian of sum_k c_k x^ax y^ay z^az vanishes exactly."""
    for n2, terms in solid.solid_exact(l):
        lap = {}
        for (ax, ay, az), c in terms.items():
            for axis, p in enumerate((ax, ay, az)):
                if p >= 2:
                    e = [ax, ay, az]
                    e[axis] -= 2
                    lap[tuple(e)] = lap.get(tuple(e), Fraction(0)) + c * p * (p - 1)
        assert all(v == 0 for v in lap.values()), (l, lap)
        assert terms, l


def _dfact(n):
    return 1 if n <= 0 else n * _dfact(n - 2)


@pytest.mark.parametrize("l", range(8))
def test_functions_are_orthonormal_in_exact_arithmetic(l):
    """<x^a|x^a'> / <x^l|x^l> = prod_i (a_i + a'_i - 1)!! / (2l - 1)!! when every
    a_i + a'_i is even (zero otherwise), for Gaussians on one centre with one
    exponent; under that metric the 2l+1 functions are orthonormal."""
    fun = solid.solid_exact(l)

    def g(a, b):
        s = [x + y for x, y in zip(a, b)]
        if any(v % 2 for v in s):
            return Fraction(0)
        return Fraction(math.prod(_dfact(v - 1) for v in s), _dfact(2 * l - 1))

    for i, (n2i, ti) in enumerate(fun):
        for j, (n2j, tj) in enumerate(fun):
            dot = sum((ci * cj * g(a, b) for a, ci in ti.items() for b, cj in tj.items()), Fraction(0))
            if i == j:
                assert n2i * dot == 1, (l, i)
            else:
                assert dot == 0, (l, i, j)


def _rot_z(alpha):
    c, s = math.cos(alpha), math.sin(alpha)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _d_z(l, alpha):
    """Solid functions evaluated at R r (R: rotation by alpha about z) in terms
    of the functions at r: S_m(R r) = sum_m' D[m][m'] S_m'(r).  A cos(m phi) /
    sin(m phi) pair mixes by the angle m alpha."""
    D = np.zeros((2 * l + 1, 2 * l + 1))
    D[l, l] = 1.0
    for m in range(1, l + 1):
        c, s = math.cos(m * alpha), math.sin(m * alpha)
        ip, im = l + m, l - m
        D[ip, ip], D[ip, im] = c, -s
        D[im, im], D[im, ip] = c, s
    return D


def _solid_block(ls, b):
    return solid.eri_solid(ls, b.centers, b.exps, b.coefs, b.nprim, scheme="os")


@pytest.mark.parametrize("ls", [(1, 0, 0, 0), (2, 1, 0, 2), (3, 2, 1, 3), (2, 3, 3, 2)])
def test_z_rotation_of_the_geometry_mixes_each_index_by_its_angle(ls):
    """Rotating every centre by R about the origin gives
    (ab|cd)[R A..] = sum D_a D_b D_c D_d (ab|cd)[A..], D from cos/sin(m alpha).
    Pins the m order, the phases and the pairing of each m with -m."""
    b = inputs.class_batch(ls, 3, 2, seed=91, exp_range=(0.2, 5.0), box=3.0)
    alpha = 0.7
    R = _rot_z(alpha)
    br = inputs.Batch(b.ls, b.centers @ R.T, b.exps, b.coefs, b.nprim)
    x0, x1 = _solid_block(ls, b), _solid_block(ls, br)
    Ds = [_d_z(l, alpha) for l in ls]
    want = np.einsum("ai,bj,ck,dl,qijkl->qabcd", *Ds, x0)
    assert np.abs(x1 - want).max() <= 1e-12 * np.abs(x0).max()


@pytest.mark.parametrize("ls", [(2, 2, 2, 2), (3, 1, 2, 3), (4, 2, 3, 1)])
def test_block_norm_is_invariant_under_any_rotation(ls):
    """An orthonormal set of 2l+1 harmonics per shell turns under a rotation by
    an orthogonal matrix, so the Frobenius norm of each quartet's block does not
    change (that of the Cartesian block does)."""
    b = inputs.class_batch(ls, 2, 1, seed=92, exp_range=(0.3, 4.0), box=3.0)
    q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))
    R = q * np.sign(np.linalg.det(q))
    br = inputs.Batch(b.ls, b.centers @ R.T, b.exps, b.coefs, b.nprim)
    x0, x1 = _solid_block(ls, b), _solid_block(ls, br)
    n0 = np.sqrt((x0 ** 2).sum(axis=(1, 2, 3, 4)))
    n1 = np.sqrt((x1 ** 2).sum(axis=(1, 2, 3, 4)))
    assert np.allclose(n0, n1, rtol=1e-12, atol=0)
    c0 = oracle.eri_os(ls, b.centers, b.exps, b.coefs, b.nprim)
    c1 = oracle.eri_os(ls, br.centers, br.exps, br.coefs, br.nprim)
    assert not np.allclose(np.sqrt((c0 ** 2).sum(axis=(1, 2, 3, 4))), np.sqrt((c1 ** 2).sum(axis=(1, 2, 3, 4))),
                           rtol=1e-6, atol=0)


def test_s_and_p_blocks_are_permuted_cartesian_blocks():
    """For l <= 1 the solid functions are Cartesian ones, reordered (y, z, x)."""
    ls = (1, 0, 1, 1)
    b = inputs.class_batch(ls, 2, 2, seed=93)
    cart = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
    perm = [1, 2, 0]
    want = cart[:, perm][:, :, :, perm][:, :, :, :, perm]
    assert np.array_equal(solid.cart_to_solid(cart, ls), want)
