"""Cartesian to real solid-harmonic transform, oracle side.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU leg);
it shares no code with the HIP library.

The paper contracts its E matrices with the coefficient matrices that express
real solid-harmonic Gaussians in Cartesian Gaussians (Sec. 2, the equation
defining H; coefficients after Schlegel and Frisch).  This module writes those
coefficients from the closed-form expansion of the real solid harmonics in
Cartesian monomials (Helgaker, Jorgensen and Olsen, "Molecular
Electronic-Structure Theory", Sec. 6.4.2), in exact rational arithmetic except
for one square root per (l, m), and applies them to whole Cartesian integral
blocks, one index at a time.

Conventions (readings; the paper states none):
  * 2l+1 functions ordered m = -l, ..., l.  For m > 0 the function is the real
    part of (x + i y)^m times a polynomial in z and r^2, for m < 0 the
    imaginary part of (x + i y)^|m| times the same polynomial (a cos(m phi) and
    a sin(|m| phi) pair), with no Condon-Shortley phase.
  * Cartesian components in the order of the integrals (a_x from l down to 0,
    then a_y from l - a_x down to 0), all sharing one contraction coefficient
    that gives x^l unit norm.  With that metric the solid functions below have
    unit norm: the normalisation constant is the one that makes
    S_l0 = z^l + ... (Racah's normalisation).
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def cart_index(l: int, ax: int, ay: int, az: int) -> int:
    """Position of x^ax y^ay z^az among the Cartesian components of shell l."""
    assert ax + ay + az == l
    return (l - ax) * (l - ax + 1) // 2 + az


@lru_cache(maxsize=None)
def solid_exact(l: int):
    """For m = -l..l: (N2, {(ax, ay, az): c}) with S_lm = sqrt(N2) * sum c x^ax y^ay z^az.

    N2 and every c are exact rationals.  The expansion runs over
    t = 0..floor((l-|m|)/2), u = 0..t and v (integer for m >= 0, half-integer
    for m < 0) with
      c_tuv = (-1)^(t + v - v_m) 4^-t C(l,t) C(l-t,|m|+t) C(t,u) C(|m|,2v)
      monomial x^(2t+|m|-2(u+v)) y^(2(u+v)) z^(l-2t-|m|)
    and N2 = 2 (l+|m|)! (l-|m|)! / 2^delta(m,0) / (2^|m| l!)^2.
    """
    out = []
    for m in range(-l, l + 1):
        am = abs(m)
        # v runs over v_m, v_m + 1, ...; work with w = 2v (odd for m < 0)
        w0 = 1 if m < 0 else 0
        w_hi = 2 * ((am - w0) // 2) + w0  # largest 2v: 2 * (floor(|m|/2 - v_m) + v_m)
        terms: dict = {}
        for t in range((l - am) // 2 + 1):
            for u in range(t + 1):
                for w in range(w0, w_hi + 1, 2):
                    sign = -1 if ((2 * t + w - w0) // 2) % 2 else 1
                    c = Fraction(sign * math.comb(l, t) * math.comb(l - t, am + t) * math.comb(t, u)
                                 * math.comb(am, w), 4 ** t)
                    py = 2 * u + w
                    px = 2 * t + am - py
                    pz = l - 2 * t - am
                    assert px >= 0 and pz >= 0
                    key = (px, py, pz)
                    terms[key] = terms.get(key, Fraction(0)) + c
        terms = {k: v for k, v in terms.items() if v != 0}
        n2 = Fraction(2 * math.factorial(l + am) * math.factorial(l - am), (2 if m == 0 else 1)
                      * (2 ** am * math.factorial(l)) ** 2)
        out.append((n2, terms))
    return out


@lru_cache(maxsize=None)
def solid_matrix(l: int) -> np.ndarray:
    """C[m + l][k]: coefficient of Cartesian component k in S_lm (float64)."""
    C = np.zeros((2 * l + 1, ncart(l)))
    for i, (n2, terms) in enumerate(solid_exact(l)):
        nrm = math.sqrt(n2.numerator) / math.sqrt(n2.denominator)
        for (ax, ay, az), c in terms.items():
            C[i, cart_index(l, ax, ay, az)] = nrm * float(c)
    C.setflags(write=False)
    return C


def cart_to_solid(block: np.ndarray, ls, absolute: bool = False) -> np.ndarray:
    """Solid-harmonic integrals from Cartesian ones.

    block: [..., Na, Nb, Nc, Nd] over the Cartesian components of shells
    l = ls; returns [..., 2la+1, 2lb+1, 2lc+1, 2ld+1].  absolute=True applies
    |C| instead of C: given |block| that is sum_k |C x C x C x C|[m, k] |block[k]|,
    the magnitude that bounds the rounding error of the transform."""
    la, lb, lc, ld = (int(x) for x in ls)
    Ca, Cb, Cc, Cd = (np.abs(solid_matrix(l)) if absolute else solid_matrix(l) for l in (la, lb, lc, ld))
    x = np.tensordot(block, Cd, axes=([-1], [1]))                   # [..., a, b, c, md]
    x = np.moveaxis(np.tensordot(x, Cc, axes=([-2], [1])), -1, -2)  # [..., a, b, mc, md]
    x = np.moveaxis(np.tensordot(x, Cb, axes=([-3], [1])), -1, -3)  # [..., a, mb, mc, md]
    x = np.moveaxis(np.tensordot(x, Ca, axes=([-4], [1])), -1, -4)  # [..., ma, mb, mc, md]
    return np.ascontiguousarray(x)


def eri_solid(ls, centers, exps, coefs, nprim, nthreads=0, scheme="md4"):
    """(ab|cd) over real solid-harmonic shells: the oracle's Cartesian
    integrals (scalar McMurchie-Davidson or Obara-Saika) transformed by
    cart_to_solid.  Arrays as for the Cartesian oracle."""
    from . import eri_md4, eri_os
    f = eri_md4 if scheme == "md4" else eri_os
    return cart_to_solid(f(ls, centers, exps, coefs, nprim, nthreads), ls)
