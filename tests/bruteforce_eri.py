"""Brute-force numerical (ab|cd) for one primitive quartet, by a route that uses
none of the recurrences or the Boys function (test infrastructure).

1/|r - r'| = (2/sqrt(pi)) int_0^inf exp(-s^2 |r - r'|^2) ds turns the 6-d
Coulomb integral into a 1-d integral over s of a product of three 2-d Gaussian
integrals (one per Cartesian axis).  Each 2-d integral of a polynomial times a
Gaussian is done exactly by tensor Gauss-Hermite quadrature after a Cholesky
change of variables; the s integral is mapped to t in [0, 1) by
s^2 = rho t^2 / (1 - t^2) and done by Gauss-Legendre quadrature, which converges
fast while T = rho |P - Q|^2 stays moderate.  Accuracy is a few 1e-12 relative to
the largest integral for the inputs the tests use.
"""
import numpy as np


def _cart(l):
    out = []
    for ax in range(l, -1, -1):
        for ay in range(l - ax, -1, -1):
            out.append((ax, ay, l - ax - ay))
    return np.array(out, dtype=np.int64)


def primitive_eri(ls, A, B, C, D, za, zb, zc, zd, n_gh=None, n_gl=96):
    la, lb, lc, ld = ls
    A, B, C, D = (np.asarray(x, dtype=np.float64) for x in (A, B, C, D))
    L = la + lb + lc + ld
    if n_gh is None:
        n_gh = L // 2 + 4
    p, q = za + zb, zc + zd
    rho = p * q / (p + q)
    P = (za * A + zb * B) / p
    Q = (zc * C + zd * D) / q
    xg, wg = np.polynomial.hermite.hermgauss(n_gh)
    tl, wl = np.polynomial.legendre.leggauss(n_gl)
    t = 0.5 * (tl + 1.0)
    wt = 0.5 * wl
    s2 = rho * t * t / (1.0 - t * t)                      # [nt]
    det = p * q + s2 * (p + q)                            # det of the 2x2 form
    W1, W2 = np.meshgrid(xg, xg, indexing="ij")
    WW = np.outer(wg, wg).ravel()                         # [ng]
    W1 = W1.ravel()
    W2 = W2.ravel()
    L11 = np.sqrt(p + s2)
    L21 = -s2 / L11
    L22 = np.sqrt(det / (p + s2))
    # z - mu = L^{-T} w
    u_off = (W1[None, :] / L11[:, None]) - (L21 / (L11 * L22))[:, None] * W2[None, :]
    v_off = W2[None, :] / L22[:, None]
    ax_I = []
    for i in range(3):
        d = P[i] - Q[i]
        mu1 = -s2 * d * q / det                           # centre of u = x - P
        mu2 = s2 * d * p / det                            # centre of v = x' - Q
        x = P[i] + mu1[:, None] + u_off                   # [nt, ng]
        xp = Q[i] + mu2[:, None] + v_off
        pref = (np.exp(-za * zb / p * (A[i] - B[i]) ** 2) * np.exp(-zc * zd / q * (C[i] - D[i]) ** 2)
                * np.exp(-s2 * d * d * p * q / det) / np.sqrt(det))   # [nt]
        XA = (x - A[i])[..., None] ** np.arange(la + 1)   # [nt, ng, la+1]
        XB = (x - B[i])[..., None] ** np.arange(lb + 1)
        XC = (xp - C[i])[..., None] ** np.arange(lc + 1)
        XD = (xp - D[i])[..., None] ** np.arange(ld + 1)
        I = np.einsum("g,tga,tgb,tgc,tgd->tabcd", WW, XA, XB, XC, XD, optimize=True)
        ax_I.append(I * pref[:, None, None, None, None])
    ca, cb, cc, cd = _cart(la), _cart(lb), _cart(lc), _cart(ld)
    ia, ib, ic, id_ = np.meshgrid(np.arange(len(ca)), np.arange(len(cb)), np.arange(len(cc)),
                                  np.arange(len(cd)), indexing="ij")
    ia, ib, ic, id_ = ia.ravel(), ib.ravel(), ic.ravel(), id_.ravel()
    prod = np.ones((len(t), ia.size))
    for i in range(3):
        prod *= ax_I[i][:, ca[ia, i], cb[ib, i], cc[ic, i], cd[id_, i]]
    jac = wt * np.sqrt(rho) * (1.0 - t * t) ** -1.5 * 2.0 / np.sqrt(np.pi)
    val = jac @ prod
    return val.reshape(len(ca), len(cb), len(cc), len(cd))
