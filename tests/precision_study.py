"""How much precision the two Hermite-to-Cartesian transforms need.

A CPU study (not a test): for (ii|ii) K=1 quartets of the benchmark workload
it builds the bra and ket E matrices and the [p|q] matrix of eqs.
(ab_to_hermite), (cd_to_hermite) and (pq) from the oracle's stage functions,
then evaluates (ab|cd) = E_ab [p|q] E_cd^T with the operands and sums held in
lower precisions, and prints the absolute error of each against the oracle's
(ab|cd):

  fp32      operands rounded to FP32, FP32 products and accumulation
  bf16x3    FP32 operands split into two BF16 parts, the three leading
            products, FP32 accumulation
  fixB      operands rounded to B-bit fixed point per row (bra) / column (ket)
            of each matrix, products and sums exact (the error of an
            exact-product splitting scheme that keeps B bits per operand)
  fixB-h    the same after the exact rescaling E^p -> E^p s^|p|,
            R_r -> R_r s^-|r| (s a power of two near sqrt(2 zeta)), which leaves
            every product E_ab^p [p|q] E_cd^q unchanged

  python tests/precision_study.py [nquartets]
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from paper_2307_03452_amd import inputs  # noqa: E402


def cart(l):
    return np.array([(ax, l - ax - az, az) for ax in range(l, -1, -1) for az in range(0, l - ax + 1)])


def herm(L):
    return np.array([(t, u, v) for t in range(L + 1) for u in range(L + 1 - t) for v in range(L + 1 - t - u)])


def e_matrix(la, lb, za, zb, A, B):
    """E_ab^p for all Cartesian pairs (rows, CCA order) and Hermite p (columns)."""
    E = oracle.md4_etab(la, lb, za, zb, A, B)
    a, b, h = cart(la), cart(lb), herm(la + lb)
    ai = np.repeat(a, len(b), axis=0)
    bi = np.tile(b, (len(a), 1))
    out = np.ones((len(ai), len(h)))
    for x in range(3):
        out *= E[x][ai[:, x][:, None], bi[:, x][:, None], h[None, :, x]]
    return out, h


def pq_matrix(hb, hk, L, zp, zq, P, Q):
    R = oracle.md4_rtuv(L, zp, zq, P, Q)
    s = hb[:, None, :] + hk[None, :, :]
    sign = np.where(hk.sum(axis=1) % 2 == 0, 1.0, -1.0)
    return R[s[..., 0], s[..., 1], s[..., 2]] * sign[None, :]


def bf16(x):
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32).view(np.float32)


def fixed(M, bits, axis):
    m = np.max(np.abs(M), axis=axis, keepdims=True)
    m[m == 0] = 1.0
    q = 2.0 ** (np.ceil(np.log2(m)) - bits)
    return np.round(M / q) * q


def variants(Eb, G, Ek, w, hb, hk, zp, zq):
    f = np.float32
    out = {}
    out["fp32"] = ((Eb.astype(f) @ G.astype(f)) @ Ek.T.astype(f)).astype(np.float64) * w

    def mm3(X, Y):
        xh, yh = bf16(X), bf16(Y)
        xl, yl = bf16(X.astype(f) - xh), bf16(Y.astype(f) - yh)
        return xh @ yh + xh @ yl + xl @ yh

    out["bf16x3"] = mm3(mm3(Eb.astype(f), G.astype(f)), Ek.T.astype(f)).astype(np.float64) * w
    s = 2.0 ** np.round(np.log2(np.sqrt(2.0 * min(zp, zq))))
    pb, pk = hb.sum(axis=1), hk.sum(axis=1)
    Ebh, Ekh = Eb * s ** pb[None, :], Ek * s ** pk[None, :]
    Gh = G / s ** pb[:, None] / s ** pk[None, :]
    for bits in (24, 32, 40, 48):
        X = fixed(Eb, bits, 1) @ fixed(G, bits, 0)
        out[f"fix{bits}"] = fixed(X, bits, 1) @ fixed(Ek, bits, 1).T * w
        X = fixed(Ebh, bits, 1) @ fixed(Gh, bits, 0)
        out[f"fix{bits}-h"] = fixed(X, bits, 1) @ fixed(Ekh, bits, 1).T * w
    return out


def main(nq=8):
    b = inputs.iiii(1, nq=nq)
    ref = oracle.eri_md4(b.ls, b.centers, b.exps, b.coefs, b.nprim).reshape(nq, 784, 784)
    names = None
    rows = []
    for q in range(nq):
        A, B, C, D = b.centers[q]
        za, zb, zc, zd = b.exps[q, :, 0]
        Eb, hb = e_matrix(6, 6, za, zb, A, B)
        Ek, hk = e_matrix(6, 6, zc, zd, C, D)
        zp, zq = za + zb, zc + zd
        P, Q = (za * A + zb * B) / zp, (zc * C + zd * D) / zq
        G = pq_matrix(hb, hk, 24, zp, zq, P, Q)
        w = np.prod(b.coefs[q, :, 0]) * np.exp(-za * zb / zp * np.sum((A - B) ** 2) - zc * zd / zq * np.sum((C - D) ** 2))
        res = variants(Eb, G, Ek, w, hb, hk, zp, zq)
        names = list(res)
        rows.append((np.abs(ref[q]).max(), [np.abs(res[k] - ref[q]).max() for k in names]))
    print("max|(ab|cd)|  " + "  ".join(f"{k:>9s}" for k in names))
    for mx, errs in rows:
        print(f"{mx:11.2e}  " + "  ".join(f"{e:9.1e}" for e in errs))
    worst = np.max([r[1] for r in rows], axis=0)
    print("worst        " + "  ".join(f"{e:9.1e}" for e in worst))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 8)
