"""Size, FLOP and byte bookkeeping of the matrix-form McMurchie-Davidson scheme.

FLOPs follow the paper's accounting (Sec. 2, the cost analysis after
eq. (cd_to_hermite)): only the two Hermite-to-Cartesian matrix products are
counted, as dense products,
    2 N_ab (K_bra N_p) (K_ket N_q)      first transform, eq. (make-abq)
    2 N_ab (K_ket N_q) N_cd             second transform, eq. (make-abcd)
with the primitive contraction folded into the product dimensions.  The
arithmetic-intensity model is eq. (AI).
"""
from __future__ import annotations


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def nsolid(l: int) -> int:
    return 2 * l + 1


def nherm(L: int) -> int:
    """Hermite functions with total order <= L (pyramidal number, Sec. 2)."""
    return (L + 1) * (L + 2) * (L + 3) // 6


def npair(la: int, lb: int, solid: bool = False) -> int:
    f = nsolid if solid else ncart
    return f(la) * f(lb)


def md4_flops(la, lb, lc, ld, kbra: int = 1, kket: int = 1, solid: bool = False) -> int:
    """Dense matrix FLOPs of one shell quartet (bra transform first)."""
    nab, ncd = npair(la, lb, solid), npair(lc, ld, solid)
    npp, nqq = nherm(la + lb), nherm(lc + ld)
    return 2 * nab * (kbra * npp) * (kket * nqq) + 2 * nab * (kket * nqq) * ncd


def md4_flops_split(la, lb, lc, ld, kbra: int = 1, kket: int = 1):
    nab, ncd = npair(la, lb), npair(lc, ld)
    npp, nqq = nherm(la + lb), nherm(lc + ld)
    return 2 * nab * (kbra * npp) * (kket * nqq), 2 * nab * (kket * nqq) * ncd


def integrals_per_quartet(la, lb, lc, ld) -> int:
    return ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)


def output_bytes(la, lb, lc, ld) -> int:
    return 8 * integrals_per_quartet(la, lb, lc, ld)


def input_bytes(kmax: int) -> int:
    """Bytes of one quartet's inputs: centres, exponents, coefficients, lengths."""
    return 4 * 3 * 8 + 2 * 4 * kmax * 8 + 4 * 4


def footprint(la, lb, lc, ld, solid: bool = False) -> dict:
    """FP64 footprints of the intermediates of one primitive quartet (Sec. 2)."""
    Lb, Lk = la + lb, lc + ld
    npp, nqq, nrr = nherm(Lb), nherm(Lk), nherm(Lb + Lk)
    return {
        "N_p": npp,
        "N_q": nqq,
        "N_r": nrr,
        "R_bytes": 8 * nrr,
        "pq_bytes": 8 * npp * nqq,
        "H_bra_elems": npair(la, lb, solid) * npp,
        "H_bra_bytes": 8 * npair(la, lb, solid) * npp,
    }


def arithmetic_intensity(la, lb, lc, ld, solid: bool = True) -> float:
    """FLOP/byte estimate of eq. (AI)."""
    nab, ncd = npair(la, lb, solid), npair(lc, ld, solid)
    npp, nqq = nherm(la + lb), nherm(lc + ld)
    num = nab * nqq * (npp + ncd)
    den = 2 * npp * nqq + nab * (npp + 2 * nqq + ncd) + ncd * nqq
    return 0.25 * num / den
