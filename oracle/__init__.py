"""CPU oracle for 4-center Coulomb integrals over contracted Cartesian Gaussians.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are its only users.  It shares no code with the HIP
library.  See ``eri4_oracle.c`` for the schemes it implements and the readings
of the paper it takes, and ``solid.py`` for the Cartesian to solid-harmonic
transform.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liberi4_oracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.oracle_boys.restype = None
        for name in ("oracle_eri_md4", "oracle_eri_os", "oracle_eri_md4_quad"):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_int] * 4 + [ctypes.c_int64, dp, dp, dp, ip, ctypes.c_int, dp, ctypes.c_int]
            f.restype = ctypes.c_int
        L.oracle_md4_etab.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.oracle_md4_etab.restype = None
        L.oracle_md4_rtuv.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.oracle_md4_rtuv.restype = None
        L.oracle_max_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def max_threads() -> int:
    return lib().oracle_max_threads()


def boys(mmax: int, T: float) -> np.ndarray:
    """F_m(T) for m = 0..mmax (quad precision, rounded to double)."""
    F = np.zeros(mmax + 1)
    lib().oracle_boys(int(mmax), float(T), _dp(F))
    return F


def _eri(fn, ls, centers, exps, coefs, nprim, nthreads):
    la, lb, lc, ld = (int(x) for x in ls)
    centers = np.ascontiguousarray(centers, dtype=np.float64)
    exps = np.ascontiguousarray(exps, dtype=np.float64)
    coefs = np.ascontiguousarray(coefs, dtype=np.float64)
    nprim = np.ascontiguousarray(nprim, dtype=np.int32)
    nq = centers.shape[0]
    kmax = exps.shape[2]
    assert centers.shape == (nq, 4, 3) and exps.shape == (nq, 4, kmax)
    assert coefs.shape == (nq, 4, kmax) and nprim.shape == (nq, 4)
    out = np.zeros((nq, ncart(la), ncart(lb), ncart(lc), ncart(ld)))
    rc = fn(la, lb, lc, ld, nq, _dp(centers), _dp(exps), _dp(coefs),
            nprim.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), kmax, _dp(out), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def eri_md4(ls, centers, exps, coefs, nprim, nthreads=0):
    """(ab|cd) by the paper's McMurchie-Davidson scheme, plain scalar form."""
    return _eri(lib().oracle_eri_md4, ls, centers, exps, coefs, nprim, nthreads)


def eri_md4_quad(ls, centers, exps, coefs, nprim, nthreads=0):
    """(ab|cd) by the same scheme as eri_md4 with every step in __float128 and
    the result rounded to double: truth values that measure eri_md4's own
    rounding error (slow; for small samples)."""
    return _eri(lib().oracle_eri_md4_quad, ls, centers, exps, coefs, nprim, nthreads)


def eri_os(ls, centers, exps, coefs, nprim, nthreads=0):
    """(ab|cd) by Obara-Saika VRR + Head-Gordon-Pople HRR (independent scheme)."""
    return _eri(lib().oracle_eri_os, ls, centers, exps, coefs, nprim, nthreads)


def md4_etab(la, lb, za, zb, A, B):
    """Hermite expansion tables E[axis][a][b][t], shape (3, la+1, lb+1, la+lb+1)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    E = np.zeros((3, la + 1, lb + 1, la + lb + 1))
    lib().oracle_md4_etab(int(la), int(lb), float(za), float(zb), _dp(A), _dp(B), _dp(E))
    return E


def md4_rtuv(L, zp, zq, P, Q):
    """R^(0)[t][u][v] (shape (L+1,)*3, zero where t+u+v > L), no weights."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    R = np.zeros((L + 1, L + 1, L + 1))
    lib().oracle_md4_rtuv(int(L), float(zp), float(zq), _dp(P), _dp(Q), _dp(R))
    return R
