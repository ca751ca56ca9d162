"""Seeded synthetic shell-quartet workloads.

This module only draws inputs: shell centres, primitive exponents, contraction
coefficients and contraction lengths, plus the unit normalisation of each
contracted shell.  It contains none of the integral method's arithmetic and is
the one piece shared by the CPU oracle tests and the HIP path.

Layouts (host numpy arrays, the same on the device):
    centers  float64 [nq][4][3]      Bohr, shells a, b, c, d of each quartet
    exps     float64 [nq][4][kmax]   primitive exponents (> 0)
    coefs    float64 [nq][4][kmax]   coefficients multiplying UNnormalised
                                     primitives x^ax y^ay z^az exp(-z r^2)
    nprim    int32   [nq][4]         contraction length of each shell, 1..kmax

Entries p >= nprim of exps/coefs are drawn like the others and never read.

Recipe (draw order is fixed so a seed reproduces a workload exactly):
  1. contraction length per shell (only when it varies),
  2. centres uniform in [0, box)^3,
  3. exponents log-uniform in [lo, hi],
  4. contraction coefficients uniform in [0.1, 1] (1 for K = 1),
  5. unit normalisation of the contracted shell's x^l component.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def _dfact(n: int) -> float:
    """(n)!! with (-1)!! = 1."""
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


def normalize_shell(l: int, exps: np.ndarray, raw: np.ndarray) -> np.ndarray:
    """Coefficients of unnormalised primitives giving a contracted shell whose
    x^l component has unit self-overlap.

    Each primitive is first normalised, N(z,l)^2 = (4z)^l (2z/pi)^{3/2} / (2l-1)!!,
    then the contraction is scaled by (sum_ij c_i c_j S_ij)^{-1/2} with
    S_ij = (2l-1)!! / (2(z_i+z_j))^l (pi/(z_i+z_j))^{3/2}, the overlap of the
    unnormalised x^l primitives.  Works on the trailing axis.
    """
    exps = np.asarray(exps, dtype=np.float64)
    raw = np.asarray(raw, dtype=np.float64)
    df = _dfact(2 * l - 1)
    nrm = np.sqrt((4.0 * exps) ** l * (2.0 * exps / np.pi) ** 1.5 / df)
    c = raw * nrm
    zs = exps[..., :, None] + exps[..., None, :]
    S = df / (2.0 * zs) ** l * (np.pi / zs) ** 1.5
    tot = np.einsum("...i,...ij,...j->...", c, S, c)
    return c / np.sqrt(tot)[..., None]


def normalize_shells(l, exps, raw, nprim):
    """Vectorised normalize_shell over [..., kmax] arrays with per-shell l and
    contraction length; entries p >= nprim keep their raw value."""
    l = np.asarray(l)
    kmax = exps.shape[-1]
    mask = np.arange(kmax) < np.asarray(nprim)[..., None]
    df = np.vectorize(lambda n: _dfact(2 * int(n) - 1), otypes=[np.float64])(l)
    lf = l.astype(np.float64)[..., None]
    nrm = np.sqrt((4.0 * exps) ** lf * (2.0 * exps / np.pi) ** 1.5 / df[..., None])
    c = np.where(mask, raw * nrm, 0.0)
    zs = exps[..., :, None] + exps[..., None, :]
    S = df[..., None, None] / (2.0 * zs) ** lf[..., None] * (np.pi / zs) ** 1.5
    tot = np.einsum("...i,...ij,...j->...", c, S, c)
    return np.where(mask, c / np.sqrt(tot)[..., None], raw)


@dataclass
class Batch:
    ls: tuple            # (la, lb, lc, ld) for single-class batches, else None
    centers: np.ndarray
    exps: np.ndarray
    coefs: np.ndarray
    nprim: np.ndarray
    lq: np.ndarray | None = None   # int32 [nq][4] for mixed-class batches

    @property
    def nq(self) -> int:
        return self.centers.shape[0]

    @property
    def kmax(self) -> int:
        return self.exps.shape[2]


def class_batch(ls, nq: int, K, seed: int, exp_range=(0.05, 50.0), box: float = 8.0,
                kmax: int | None = None) -> Batch:
    """One class (la lb|lc ld), nq quartets.

    K is an int (same contraction length for every shell), a pair (lo, hi)
    for a per-shell length drawn uniformly from lo..hi, or a dict
    {"shells": (ka, kb, kc, kd)} for fixed lengths per shell position.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if isinstance(K, dict):
        ks = np.array(K["shells"], dtype=np.int32)
        nprim = np.tile(ks, (nq, 1))
        km = int(ks.max())
    elif isinstance(K, (tuple, list)):
        klo, khi = int(K[0]), int(K[1])
        nprim = rng.integers(klo, khi + 1, size=(nq, 4)).astype(np.int32)
        km = khi
    else:
        km = int(K)
        nprim = np.full((nq, 4), km, dtype=np.int32)
    if kmax is None:
        kmax = km
    centers = rng.uniform(0.0, box, size=(nq, 4, 3))
    lo, hi = exp_range
    exps = np.exp(rng.uniform(np.log(lo), np.log(hi), size=(nq, 4, kmax)))
    if km == 1 and isinstance(K, int):
        raw = np.ones((nq, 4, kmax))
    else:
        raw = rng.uniform(0.1, 1.0, size=(nq, 4, kmax))
    coefs = np.zeros((nq, 4, kmax))
    for q in range(nq):
        for s in range(4):
            k = int(nprim[q, s])
            coefs[q, s, :k] = normalize_shell(int(ls[s]), exps[q, s, :k], raw[q, s, :k])
            coefs[q, s, k:] = raw[q, s, k:]
    return Batch(tuple(int(x) for x in ls), centers, exps, coefs, nprim)


def subset(b: Batch, idx) -> Batch:
    idx = np.asarray(idx)
    return Batch(b.ls, b.centers[idx].copy(), b.exps[idx].copy(), b.coefs[idx].copy(),
                 b.nprim[idx].copy(), None if b.lq is None else b.lq[idx].copy())


# Named workloads (sizes of the paper's high angular momentum classes).
def gggg_k1(nq: int = 64, seed: int = 1001) -> Batch:
    """(gg|gg), l = 4, uncontracted, exponents log-uniform [0.05, 50]."""
    return class_batch((4, 4, 4, 4), nq, 1, seed, exp_range=(0.05, 50.0))


def iiii(K: int = 1, nq: int = 512, seed: int | None = None) -> Batch:
    """(ii|ii), l = 6, K primitives per shell, exponents log-uniform [0.05, 200]."""
    if seed is None:
        seed = 1002 if K == 1 else 1003
    return class_batch((6, 6, 6, 6), nq, K, seed, exp_range=(0.05, 200.0))


# The paper's K for its low-l table is the product K_bra K_ket of the four
# contraction lengths; read here as lengths (1,1,1,1), (5,1,1,1), (5,1,5,1).
PAPER_K_SHELLS = {1: (1, 1, 1, 1), 5: (5, 1, 1, 1), 25: (5, 1, 5, 1)}


def low_l_batch(l: int, K: int, nq: int, seed: int) -> Batch:
    """(ll|ll) for l = 2 (d) or 3 (f) with the paper's K = K_bra K_ket in
    {1, 5, 25}, exponents log-uniform [0.05, 50], 8-Bohr cube."""
    return class_batch((l, l, l, l), nq, {"shells": PAPER_K_SHELLS[K]}, seed, exp_range=(0.05, 50.0))


def stream_batch(nq: int = 50000, seed: int = 1006) -> Batch:
    """Serving-style stream: 50 000 quartets over the 256 ordered classes in
    {4,5,6,7}^4 with Zipf(1.2) class counts, 3 primitives per shell."""
    return uneven_batch(nq=nq, seed=seed, lvals=(4, 5, 6, 7), k_fixed=3)


def zipf_classes(lvals=(4, 5, 6), s=1.2):
    """Ordered classes (la lb|lc ld) over lvals^4, ranked by (total L, tuple),
    with probabilities proportional to rank^-s."""
    import itertools
    cls = sorted(itertools.product(lvals, repeat=4), key=lambda t: (sum(t), t))
    p = np.arange(1, len(cls) + 1, dtype=np.float64) ** -s
    return cls, p / p.sum()


def uneven_batch(nq: int = 20000, seed: int = 1004, lvals=(4, 5, 6), kmax: int = 8,
                 exp_range=(0.05, 200.0), box: float = 8.0, k_fixed: int | None = None) -> Batch:
    """Mixed batch: class counts multinomial over Zipf(1.2) ranked classes,
    quartets shuffled, contraction length per shell uniform in 1..kmax (or
    k_fixed for every shell, with kmax = k_fixed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cls, p = zipf_classes(lvals)
    counts = rng.multinomial(nq, p)
    lq = np.repeat(np.array(cls, dtype=np.int32), counts, axis=0)
    lq = lq[rng.permutation(nq)]
    if k_fixed is not None:
        kmax = int(k_fixed)
        nprim = np.full((nq, 4), kmax, dtype=np.int32)
    else:
        nprim = rng.integers(1, kmax + 1, size=(nq, 4)).astype(np.int32)
    centers = rng.uniform(0.0, box, size=(nq, 4, 3))
    lo, hi = exp_range
    exps = np.exp(rng.uniform(np.log(lo), np.log(hi), size=(nq, 4, kmax)))
    raw = rng.uniform(0.1, 1.0, size=(nq, 4, kmax))
    raw = np.where(nprim[..., None] == 1, 1.0, raw)
    coefs = normalize_shells(lq, exps, raw, nprim)
    return Batch(None, centers, exps, coefs, nprim, lq)


@dataclass
class PairList:
    """A list of shell pairs (one side of a bra-list x ket-list batch).

    l, nprim  int32 [n][2]; centers float64 [n][2][3]; exps, coefs float64 [n][2][kmax]."""
    l: np.ndarray
    nprim: np.ndarray
    centers: np.ndarray
    exps: np.ndarray
    coefs: np.ndarray

    @property
    def n(self) -> int:
        return self.l.shape[0]


def pair_list(n: int, seed: int, lvals=(4, 5, 6), kmax: int = 4, exp_range=(0.05, 200.0),
              box: float = 8.0) -> PairList:
    """n shell pairs, each shell's l uniform over lvals and contraction length
    uniform in 1..kmax; centres, exponents and coefficients as in uneven_batch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    l = rng.choice(np.asarray(lvals, dtype=np.int32), size=(n, 2)).astype(np.int32)
    nprim = rng.integers(1, kmax + 1, size=(n, 2)).astype(np.int32)
    centers = rng.uniform(0.0, box, size=(n, 2, 3))
    lo, hi = exp_range
    exps = np.exp(rng.uniform(np.log(lo), np.log(hi), size=(n, 2, kmax)))
    raw = rng.uniform(0.1, 1.0, size=(n, 2, kmax))
    raw = np.where(nprim[..., None] == 1, 1.0, raw)
    coefs = normalize_shells(l, exps, raw, nprim)
    return PairList(l, nprim, centers, exps, coefs)


def expand_pairs(bra: PairList, ket: PairList) -> Batch:
    """The quartet batch of every bra pair with every ket pair, quartet
    (i, j) at index i * ket.n + j (shells a, b from bra pair i; c, d from ket
    pair j).  Both lists must have the same kmax."""
    nb, nk = bra.n, ket.n
    cat = lambda x, y: np.concatenate([np.repeat(x, nk, axis=0), np.tile(y, (nb,) + (1,) * (y.ndim - 1))], axis=1)
    return Batch(None, cat(bra.centers, ket.centers), cat(bra.exps, ket.exps), cat(bra.coefs, ket.coefs),
                 cat(bra.nprim, ket.nprim).astype(np.int32), cat(bra.l, ket.l).astype(np.int32))


def ket_densities(b: Batch, seed: int, ls=None) -> np.ndarray:
    """A density block D[q][Nc][Nd] per quartet (uniform in [-1, 1]) for the
    Coulomb contraction; ls defaults to the batch's class."""
    ls = b.ls if ls is None else ls
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=(b.nq, ncart(ls[2]), ncart(ls[3])))


def exchange_densities(b: Batch, seed: int, ls=None) -> np.ndarray:
    """A density block D[q][Nb][Nd] per quartet (uniform in [-1, 1]) for the
    exchange contraction K_ac = sum_bd (ab|cd) D_bd; ls defaults to the
    batch's class."""
    ls = b.ls if ls is None else ls
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=(b.nq, ncart(ls[1]), ncart(ls[3])))
