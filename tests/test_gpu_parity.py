"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: FP64 integrals within 1e-12 of each quartet's largest |integral|;
component order and quartet order are checked exactly by comparing every
element at its own index on distinct quartets.  Stage outputs (Boys, Hermite
R, Hermite E) are compared with the oracle's intermediates.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2307_03452_amd import eri4, inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12
# Quartets whose integrals all lie below this size are numerically zero (the
# Gaussian-product prefactor underflowed); FP64 keeps no relative precision
# there (subnormal intermediates), so they are compared on an absolute floor.
ZERO_SCALE = 1e-250


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a ROCm device"
    eri4.init()
    return _t


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def run_gpu(torch, b: inputs.Batch, ls=None):
    ls = b.ls if ls is None else ls
    out = eri4.batch(ls, dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs),
                     dev(torch, b.nprim, torch.int32))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def assert_quartets_close(g, o, tol=TOL, label=""):
    assert g.shape == o.shape, (g.shape, o.shape)
    for q in range(o.shape[0]):
        scale = max(np.abs(o[q]).max(), ZERO_SCALE)
        err = np.abs(g[q] - o[q]).max()
        assert np.isfinite(g[q]).all(), (label, q)
        assert err <= tol * scale, (label, q, err, scale, err / scale)


# ------------------------------------------------------------------ stages

def test_boys_stage(torch):
    Ts = np.concatenate([[0.0, 1e-14, 1e-8, 1.0 / 64, 0.5, 1.0, 10.0, 29.99, 30.0, 50.0, 119.98,
                          119.99, 120.0, 120.01, 300.0, 1e4, 4e4],
                         np.random.default_rng(0).uniform(0, 130, 200)])
    F = eri4.boys(28, dev(torch, Ts)).cpu().numpy()
    for i, T in enumerate(Ts):
        ref = oracle.boys(28, T)
        assert np.all(np.abs(F[i] - ref) <= 2e-15 * ref), (T, np.max(np.abs(F[i] - ref) / ref))


def test_boys_stage_negative_argument_is_nan(torch):
    F = eri4.boys(3, dev(torch, np.array([-1.0, 2.0]))).cpu().numpy()
    assert np.isnan(F[0]).all() and np.isfinite(F[1]).all()


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 0), (2, 3), (4, 4), (6, 6), (7, 7), (6, 2)])
def test_hermite_e_stage(torch, la, lb):
    rng = np.random.default_rng(la * 10 + lb)
    n = 5
    za, zb = rng.uniform(0.05, 200, n), rng.uniform(0.05, 200, n)
    A, B = rng.uniform(0, 8, (n, 3)), rng.uniform(0, 8, (n, 3))
    E = eri4.hermite_e(la, lb, dev(torch, za), dev(torch, zb), dev(torch, A), dev(torch, B)).cpu().numpy()
    for i in range(n):
        ref = oracle.md4_etab(la, lb, za[i], zb[i], A[i], B[i])
        eps = 2.2e-16
        mag = _etab_magnitude(la, lb, za[i], zb[i], A[i], B[i], 0.0)
        # P - A and P - B carry an input rounding of a few ulps of |P| (the
        # oracle subtracts absolute positions); its first-order effect is the
        # growth of the magnitude recursion under that perturbation
        pert = _etab_magnitude(la, lb, za[i], zb[i], A[i], B[i], 4 * eps * (np.abs(A[i]) + np.abs(B[i]))) - mag
        bound = 4 * (la + lb + 1) * eps * mag + pert
        assert np.all(np.abs(E[i] - ref) <= bound + 1e-300)


def _etab_magnitude(la, lb, za, zb, A, B, delta):
    """The E recursions run on |P-A| + delta, |P-B| + delta: bounds every term."""
    zp = za + zb
    out = np.zeros((3, la + 1, lb + 1, la + lb + 1))
    delta = np.broadcast_to(delta, (3,))
    for ax in range(3):
        P = (za * A[ax] + zb * B[ax]) / zp
        pa, pb, h = abs(P - A[ax]) + delta[ax], abs(P - B[ax]) + delta[ax], 1.0 / (2 * zp)
        M = np.zeros((la + 1, lb + 1, la + lb + 2))
        M[0, 0, 0] = 1.0
        for a in range(la):
            for t in range(a + 2):
                M[a + 1, 0, t] = h * (M[a, 0, t - 1] if t else 0) + pa * M[a, 0, t] + (t + 1) * M[a, 0, t + 1]
        for a in range(la + 1):
            for b in range(lb):
                for t in range(a + b + 2):
                    M[a, b + 1, t] = h * (M[a, b, t - 1] if t else 0) + pb * M[a, b, t] + (t + 1) * M[a, b, t + 1]
        out[ax] = M[:, :, :la + lb + 1]
    return out


@pytest.mark.parametrize("L", [0, 1, 2, 5, 12, 16, 20, 24, 25, 26, 28])
def test_hermite_r_stage(torch, L):
    rng = np.random.default_rng(L)
    n = 4
    zp, zq = rng.uniform(0.1, 400, n), rng.uniform(0.1, 400, n)
    P, Q = rng.uniform(0, 8, (n, 3)), rng.uniform(0, 8, (n, 3))
    P[0] = Q[0]  # T = 0
    R = eri4.hermite_r(L, dev(torch, zp), dev(torch, zq), dev(torch, P), dev(torch, Q)).cpu().numpy()
    for i in range(n):
        ref = oracle.md4_rtuv(L, zp[i], zq[i], P[i], Q[i])
        mag = _rtuv_magnitude(L, zp[i], zq[i], P[i] - Q[i], oracle.boys(L, zp[i] * zq[i] / (zp[i] + zq[i]) * np.sum((P[i] - Q[i]) ** 2)))
        # a few ulps per recursion level of the size the terms reach (large T
        # makes the alternating terms of eq. (md1) cancel)
        assert np.all(np.abs(R[i] - ref) <= 4 * (L + 2) * 2.2e-16 * mag + 1e-300), (L, i)


def _rtuv_magnitude(L, zp, zq, X, F):
    """eq. (md1) run on |[0]^(m)| and |P-Q|: bounds the size of every term."""
    rho = zp * zq / (zp + zq)
    base = (2 * rho) ** np.arange(L + 1) * 2 * np.pi ** 2.5 / (zp * zq * np.sqrt(zp + zq)) * F
    X = np.abs(X)
    M = np.zeros((L + 1, L + 1, L + 1, L + 1))  # [t,u,v,m]
    M[0, 0, 0, :] = base
    for nn in range(1, L + 1):
        for t in range(nn + 1):
            for u in range(nn - t + 1):
                v = nn - t - u
                k = L - nn + 1
                if t > 0:
                    val = X[0] * M[t - 1, u, v, 1:k + 1] + (t - 1) * (M[t - 2, u, v, 1:k + 1] if t > 1 else 0)
                elif u > 0:
                    val = X[1] * M[t, u - 1, v, 1:k + 1] + (u - 1) * (M[t, u - 2, v, 1:k + 1] if u > 1 else 0)
                else:
                    val = X[2] * M[t, u, v - 1, 1:k + 1] + (v - 1) * (M[t, u, v - 2, 1:k + 1] if v > 1 else 0)
                M[t, u, v, :k] = val
    return M[:, :, :, 0]


# --------------------------------------------------------- full integrals

def test_ssss_matches_oracle(torch):
    b = inputs.class_batch((0, 0, 0, 0), 50, 3, seed=5)
    g = run_gpu(torch, b)
    o = oracle.eri_md4(b.ls, b.centers, b.exps, b.coefs, b.nprim)
    assert_quartets_close(g, o)


def test_all_low_classes_contracted(torch):
    rng = np.random.default_rng(11)
    for la in range(3):
        for lb in range(3):
            for lc in range(3):
                for ld in range(3):
                    ls = (la, lb, lc, ld)
                    b = inputs.class_batch(ls, 3, (1, 3), seed=int(rng.integers(1 << 30)), exp_range=(0.1, 20.0),
                                           box=3.0, kmax=4)
                    g = run_gpu(torch, b)
                    o = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
                    assert_quartets_close(g, o, label=ls)


def test_gggg_uncontracted_64_quartets(torch):
    """(gg|gg), l = 4, K = 1, 64 quartets, exponents [0.05, 50], 8-Bohr cube."""
    b = inputs.gggg_k1()
    g = run_gpu(torch, b)
    o = oracle.eri_md4(b.ls, b.centers, b.exps, b.coefs, b.nprim)
    assert_quartets_close(g, o, label="gggg")


@pytest.mark.parametrize("ls", [(4, 5, 6, 4), (6, 4, 5, 3), (0, 6, 6, 0), (6, 6, 0, 0), (3, 6, 2, 5), (5, 5, 5, 5),
                                (7, 0, 0, 7), (7, 6, 5, 7), (6, 7, 6, 7), (7, 7, 6, 6), (7, 7, 7, 7)])
def test_mixed_l_classes(torch, ls):
    b = inputs.class_batch(ls, 6, (1, 2), seed=sum(ls) * 7 + ls[0], exp_range=(0.05, 200.0), kmax=3)
    g = run_gpu(torch, b)
    o = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
    assert_quartets_close(g, o, label=ls)


def test_iiii_k1_full_batch_sampled(torch):
    """(ii|ii), K = 1, all 512 quartets on the GPU in one launch; 12 sampled
    quartets (first, last and random) checked against the oracle."""
    b = inputs.iiii(K=1)
    g = run_gpu(torch, b)
    idx = sorted({0, 511, *np.random.default_rng(1).choice(512, 10, replace=False).tolist()})
    s = inputs.subset(b, idx)
    o = oracle.eri_md4(b.ls, s.centers, s.exps, s.coefs, s.nprim)
    assert_quartets_close(g[idx], o, label="iiii")


def test_iiii_contracted_k2(torch):
    b = inputs.iiii(K=2, nq=4, seed=77)
    g = run_gpu(torch, b)
    o = oracle.eri_md4(b.ls, b.centers, b.exps, b.coefs, b.nprim)
    assert_quartets_close(g, o, label="iiii K2")


def test_gggg_k5(torch):
    b = inputs.class_batch((4, 4, 4, 4), 3, 5, seed=1013, exp_range=(0.05, 200.0))
    g = run_gpu(torch, b)
    o = oracle.eri_md4(b.ls, b.centers, b.exps, b.coefs, b.nprim)
    assert_quartets_close(g, o, label="gggg K5")


def test_coincident_centres(torch):
    ls = (4, 3, 4, 3)
    b = inputs.class_batch(ls, 3, 2, seed=3)
    b.centers[0, :, :] = b.centers[0, 0, :]          # A = B = C = D
    b.centers[1, 1, :] = b.centers[1, 0, :]          # A = B
    b.centers[2, 2:, :] = b.centers[2, 0, :]         # C = D = A
    g = run_gpu(torch, b)
    o = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
    assert_quartets_close(g, o, label="coincident")


def test_distant_pairs_large_T(torch):
    ls = (4, 4, 4, 4)
    b = inputs.class_batch(ls, 3, 1, seed=4, exp_range=(20.0, 200.0))
    b.centers[:, 2:, :] += 30.0     # T far beyond the interpolation grid
    g = run_gpu(torch, b)
    o = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
    assert_quartets_close(g, o, label="far")


def test_padded_kmax_and_per_shell_lengths(torch):
    ls = (4, 4, 5, 4)
    b = inputs.class_batch(ls, 5, (1, 3), seed=8, kmax=7)
    # padded entries are never read: poison them
    for q in range(b.nq):
        for s in range(4):
            b.exps[q, s, b.nprim[q, s]:] = np.nan
            b.coefs[q, s, b.nprim[q, s]:] = np.nan
    g = run_gpu(torch, b)
    o = oracle.eri_md4(ls, np.nan_to_num(b.centers), np.nan_to_num(b.exps, nan=1.0),
                       np.nan_to_num(b.coefs), b.nprim)
    assert_quartets_close(g, o, label="padded")


def test_invalid_contraction_length_gives_nan_only_there(torch):
    ls = (4, 4, 4, 4)
    b = inputs.class_batch(ls, 3, 1, seed=9, kmax=2)
    b.nprim[1, 2] = 3   # > kmax
    g = run_gpu(torch, b)
    assert np.isnan(g[1]).all()
    assert np.isfinite(g[0]).all() and np.isfinite(g[2]).all()


def test_empty_batch_is_a_no_op(torch):
    b = inputs.class_batch((4, 4, 4, 4), 1, 1, seed=1)
    z = torch.zeros(0, 4, 3, dtype=torch.float64, device="cuda")
    out = torch.zeros(0, 15, 15, 15, 15, dtype=torch.float64, device="cuda")
    eri4.batch((4, 4, 4, 4), z, torch.zeros(0, 4, 1, dtype=torch.float64, device="cuda"),
               torch.zeros(0, 4, 1, dtype=torch.float64, device="cuda"),
               torch.zeros(0, 4, dtype=torch.int32, device="cuda"), out=out)
    torch.cuda.synchronize()


def test_run_to_run_bitwise_determinism_and_stream(torch):
    b = inputs.class_batch((6, 5, 6, 5), 8, 2, seed=12)
    g1 = run_gpu(torch, b)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = eri4.batch(b.ls, dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs),
                         dev(torch, b.nprim, torch.int32), stream=s)
    s.synchronize()
    g2 = out.cpu().numpy()
    assert np.array_equal(g1, g2)


def test_bra_ket_swap_symmetry_at_full_size(torch):
    """(ab|cd) = (cd|ab) on all 512 (ii|ii) quartets, GPU only (a property
    that holds at any size)."""
    b = inputs.iiii(K=1)
    g = run_gpu(torch, b)
    sw = inputs.Batch(b.ls, b.centers[:, [2, 3, 0, 1]].copy(), b.exps[:, [2, 3, 0, 1]].copy(),
                      b.coefs[:, [2, 3, 0, 1]].copy(), b.nprim[:, [2, 3, 0, 1]].copy())
    h = run_gpu(torch, sw)
    ht = np.transpose(h, (0, 3, 4, 1, 2))
    for q in range(b.nq):
        assert np.abs(g[q] - ht[q]).max() <= 2 * TOL * max(np.abs(g[q]).max(), ZERO_SCALE)


def test_kkkk_contracted_k2(torch):
    """(kk|kk), l = 7, K = 2 per shell (16-row tiles, slab layout of R)."""
    b = inputs.class_batch((7, 7, 7, 7), 2, 2, seed=1005, exp_range=(0.05, 200.0))
    g = run_gpu(torch, b)
    o = oracle.eri_md4(b.ls, b.centers, b.exps, b.coefs, b.nprim)
    assert_quartets_close(g, o, label="kkkk K2")


def test_maximum_contraction_length(torch):
    """kmax = ERI4_MAX_K = 16: (ss|ss) with 16 primitives on every shell
    (65 536 primitive quartets per quartet) and (pd|sp) with mixed lengths."""
    assert eri4.ERI4_MAX_K == 16
    for b in (inputs.class_batch((0, 0, 0, 0), 2, 16, seed=31, exp_range=(0.1, 20.0)),
              inputs.class_batch((1, 2, 0, 1), 3, (1, 16), seed=32, exp_range=(0.1, 20.0), kmax=16)):
        assert b.kmax == 16
        g = run_gpu(torch, b)
        o = oracle.eri_md4(b.ls, b.centers, b.exps, b.coefs, b.nprim)
        assert_quartets_close(g, o, label=b.ls)


@pytest.mark.parametrize("l", [2, 3])
@pytest.mark.parametrize("K", [1, 5, 25])
def test_low_l_classes_at_the_papers_contraction_sizes(torch, l, K):
    """(dd|dd) and (ff|ff) with K = K_bra K_ket in {1, 5, 25}."""
    b = inputs.low_l_batch(l, K, 8, seed=300 + 10 * l + K)
    g = run_gpu(torch, b)
    o = oracle.eri_md4(b.ls, b.centers, b.exps, b.coefs, b.nprim)
    assert_quartets_close(g, o, label=(l, K))


def test_every_class_up_to_f_through_the_one_wave_kernel(torch):
    """Classes whose four shells all have l <= 3 run one quartet per wave
    (eri4_small.hip): all 256 of them, mixed contraction lengths, against the
    oracle; and against the 8-wave tile kernel (which plans use) on a mixed
    batch of them."""
    rng = np.random.default_rng(12)
    for la in range(4):
        for lb in range(4):
            for lc in range(4):
                for ld in range(4):
                    ls = (la, lb, lc, ld)
                    b = inputs.class_batch(ls, 2, (1, 3), seed=int(rng.integers(1 << 30)), exp_range=(0.05, 50.0),
                                           kmax=3)
                    g = run_gpu(torch, b)
                    o = oracle.eri_md4(ls, b.centers, b.exps, b.coefs, b.nprim)
                    assert_quartets_close(g, o, label=ls)
    m = inputs.uneven_batch(nq=120, seed=31, lvals=(0, 1, 2, 3), kmax=3)
    p = eri4.Plan(m.lq, m.nprim, m.kmax)
    gp = p.execute(dev(torch, m.centers), dev(torch, m.exps), dev(torch, m.coefs))
    torch.cuda.synchronize()
    gp = gp.cpu().numpy()
    off = p.offsets()
    for q in range(m.nq):
        s = inputs.subset(m, [q])
        gq = run_gpu(torch, s, ls=tuple(int(x) for x in m.lq[q]))[0]
        ref = gp[off[q]:off[q] + gq.size].reshape(gq.shape)
        assert np.abs(gq - ref).max() <= 1e-13 * max(np.abs(ref).max(), ZERO_SCALE), q
