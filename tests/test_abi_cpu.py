"""The C ABI library loads, exports what include/eri4.h declares, and rejects
bad arguments on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2307_03452_amd import eri4

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eri4.h")
STATUS_INVALID, STATUS_UNSUPPORTED = 1, 2


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eri4_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = eri4.lib()
    names = declared_functions()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(L, n), n
    assert sorted(eri4.EXPORTS) == names


def test_header_constants_match_binding():
    text = open(HEADER).read()
    for name in ("ERI4_MAX_L", "ERI4_MAX_K", "ERI4_MAX_BOYS_M"):
        v = int(re.search(r"#define\s+%s\s+(\d+)" % name, text).group(1))
        assert v == getattr(eri4, name)


def test_sizes():
    assert [eri4.ncart(l) for l in range(8)] == [1, 3, 6, 10, 15, 21, 28, 36]
    assert eri4.ncart(-1) == -1
    assert eri4.quartet_size(6, 6, 6, 6) == 28 ** 4
    assert eri4.quartet_size(4, 5, 6, 0) == 15 * 21 * 28
    assert eri4.quartet_size(-1, 0, 0, 0) == -1
    assert "gfx950" in eri4.version()


def _batch(la, lb, lc, ld, nq, kmax, ptr=1):
    p = ctypes.c_void_p(ptr) if ptr else None
    return eri4.lib().eri4_batch(la, lb, lc, ld, nq, p, p, p, p, kmax, p, None)


def test_batch_rejects_bad_arguments_on_host():
    L = eri4.lib()
    assert _batch(-1, 0, 0, 0, 1, 1) == STATUS_INVALID
    assert b"angular" in L.eri4_last_error()
    assert _batch(8, 0, 0, 0, 1, 1) == STATUS_UNSUPPORTED
    assert _batch(0, 0, 0, 0, -1, 1) == STATUS_INVALID
    assert _batch(0, 0, 0, 0, 1, 0) == STATUS_INVALID
    assert _batch(0, 0, 0, 0, 1, 17) == STATUS_INVALID
    assert _batch(4, 4, 4, 4, 5, 1, ptr=0) == STATUS_INVALID
    assert b"NULL" in L.eri4_last_error()
    # nothing to do: success without touching the device or the pointers
    assert _batch(4, 4, 4, 4, 0, 1, ptr=0) == 0


def test_stage_entry_points_reject_bad_arguments_on_host():
    L = eri4.lib()
    n = ctypes.c_void_p(None)
    assert L.eri4_boys(-1, 1, n, n, None) == STATUS_INVALID
    assert L.eri4_boys(29, 1, n, n, None) == STATUS_INVALID
    assert L.eri4_boys(4, 3, n, n, None) == STATUS_INVALID
    assert L.eri4_boys(4, 0, n, n, None) == 0
    assert L.eri4_hermite_r(29, 1, n, n, n, n, n, None) == STATUS_INVALID
    assert L.eri4_hermite_r(4, 1, n, n, n, n, n, None) == STATUS_INVALID
    assert L.eri4_hermite_e(8, 0, 1, n, n, n, n, n, None) == STATUS_INVALID
    assert L.eri4_hermite_e(2, 2, -1, n, n, n, n, n, None) == STATUS_INVALID


def test_errors_are_per_thread():
    import threading
    L = eri4.lib()
    assert _batch(-1, 0, 0, 0, 1, 1) == STATUS_INVALID
    seen = []
    t = threading.Thread(target=lambda: seen.append(L.eri4_last_error()))
    t.start()
    t.join()
    assert seen == [b""]
    assert L.eri4_last_error() != b""


def test_plan_create_rejects_bad_host_arrays_before_touching_a_device():
    import numpy as np
    L = eri4.lib()
    h = ctypes.c_void_p()
    lq = np.full((3, 4), 4, np.int32)
    npr = np.ones((3, 4), np.int32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert L.eri4_plan_create(None, 3, ptr(lq), ptr(npr), 1, 0) == STATUS_INVALID
    assert L.eri4_plan_create(ctypes.byref(h), -1, ptr(lq), ptr(npr), 1, 0) == STATUS_INVALID
    assert L.eri4_plan_create(ctypes.byref(h), 3, ptr(lq), ptr(npr), 0, 0) == STATUS_INVALID
    assert L.eri4_plan_create(ctypes.byref(h), 3, None, ptr(npr), 1, 0) == STATUS_INVALID
    bad = lq.copy(); bad[2, 1] = 8
    assert L.eri4_plan_create(ctypes.byref(h), 3, ptr(bad), ptr(npr), 1, 0) == STATUS_UNSUPPORTED
    bad[2, 1] = -1
    assert L.eri4_plan_create(ctypes.byref(h), 3, ptr(bad), ptr(npr), 1, 0) == STATUS_INVALID
    badn = npr.copy(); badn[1, 3] = 2
    assert L.eri4_plan_create(ctypes.byref(h), 3, ptr(lq), ptr(badn), 1, 0) == STATUS_INVALID
    assert b"contraction length" in L.eri4_last_error()
    assert L.eri4_plan_create(ctypes.byref(h), 3, ptr(lq), ptr(npr), 1, 7) == STATUS_INVALID
    assert b"precision" in L.eri4_last_error()
    assert h.value is None
    assert L.eri4_plan_output_size(None) == -1
    assert L.eri4_plan_execute(None, None, None, None, None, None) == STATUS_INVALID
    assert L.eri4_plan_destroy(None) == 0


def test_plan_create_tuned_rejects_bad_tile_tables_before_touching_a_device():
    import numpy as np
    L = eri4.lib()
    h = ctypes.c_void_p()
    lq = np.full((3, 4), 4, np.int32)
    npr = np.ones((3, 4), np.int32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)

    def create(entries, n=None):
        arr = eri4.tile_choices(entries)
        return L.eri4_plan_create_tuned(ctypes.byref(h), 3, ptr(lq), ptr(npr), 1, 0,
                                        ctypes.cast(arr, ctypes.c_void_p), len(entries) if n is None else n)

    good = {"l": (4, 4, 4, 4), "kq": (1, 1), "rows16": 2, "layout": "box2"}
    assert create([dict(good, rows16=3)]) == STATUS_INVALID and b"rows16" in L.eri4_last_error()
    assert create([dict(good, rows16=8)]) == STATUS_INVALID and b"rows16" in L.eri4_last_error()
    assert create([dict(good, layout=7)]) == STATUS_INVALID and b"layout" in L.eri4_last_error()
    assert create([dict(good, kq=(5, 2))]) == STATUS_INVALID and b"kq_min" in L.eri4_last_error()
    assert create([dict(good, l=(4, 4, 8, 4))]) == STATUS_INVALID and b"angular momentum" in L.eri4_last_error()
    assert create([good], n=-1) == STATUS_INVALID
    assert L.eri4_plan_create_tuned(ctypes.byref(h), 3, ptr(lq), ptr(npr), 1, 0, None, 2) == STATUS_INVALID
    assert h.value is None


def test_plan_create_pairs_rejects_bad_host_arrays_before_touching_a_device():
    import numpy as np
    L = eri4.lib()
    h = ctypes.c_void_p()
    bl, bn = np.full((3, 2), 4, np.int32), np.ones((3, 2), np.int32)
    kl, kn = np.full((2, 2), 5, np.int32), np.ones((2, 2), np.int32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)

    def create(nbra=3, bl=bl, bn=bn, nket=2, kl=kl, kn=kn, kmax=1, prec=0, plan=True, fn=0):
        return L.eri4_plan_create_pairs(ctypes.byref(h) if plan else None, nbra, ptr(bl) if bl is not None else None,
                                        ptr(bn), nket, ptr(kl) if kl is not None else None, ptr(kn), kmax, prec, fn,
                                        None, 0)

    assert create(plan=False) == STATUS_INVALID
    assert create(nbra=-1) == STATUS_INVALID and b"negative" in L.eri4_last_error()
    assert create(nbra=1 << 16, nket=1 << 16) == STATUS_INVALID and b"2^31" in L.eri4_last_error()
    assert create(bl=None) == STATUS_INVALID and b"NULL" in L.eri4_last_error()
    assert create(kl=None) == STATUS_INVALID
    bad = kl.copy(); bad[1, 0] = 8
    assert create(kl=bad) == STATUS_UNSUPPORTED
    badn = bn.copy(); badn[2, 1] = 3
    assert create(bn=badn, kmax=2) == STATUS_INVALID and b"contraction length" in L.eri4_last_error()
    assert create(prec=5) == STATUS_INVALID and b"precision" in L.eri4_last_error()
    assert create(fn=2) == STATUS_INVALID and b"functions" in L.eri4_last_error()
    assert create(fn=1, prec=1) == STATUS_INVALID and b"FP64" in L.eri4_last_error()
    assert h.value is None
    assert L.eri4_plan_execute_pairs(None, None, None, None, None, None, None, None, 0, None, None) == STATUS_INVALID
    assert L.eri4_plan_work_size(None) == -1


def test_pair_list_expansion_is_bra_major():
    import numpy as np
    from paper_2307_03452_amd import inputs
    bra, ket = inputs.pair_list(3, 11, kmax=3), inputs.pair_list(4, 12, kmax=3)
    b = inputs.expand_pairs(bra, ket)
    assert b.nq == 12 and b.lq.shape == (12, 4) and b.exps.shape == (12, 4, 3)
    for i in range(3):
        for j in range(4):
            q = i * 4 + j
            assert np.array_equal(b.lq[q], np.r_[bra.l[i], ket.l[j]])
            assert np.array_equal(b.nprim[q], np.r_[bra.nprim[i], ket.nprim[j]])
            assert np.array_equal(b.centers[q], np.r_[bra.centers[i], ket.centers[j]])
            assert np.array_equal(b.coefs[q], np.r_[bra.coefs[i], ket.coefs[j]])
    assert set(np.unique(bra.l)) <= {4, 5, 6} and bra.nprim.min() >= 1 and bra.nprim.max() <= 3


def test_uneven_batch_recipe():
    import numpy as np
    from paper_2307_03452_amd import inputs
    cls, p = inputs.zipf_classes()
    assert len(cls) == 81 and cls[0] == (4, 4, 4, 4) and cls[-1] == (6, 6, 6, 6)
    assert abs(p[0] - 0.2843) < 1e-3 and abs(p.sum() - 1) < 1e-12
    b = inputs.uneven_batch(nq=500, seed=3)
    assert b.lq.shape == (500, 4) and b.nprim.min() >= 1 and b.nprim.max() <= 8
    # every contracted shell's x^l component has unit norm (same check as the single-class generator)
    for q in range(0, 500, 97):
        for s in range(4):
            k, l = int(b.nprim[q, s]), int(b.lq[q, s])
            z = b.exps[q, s, :k]; c = b.coefs[q, s, :k]
            zz = z[:, None] + z[None, :]
            S = inputs._dfact(2 * l - 1) / (2 * zz) ** l * (np.pi / zz) ** 1.5
            assert abs(c @ S @ c - 1.0) < 1e-12


def test_library_solid_coefficients_match_the_oracles():
    """The library writes its own Cartesian-to-solid table (host C++); it must
    agree with the oracle's exact-rational one for every l."""
    import numpy as np
    from oracle import solid
    for l in range(8):
        C = eri4.solid_coefficients(l)
        ref = solid.solid_matrix(l)
        assert C.shape == ref.shape
        assert np.array_equal(C != 0, ref != 0), l
        assert np.abs(C - ref).max() <= 4e-16 * np.abs(ref).max(), l
    L = eri4.lib()
    assert L.eri4_solid_coefficients(8, ctypes.c_void_p(1)) == STATUS_INVALID
    assert L.eri4_solid_coefficients(2, None) == STATUS_INVALID


def test_solid_work_size_and_host_errors():
    import numpy as np
    L = eri4.lib()
    # (ii|ii), K=1: H for one bra pair (13 x 13 = 169 rows, padded to whole tiles)
    # and one ket pair (169 columns, padded to 16), times the padded Hermite counts
    n1 = eri4.solid_work_size((6, 6, 6, 6), 1, 1)
    assert n1 > 0 and eri4.solid_work_size((6, 6, 6, 6), 1, 10) == 10 * n1
    assert eri4.solid_work_size((6, 6, 6, 6), 2, 1) == 4 * n1
    nk = 11 * 16 * 456
    assert (n1 - nk) % (16 * 456) == 0 and (n1 - nk) // (16 * 456) >= 11
    assert L.eri4_solid_work_size(8, 0, 0, 0, 1, 1) == -1
    assert L.eri4_solid_work_size(0, 0, 0, 0, 0, 1) == -1
    assert L.eri4_solid_work_size(0, 0, 0, 0, 1, -1) == -1
    p = ctypes.c_void_p(16)  # never dereferenced: the calls fail on the host first
    assert L.eri4_batch_solid(2, 2, 2, 2, 4, p, p, p, p, 1, p, 1, p, None) == STATUS_INVALID
    assert b"workspace" in L.eri4_last_error()
    assert L.eri4_batch_solid(2, 2, 2, 2, 4, p, p, p, p, 1, None, 10 ** 9, p, None) == STATUS_INVALID
    assert L.eri4_batch_solid(2, 2, 9, 2, 4, p, p, p, p, 1, p, 10 ** 9, p, None) == STATUS_UNSUPPORTED
    assert L.eri4_batch_solid(2, 2, 2, 2, 0, None, None, None, None, 1, None, 0, None, None) == 0


def test_coulomb_work_size_and_host_errors():
    L = eri4.lib()
    n1 = eri4.coulomb_work_size((6, 6, 6, 6), 1, 1)
    # per primitive pair slot: dket (455 ket Hermite functions in 29 blocks of
    # 16) and one bra pair's J rows (28 x 28)
    assert n1 == 16 * 29 + 28 * 28
    assert eri4.coulomb_work_size((6, 6, 6, 6), 3, 2) == 2 * 9 * n1
    assert L.eri4_coulomb_work_size(0, 0, 0, 8, 1, 1) == -1
    p = ctypes.c_void_p(16)  # never dereferenced: the calls fail on the host first
    assert L.eri4_batch_coulomb(2, 2, 2, 2, 4, p, p, p, p, 1, p, p, 1, p, None) == STATUS_INVALID
    assert b"workspace" in L.eri4_last_error()
    assert L.eri4_batch_coulomb(2, 2, 2, 2, 4, p, p, p, p, 1, None, p, 10 ** 6, p, None) == STATUS_INVALID
    assert L.eri4_batch_coulomb(2, 2, 2, 2, 0, None, None, None, None, 1, None, None, 0, None, None) == 0


def test_coulomb_plan_create_rejects_bad_host_arrays():
    import numpy as np
    L = eri4.lib()
    h = ctypes.c_void_p()
    bl, bn = np.full((2, 2), 4, np.int32), np.ones((2, 2), np.int32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert L.eri4_plan_create_coulomb(None, 2, ptr(bl), ptr(bn), 2, ptr(bl), ptr(bn), 1) == STATUS_INVALID
    assert L.eri4_plan_create_coulomb(ctypes.byref(h), -2, ptr(bl), ptr(bn), 2, ptr(bl), ptr(bn), 1) == STATUS_INVALID
    assert L.eri4_plan_create_coulomb(ctypes.byref(h), 2, None, ptr(bn), 2, ptr(bl), ptr(bn), 1) == STATUS_INVALID
    bad = bl.copy(); bad[1, 1] = 9
    assert L.eri4_plan_create_coulomb(ctypes.byref(h), 2, ptr(bad), ptr(bn), 2, ptr(bl), ptr(bn), 1) == STATUS_UNSUPPORTED
    assert h.value is None
    assert L.eri4_plan_execute_coulomb(None, *([None] * 7), None, 0, None, None) == STATUS_INVALID
