"""Thin Python binding of liberi4.so (the gfx950 HIP library).

Argument marshalling only: every step of the computation runs in the library's
kernels.  Device buffers are torch tensors on the current ROCm device; the
stream is torch's current stream unless one is given.  The functions mirror
the C entry points declared in include/eri4.h.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# ERI4_LIBRARY may name another build of the same library (the stage-timer
# variant, liberi4_stages.so); the default is the in-tree liberi4.so
LIB_PATH = os.environ.get("ERI4_LIBRARY") or os.path.join(HERE, "liberi4.so")

ERI4_MAX_L = 7
ERI4_MAX_K = 16
ERI4_MAX_BOYS_M = 28

# eri4_precision: arithmetic of the two transforms of a plan
PRECISION = {"fp64": 0, "fp32": 1}
# eri4_functions: basis functions of a pair-list plan's output
FUNCTIONS = {"cartesian": 0, "solid": 1}
# eri4_layout: where the Hermite integrals of a tile live in LDS
LAYOUT = {"box": 0, "slab": 1, "box2": 2}
# the tile table tuned on MI355X (gfx950) by autotune.py, read by the library
TUNE_FILE = os.path.join(HERE, "tune_gfx950.txt")


class TileChoice(ctypes.Structure):
    """eri4_tile_choice: tile height and R layout for the quartets of class l
    whose product of the four contraction lengths is in [kq_min, kq_max]."""
    _fields_ = [("l", ctypes.c_int32 * 4), ("kq_min", ctypes.c_int32), ("kq_max", ctypes.c_int32),
                ("rows16", ctypes.c_int32), ("layout", ctypes.c_int32)]


def read_tile_table(path):
    """The entries of a tile table file (format: eri4_plan_create_tunefile in
    include/eri4.h) as tile-choice dicts, for calls that take them as a list."""
    out = []
    with open(path) as f:
        for line in f:
            w = line.split()
            if not w or w[0].startswith("#") or w[0] == "arch":
                continue
            out.append({"l": [int(x) for x in w[:4]], "kq": [int(w[4]), int(w[5])], "rows16": int(w[6]),
                        "layout": w[7]})
    return out


def tile_choices(entries):
    """ctypes array of TileChoice from dicts {"l": (la,lb,lc,ld), "kq": (min, max),
    "rows16": 1|2, "layout": "box"|"slab"|"box2"}."""
    arr = (TileChoice * len(entries))()
    for i, e in enumerate(entries):
        arr[i].l[:] = [int(x) for x in e["l"]]
        arr[i].kq_min, arr[i].kq_max = int(e["kq"][0]), int(e["kq"][1])
        arr[i].rows16 = int(e["rows16"])
        arr[i].layout = LAYOUT[e["layout"]] if isinstance(e["layout"], str) else int(e["layout"])
    return arr

STATUS = {0: "ERI4_SUCCESS", 1: "ERI4_ERROR_INVALID_ARGUMENT", 2: "ERI4_ERROR_UNSUPPORTED",
          3: "ERI4_ERROR_OUT_OF_MEMORY", 4: "ERI4_ERROR_HIP", 5: "ERI4_ERROR_INTERNAL"}

# every symbol include/eri4.h declares
EXPORTS = ("eri4_ncart", "eri4_quartet_size", "eri4_last_error", "eri4_version", "eri4_init",
           "eri4_batch", "eri4_plan_create", "eri4_plan_create_tuned", "eri4_plan_output_size", "eri4_plan_output_offsets",
           "eri4_plan_execute", "eri4_plan_destroy", "eri4_plan_create_pairs", "eri4_plan_execute_pairs", "eri4_plan_work_size",
           "eri4_plan_create_coulomb", "eri4_plan_execute_coulomb", "eri4_plan_create_tunefile",
           "eri4_boys", "eri4_hermite_r", "eri4_hermite_e", "eri4_solid_coefficients", "eri4_solid_work_size",
           "eri4_batch_solid", "eri4_coulomb_work_size", "eri4_batch_coulomb", "eri4_exchange_work_size",
           "eri4_batch_exchange", "eri4_static_scratch_bytes",
           "eri4_batch_coulomb_static", "eri4_plan_create_solid", "eri4_plan_execute_solid")

_lib = None


class Eri4Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """Load liberi4.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2307_03452_amd.build`; "
                               "there is no non-HIP fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.eri4_ncart.argtypes = [c_int]
        L.eri4_ncart.restype = c_int
        L.eri4_quartet_size.argtypes = [c_int] * 4
        L.eri4_quartet_size.restype = i64
        L.eri4_last_error.restype = ctypes.c_char_p
        L.eri4_version.restype = ctypes.c_char_p
        L.eri4_init.restype = c_int
        L.eri4_batch.argtypes = [c_int] * 4 + [i64, vp, vp, vp, vp, c_int, vp, vp]
        L.eri4_batch.restype = c_int
        L.eri4_solid_coefficients.argtypes = [c_int, vp]
        L.eri4_solid_coefficients.restype = c_int
        L.eri4_solid_work_size.argtypes = [c_int] * 5 + [i64]
        L.eri4_solid_work_size.restype = i64
        L.eri4_batch_solid.argtypes = [c_int] * 4 + [i64, vp, vp, vp, vp, c_int, vp, i64, vp, vp]
        L.eri4_batch_solid.restype = c_int
        L.eri4_coulomb_work_size.argtypes = [c_int] * 5 + [i64]
        L.eri4_coulomb_work_size.restype = i64
        L.eri4_batch_coulomb.argtypes = [c_int] * 4 + [i64, vp, vp, vp, vp, c_int, vp, vp, i64, vp, vp]
        L.eri4_batch_coulomb.restype = c_int
        L.eri4_exchange_work_size.argtypes = [c_int] * 5 + [i64]
        L.eri4_exchange_work_size.restype = i64
        L.eri4_batch_exchange.argtypes = [c_int] * 4 + [i64, vp, vp, vp, vp, c_int, vp, vp, i64, vp, vp]
        L.eri4_batch_exchange.restype = c_int
        L.eri4_static_scratch_bytes.argtypes = []
        L.eri4_static_scratch_bytes.restype = i64
        L.eri4_batch_coulomb_static.argtypes = [c_int] * 4 + [i64, vp, vp, vp, vp, c_int, vp, vp, vp]
        L.eri4_batch_coulomb_static.restype = c_int
        L.eri4_plan_create.argtypes = [ctypes.POINTER(vp), i64, vp, vp, c_int, c_int]
        L.eri4_plan_create.restype = c_int
        L.eri4_plan_create_tuned.argtypes = [ctypes.POINTER(vp), i64, vp, vp, c_int, c_int, vp, c_int]
        L.eri4_plan_create_tuned.restype = c_int
        L.eri4_plan_create_tunefile.argtypes = [ctypes.POINTER(vp), i64, vp, vp, c_int, c_int, ctypes.c_char_p]
        L.eri4_plan_create_tunefile.restype = c_int
        L.eri4_plan_output_size.argtypes = [vp]
        L.eri4_plan_output_size.restype = i64
        L.eri4_plan_output_offsets.argtypes = [vp, vp]
        L.eri4_plan_output_offsets.restype = c_int
        L.eri4_plan_execute.argtypes = [vp, vp, vp, vp, vp, vp]
        L.eri4_plan_execute.restype = c_int
        L.eri4_plan_destroy.argtypes = [vp]
        L.eri4_plan_destroy.restype = c_int
        L.eri4_plan_create_pairs.argtypes = [ctypes.POINTER(vp), i64, vp, vp, i64, vp, vp, c_int, c_int, c_int, vp,
                                             c_int]
        L.eri4_plan_create_pairs.restype = c_int
        L.eri4_plan_create_coulomb.argtypes = [ctypes.POINTER(vp), i64, vp, vp, i64, vp, vp, c_int]
        L.eri4_plan_create_coulomb.restype = c_int
        L.eri4_plan_execute_coulomb.argtypes = [vp] * 8 + [vp, i64, vp, vp]
        L.eri4_plan_execute_coulomb.restype = c_int
        L.eri4_plan_work_size.argtypes = [vp]
        L.eri4_plan_work_size.restype = i64
        L.eri4_plan_execute_pairs.argtypes = [vp] * 7 + [vp, i64, vp, vp]
        L.eri4_plan_execute_pairs.restype = c_int
        L.eri4_plan_create_solid.argtypes = [ctypes.POINTER(vp), i64, vp, vp, c_int, ctypes.c_char_p]
        L.eri4_plan_create_solid.restype = c_int
        L.eri4_plan_execute_solid.argtypes = [vp] * 5 + [i64, vp, vp]
        L.eri4_plan_execute_solid.restype = c_int
        L.eri4_boys.argtypes = [c_int, i64, vp, vp, vp]
        L.eri4_boys.restype = c_int
        L.eri4_hermite_r.argtypes = [c_int, i64, vp, vp, vp, vp, vp, vp]
        L.eri4_hermite_r.restype = c_int
        L.eri4_hermite_e.argtypes = [c_int, c_int, i64, vp, vp, vp, vp, vp, vp]
        L.eri4_hermite_e.restype = c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise Eri4Error(st, lib().eri4_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype_name: str):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensors expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensors expected")
    if str(t.dtype) != "torch." + dtype_name:
        raise ValueError(f"{dtype_name} tensor expected, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _check_shells(centers, exps, coefs, nprim=None):
    """Shapes of per-quartet shell arrays: centers [nq,4,3], exps/coefs
    [nq,4,kmax], nprim [nq,4]; returns (nq, kmax)."""
    nq = centers.shape[0]
    if tuple(centers.shape) != (nq, 4, 3) or exps.dim() != 3 or tuple(exps.shape[:2]) != (nq, 4):
        raise ValueError("centers must be [nq,4,3] and exps [nq,4,kmax]")
    kmax = exps.shape[2]
    if tuple(coefs.shape) != (nq, 4, kmax):
        raise ValueError("coefs must have the shape of exps")
    if nprim is not None and tuple(nprim.shape) != (nq, 4):
        raise ValueError("nprim must be [nq,4]")
    return nq, kmax


def _check_out(t, n, what="output"):
    if t.numel() < n:
        raise ValueError(f"{what} buffer holds {t.numel()} doubles, {n} needed")


def ncart(l: int) -> int:
    return lib().eri4_ncart(int(l))


def quartet_size(la, lb, lc, ld) -> int:
    return lib().eri4_quartet_size(int(la), int(lb), int(lc), int(ld))


def version() -> str:
    return lib().eri4_version().decode()


def init():
    _check(lib().eri4_init())


def batch(ls, centers, exps, coefs, nprim, out=None, stream=None):
    """(ab|cd) for one class ls = (la, lb, lc, ld).

    centers float64 [nq,4,3], exps/coefs float64 [nq,4,kmax], nprim int32 [nq,4]
    (all device tensors); returns out float64 [nq, Na, Nb, Nc, Nd].
    """
    import torch
    la, lb, lc, ld = (int(x) for x in ls)
    nq, kmax = _check_shells(centers, exps, coefs, nprim)
    if out is None:
        out = torch.empty((nq, ncart(la), ncart(lb), ncart(lc), ncart(ld)), dtype=torch.float64,
                          device=centers.device)
    _check_out(out, nq * ncart(la) * ncart(lb) * ncart(lc) * ncart(ld))
    _check(lib().eri4_batch(la, lb, lc, ld, nq, _ptr(centers, "float64"), _ptr(exps, "float64"),
                            _ptr(coefs, "float64"), _ptr(nprim, "int32"), kmax, _ptr(out, "float64"),
                            _stream(stream)))
    return out


def nsolid(l: int) -> int:
    return 2 * int(l) + 1


def solid_coefficients(l: int):
    """The library's C[2l+1][ncart(l)] (host numpy array): coefficient of each
    Cartesian component in each real solid harmonic, rows m = -l..l."""
    import numpy as np
    C = np.zeros((nsolid(l), ncart(l)))
    _check(lib().eri4_solid_coefficients(int(l), C.ctypes.data_as(ctypes.c_void_p)))
    return C


def solid_work_size(ls, kmax: int, nq: int) -> int:
    """Doubles of workspace eri4_batch_solid needs to run nq quartets in one pass."""
    n = lib().eri4_solid_work_size(*(int(x) for x in ls), int(kmax), int(nq))
    if n < 0:
        raise ValueError("bad class or sizes")
    return n


def batch_solid(ls, centers, exps, coefs, nprim, work=None, out=None, stream=None):
    """(ab|cd) over real solid harmonics for one class: out float64
    [nq, 2la+1, 2lb+1, 2lc+1, 2ld+1].  work: float64 device scratch for the H
    matrices (default: enough for one pass over all quartets)."""
    import torch
    la, lb, lc, ld = (int(x) for x in ls)
    nq, kmax = _check_shells(centers, exps, coefs, nprim)
    if out is None:
        out = torch.empty((nq, nsolid(la), nsolid(lb), nsolid(lc), nsolid(ld)), dtype=torch.float64,
                          device=centers.device)
    _check_out(out, nq * nsolid(la) * nsolid(lb) * nsolid(lc) * nsolid(ld))
    if work is None:
        work = torch.empty(max(1, solid_work_size(ls, kmax, nq)), dtype=torch.float64, device=centers.device)
    _check(lib().eri4_batch_solid(la, lb, lc, ld, nq, _ptr(centers, "float64"), _ptr(exps, "float64"),
                                  _ptr(coefs, "float64"), _ptr(nprim, "int32"), kmax, _ptr(work, "float64"),
                                  work.numel(), _ptr(out, "float64"), _stream(stream)))
    return out


def coulomb_work_size(ls, kmax: int, nq: int) -> int:
    """Doubles of workspace eri4_batch_coulomb needs to run nq quartets in one pass."""
    n = lib().eri4_coulomb_work_size(*(int(x) for x in ls), int(kmax), int(nq))
    if n < 0:
        raise ValueError("bad class or sizes")
    return n


def batch_coulomb(ls, centers, exps, coefs, nprim, dens, work=None, out=None, stream=None):
    """J_ab = sum_cd (ab|cd) D_cd for every quartet of one class, without
    forming (ab|cd): dens float64 [nq, Nc, Nd] (device), returns float64
    [nq, Na, Nb]."""
    import torch
    la, lb, lc, ld = (int(x) for x in ls)
    nq, kmax = _check_shells(centers, exps, coefs, nprim)
    if out is None:
        out = torch.empty((nq, ncart(la), ncart(lb)), dtype=torch.float64, device=centers.device)
    _check_out(out, nq * ncart(la) * ncart(lb))
    _check_out(dens, nq * ncart(lc) * ncart(ld), "density")
    if work is None:
        work = torch.empty(max(1, coulomb_work_size(ls, kmax, nq)), dtype=torch.float64, device=centers.device)
    _check(lib().eri4_batch_coulomb(la, lb, lc, ld, nq, _ptr(centers, "float64"), _ptr(exps, "float64"),
                                    _ptr(coefs, "float64"), _ptr(nprim, "int32"), kmax, _ptr(dens, "float64"),
                                    _ptr(work, "float64"), work.numel(), _ptr(out, "float64"), _stream(stream)))
    return out


def exchange_work_size(ls, kmax: int, nq: int) -> int:
    """Doubles of workspace eri4_batch_exchange needs to run nq quartets in one pass."""
    n = lib().eri4_exchange_work_size(*(int(x) for x in ls), int(kmax), int(nq))
    if n < 0:
        raise ValueError("bad class or sizes")
    return n


def batch_exchange(ls, centers, exps, coefs, nprim, dens, work=None, out=None, stream=None):
    """K_ac = sum_bd (ab|cd) D_bd for every quartet of one class, without
    forming (ab|cd): dens float64 [nq, Nb, Nd] (device), returns float64
    [nq, Na, Nc]."""
    import torch
    la, lb, lc, ld = (int(x) for x in ls)
    nq, kmax = _check_shells(centers, exps, coefs, nprim)
    if out is None:
        out = torch.empty((nq, ncart(la), ncart(lc)), dtype=torch.float64, device=centers.device)
    _check_out(out, nq * ncart(la) * ncart(lc))
    _check_out(dens, nq * ncart(lb) * ncart(ld), "density")
    if work is None:
        work = torch.empty(max(1, exchange_work_size(ls, kmax, nq)), dtype=torch.float64, device=centers.device)
    _check(lib().eri4_batch_exchange(la, lb, lc, ld, nq, _ptr(centers, "float64"), _ptr(exps, "float64"),
                                     _ptr(coefs, "float64"), _ptr(nprim, "int32"), kmax, _ptr(dens, "float64"),
                                     _ptr(work, "float64"), work.numel(), _ptr(out, "float64"), _stream(stream)))
    return out


def static_scratch_bytes() -> int:
    """Bytes of the static device array eri4_batch_coulomb_static works in."""
    return int(lib().eri4_static_scratch_bytes())


def batch_coulomb_static(ls, centers, exps, coefs, nprim, dens, out, stream=None):
    """eri4_batch_coulomb_static: batch_coulomb with no workspace and no
    device allocation in the library call (the caller passes out, float64
    [nq, Na, Nb]; init() must have run on the device)."""
    la, lb, lc, ld = (int(x) for x in ls)
    nq, kmax = _check_shells(centers, exps, coefs, nprim)
    _check_out(out, nq * ncart(la) * ncart(lb))
    _check_out(dens, nq * ncart(lc) * ncart(ld), "density")
    _check(lib().eri4_batch_coulomb_static(la, lb, lc, ld, nq, _ptr(centers, "float64"), _ptr(exps, "float64"),
                                           _ptr(coefs, "float64"), _ptr(nprim, "int32"), kmax,
                                           _ptr(dens, "float64"), _ptr(out, "float64"), _stream(stream)))
    return out


def boys(mmax, T, F=None, stream=None):
    import torch
    n = T.shape[0]
    if F is None:
        F = torch.empty((n, mmax + 1), dtype=torch.float64, device=T.device)
    _check(lib().eri4_boys(int(mmax), n, _ptr(T, "float64"), _ptr(F, "float64"), _stream(stream)))
    return F


def hermite_r(L, zp, zq, P, Q, R=None, stream=None):
    import torch
    n = zp.shape[0]
    if R is None:
        R = torch.empty((n, L + 1, L + 1, L + 1), dtype=torch.float64, device=zp.device)
    _check(lib().eri4_hermite_r(int(L), n, _ptr(zp, "float64"), _ptr(zq, "float64"), _ptr(P, "float64"),
                                _ptr(Q, "float64"), _ptr(R, "float64"), _stream(stream)))
    return R


def hermite_e(la, lb, za, zb, A, B, E=None, stream=None):
    import torch
    n = za.shape[0]
    if E is None:
        E = torch.empty((n, 3, la + 1, lb + 1, la + lb + 1), dtype=torch.float64, device=za.device)
    _check(lib().eri4_hermite_e(int(la), int(lb), n, _ptr(za, "float64"), _ptr(zb, "float64"),
                                _ptr(A, "float64"), _ptr(B, "float64"), _ptr(E, "float64"), _stream(stream)))
    return E


class Plan:
    """A mixed-class batch computed by one persistent launch (eri4_plan_*).

    lq, nprim: host int32 arrays [nq, 4] (angular momenta, contraction lengths).
    precision: "fp64" or "fp32", the arithmetic of the two transforms.
    tiles: optional tile choices (see tile_choices), e.g. an autotuner's table;
    tune_file: or the path of a tile table file the library reads itself
    (eri4_plan_create_tunefile; TUNE_FILE is the one tuned here).
    """

    def __init__(self, lq, nprim, kmax: int, precision: str = "fp64", tiles=None, tune_file=None):
        import numpy as np
        self._lq = np.ascontiguousarray(lq, dtype=np.int32)
        self._np = np.ascontiguousarray(nprim, dtype=np.int32)
        assert self._lq.shape == self._np.shape and self._lq.ndim == 2 and self._lq.shape[1] == 4
        self.nq = self._lq.shape[0]
        self.kmax = int(kmax)
        self.precision = precision
        h = ctypes.c_void_p()
        if tune_file is not None:
            if tiles:
                raise ValueError("give tiles or tune_file, not both")
            _check(lib().eri4_plan_create_tunefile(
                ctypes.byref(h), self.nq, self._lq.ctypes.data_as(ctypes.c_void_p),
                self._np.ctypes.data_as(ctypes.c_void_p), self.kmax,
                PRECISION[precision] if isinstance(precision, str) else int(precision), str(tune_file).encode()))
            self._h = h
            return
        arr = tile_choices(tiles) if tiles else None
        _check(lib().eri4_plan_create_tuned(
            ctypes.byref(h), self.nq, self._lq.ctypes.data_as(ctypes.c_void_p),
            self._np.ctypes.data_as(ctypes.c_void_p), self.kmax,
            PRECISION[precision] if isinstance(precision, str) else int(precision),
            ctypes.cast(arr, ctypes.c_void_p) if arr is not None else None, len(arr) if arr is not None else 0))
        self._h = h

    @property
    def output_size(self) -> int:
        return lib().eri4_plan_output_size(self._h)

    def offsets(self):
        import numpy as np
        off = np.zeros(self.nq, dtype=np.int64)
        _check(lib().eri4_plan_output_offsets(self._h, off.ctypes.data_as(ctypes.c_void_p)))
        return off

    def execute(self, centers, exps, coefs, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.output_size, dtype=torch.float64, device=centers.device)
        if out.numel() < self.output_size:
            raise ValueError("output buffer too small")
        if exps.shape[2] != self.kmax or centers.shape[0] != self.nq:
            raise ValueError("inputs do not match the plan")
        _check(lib().eri4_plan_execute(self._h, _ptr(centers, "float64"), _ptr(exps, "float64"),
                                       _ptr(coefs, "float64"), _ptr(out, "float64"), _stream(stream)))
        return out

    def destroy(self):
        if getattr(self, "_h", None):
            lib().eri4_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class SolidPlan(Plan):
    """A mixed-class batch over real solid harmonics (eri4_plan_*_solid): host
    int32 arrays lq, nprim [nq, 4] as Plan, FP64 transforms, an optional tile
    table file.  execute() takes the device arrays of Plan.execute and a
    float64 device workspace of work_size doubles (allocated if not given);
    quartet q's [2la+1][2lb+1][2lc+1][2ld+1] block starts at offsets()[q]."""

    def __init__(self, lq, nprim, kmax: int, tune_file=None):
        import numpy as np
        self._lq = np.ascontiguousarray(lq, dtype=np.int32)
        self._np = np.ascontiguousarray(nprim, dtype=np.int32)
        assert self._lq.shape == self._np.shape and self._lq.ndim == 2 and self._lq.shape[1] == 4
        self.nq = self._lq.shape[0]
        self.kmax = int(kmax)
        self.precision = "fp64"
        h = ctypes.c_void_p()
        _check(lib().eri4_plan_create_solid(
            ctypes.byref(h), self.nq, self._lq.ctypes.data_as(ctypes.c_void_p),
            self._np.ctypes.data_as(ctypes.c_void_p), self.kmax,
            str(tune_file).encode() if tune_file is not None else None))
        self._h = h

    @property
    def work_size(self) -> int:
        return lib().eri4_plan_work_size(self._h)

    def execute(self, centers, exps, coefs, out=None, work=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.output_size, dtype=torch.float64, device=centers.device)
        if work is None:
            work = torch.empty(max(1, self.work_size), dtype=torch.float64, device=centers.device)
        if out.numel() < self.output_size:
            raise ValueError("output buffer too small")
        if work.numel() < self.work_size:
            raise ValueError("workspace too small")
        if (tuple(centers.shape) != (self.nq, 4, 3) or tuple(exps.shape) != (self.nq, 4, self.kmax)
                or tuple(coefs.shape) != (self.nq, 4, self.kmax)):
            raise ValueError("inputs do not match the plan")
        _check(lib().eri4_plan_execute_solid(
            self._h, _ptr(centers, "float64"), _ptr(exps, "float64"), _ptr(coefs, "float64"),
            _ptr(work, "float64"), work.numel(), _ptr(out, "float64"), _stream(stream)))
        return out


class PairPlan(Plan):
    """Every bra shell pair with every ket shell pair (eri4_plan_*_pairs).

    bra_l, bra_nprim: host int32 [nbra, 2]; ket_l, ket_nprim: host int32 [nket, 2].
    Quartet (i, j) is bra pair i with ket pair j, at index q = i * nket + j of
    offsets().  execute() takes the device lists: centers float64 [n, 2, 3],
    exps / coefs float64 [n, 2, kmax] for the bra and the ket side.
    functions="solid": integrals over real solid harmonics; execute() then needs
    a float64 device workspace of work_size doubles (allocated if not given).
    """

    def __init__(self, bra_l, bra_nprim, ket_l, ket_nprim, kmax: int, precision: str = "fp64", tiles=None,
                 functions: str = "cartesian"):
        import numpy as np
        bl, bn = (np.ascontiguousarray(a, dtype=np.int32).reshape(-1, 2) for a in (bra_l, bra_nprim))
        kl, kn = (np.ascontiguousarray(a, dtype=np.int32).reshape(-1, 2) for a in (ket_l, ket_nprim))
        assert bl.shape == bn.shape and kl.shape == kn.shape
        self.nbra, self.nket = bl.shape[0], kl.shape[0]
        self.nq = self.nbra * self.nket
        self.kmax = int(kmax)
        self.precision = precision
        h = ctypes.c_void_p()
        arr = tile_choices(tiles) if tiles else None
        vp = ctypes.c_void_p
        _check(lib().eri4_plan_create_pairs(
            ctypes.byref(h), self.nbra, bl.ctypes.data_as(vp), bn.ctypes.data_as(vp), self.nket,
            kl.ctypes.data_as(vp), kn.ctypes.data_as(vp), self.kmax,
            PRECISION[precision] if isinstance(precision, str) else int(precision), FUNCTIONS[functions],
            ctypes.cast(arr, vp) if arr is not None else None, len(arr) if arr is not None else 0))
        self._h = h
        self.functions = functions

    @property
    def work_size(self) -> int:
        return lib().eri4_plan_work_size(self._h)

    def execute(self, bra_centers, bra_exps, bra_coefs, ket_centers, ket_exps, ket_coefs, out=None, work=None,
                stream=None):
        import torch
        if out is None:
            out = torch.empty(self.output_size, dtype=torch.float64, device=bra_centers.device)
        if work is None and self.work_size > 0:
            work = torch.empty(self.work_size, dtype=torch.float64, device=bra_centers.device)
        if out.numel() < self.output_size:
            raise ValueError("output buffer too small")
        for c, e, w, n in ((bra_centers, bra_exps, bra_coefs, self.nbra), (ket_centers, ket_exps, ket_coefs, self.nket)):
            if tuple(c.shape) != (n, 2, 3) or tuple(e.shape) != (n, 2, self.kmax) or tuple(w.shape) != (n, 2, self.kmax):
                raise ValueError("pair lists do not match the plan")
        _check(lib().eri4_plan_execute_pairs(
            self._h, _ptr(bra_centers, "float64"), _ptr(bra_exps, "float64"), _ptr(bra_coefs, "float64"),
            _ptr(ket_centers, "float64"), _ptr(ket_exps, "float64"), _ptr(ket_coefs, "float64"),
            _ptr(work, "float64"), work.numel() if work is not None else 0, _ptr(out, "float64"), _stream(stream)))
        return out


class CoulombPlan(Plan):
    """J_i = sum_j sum_cd (ab|cd)_ij D_j[cd] for every bra entry i of a bra list
    and a ket list of shell pairs (eri4_plan_*_coulomb).  Host int32 arrays as
    PairPlan; execute() takes the device lists, ket_dens (the ket entries'
    blocks D_j[Nc][Nd] one after the other) and returns the bra entries' blocks
    J_i[Na][Nb] one after the other (offsets(): where each starts)."""

    def __init__(self, bra_l, bra_nprim, ket_l, ket_nprim, kmax: int):
        import numpy as np
        bl, bn = (np.ascontiguousarray(a, dtype=np.int32).reshape(-1, 2) for a in (bra_l, bra_nprim))
        kl, kn = (np.ascontiguousarray(a, dtype=np.int32).reshape(-1, 2) for a in (ket_l, ket_nprim))
        self.nbra, self.nket = bl.shape[0], kl.shape[0]
        self.nq = self.nbra * self.nket
        self.kmax = int(kmax)
        self.ket_dens_size = int(sum(ncart(int(a)) * ncart(int(b)) for a, b in kl))
        h = ctypes.c_void_p()
        vp = ctypes.c_void_p
        _check(lib().eri4_plan_create_coulomb(ctypes.byref(h), self.nbra, bl.ctypes.data_as(vp), bn.ctypes.data_as(vp),
                                              self.nket, kl.ctypes.data_as(vp), kn.ctypes.data_as(vp), self.kmax))
        self._h = h

    @property
    def work_size(self) -> int:
        return lib().eri4_plan_work_size(self._h)

    def offsets(self):
        import numpy as np
        off = np.zeros(self.nbra, dtype=np.int64)
        _check(lib().eri4_plan_output_offsets(self._h, off.ctypes.data_as(ctypes.c_void_p)))
        return off

    def execute(self, bra_centers, bra_exps, bra_coefs, ket_centers, ket_exps, ket_coefs, ket_dens, out=None,
                work=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(max(1, self.output_size), dtype=torch.float64, device=bra_centers.device)
        if work is None:
            work = torch.empty(max(1, self.work_size), dtype=torch.float64, device=bra_centers.device)
        _check_out(out, self.output_size)
        _check_out(ket_dens, self.ket_dens_size, "ket density")
        for c, e, w, n in ((bra_centers, bra_exps, bra_coefs, self.nbra), (ket_centers, ket_exps, ket_coefs, self.nket)):
            if tuple(c.shape) != (n, 2, 3) or tuple(e.shape) != (n, 2, self.kmax) or tuple(w.shape) != (n, 2, self.kmax):
                raise ValueError("pair lists do not match the plan")
        _check(lib().eri4_plan_execute_coulomb(
            self._h, _ptr(bra_centers, "float64"), _ptr(bra_exps, "float64"), _ptr(bra_coefs, "float64"),
            _ptr(ket_centers, "float64"), _ptr(ket_exps, "float64"), _ptr(ket_coefs, "float64"),
            _ptr(ket_dens, "float64"), _ptr(work, "float64"), work.numel(), _ptr(out, "float64"), _stream(stream)))
        return out
