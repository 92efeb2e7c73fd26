"""ctypes loader of the gfx950 J/K library (``libjk_gfx950.so``).

The library is the whole product path: if it is missing, every call raises.
There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjk_gfx950.so")

JK_OK, JK_EINVAL, JK_EWORKSPACE, JK_EUNSUPPORTED, JK_EHIP, JK_ENOMEM = 0, 1, 2, 3, 4, 5
JK_FP64, JK_MIXED = 0, 1
JK_WANT_J, JK_WANT_K, JK_B_PACKED = 1, 2, 4

# Every symbol include/jk.h and include/jk_prof.h declare.
EXPORTS = ("jk_workspace_bytes", "jk_build", "jk_build_noalloc", "jk_slices_bytes", "jk_slice_b",
           "jk_build_sliced", "jk_fock_workspace_bytes", "jk_fock",
           "jk_batched_workspace_bytes", "jk_build_batched", "jk_vjp", "jk_status_str")
LAPLACE_EXPORTS = ("jk_laplace_quadrature", "jk_laplace_factors", "jk_laplace_workspace_bytes",
                   "jk_laplace_build")
LAPLACE_MAX_POINTS = 20
TUNE_EXPORTS = ("jk_autotune", "jk_tuning_get", "jk_tuning_set", "jk_tuning_clear",
                "jk_tuning_save", "jk_tuning_load", "jk_plan_describe")
PROF_EXPORTS = ("jk_prof_enable", "jk_prof_reset", "jk_prof_collect", "jk_prof_entry",
                "jk_prof_dropped", "jk_peak_mfma")


class Problem(ctypes.Structure):
    _fields_ = [("nao", ctypes.c_int64), ("naux", ctypes.c_int64), ("ndens", ctypes.c_int64),
                ("rank", ctypes.c_int64), ("precision", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("nslice", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class LaplaceProblem(ctypes.Structure):
    _fields_ = [("nao", ctypes.c_int64), ("naux", ctypes.c_int64), ("nocc", ctypes.c_int64),
                ("nvir", ctypes.c_int64), ("nvec", ctypes.c_int64), ("npts", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32), ("nslice", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("ht_tile", ctypes.c_int32), ("chunk_mb", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("chunk_slabs", ctypes.c_int32), ("nsplit", ctypes.c_int32),
                ("nsplit_sym", ctypes.c_int32), ("int_depth", ctypes.c_int32),
                ("int_depth_cap", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class JKError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} (status {status})")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        pp = ctypes.POINTER(Problem)
        L.jk_workspace_bytes.restype = sz
        L.jk_workspace_bytes.argtypes = [pp]
        L.jk_build.restype = ctypes.c_int
        L.jk_build.argtypes = [pp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.jk_build_noalloc.restype = ctypes.c_int
        L.jk_build_noalloc.argtypes = [pp, vp, vp, vp, vp, vp, vp]
        L.jk_slices_bytes.restype = sz
        L.jk_slices_bytes.argtypes = [pp]
        L.jk_slice_b.restype = ctypes.c_int
        L.jk_slice_b.argtypes = [pp, vp, vp, sz, vp]
        L.jk_build_sliced.restype = ctypes.c_int
        L.jk_build_sliced.argtypes = [pp, vp, vp, sz, vp, vp, vp, vp, vp, sz, vp]
        L.jk_fock_workspace_bytes.restype = sz
        L.jk_fock_workspace_bytes.argtypes = [pp, ctypes.c_int64]
        L.jk_fock.restype = ctypes.c_int
        L.jk_fock.argtypes = [pp, vp, vp, ctypes.c_int64, vp, vp, ctypes.POINTER(ctypes.c_double),
                              vp, vp, sz, vp]
        L.jk_batched_workspace_bytes.restype = sz
        L.jk_batched_workspace_bytes.argtypes = [ctypes.c_int32, pp]
        L.jk_build_batched.restype = ctypes.c_int
        L.jk_build_batched.argtypes = [ctypes.c_int32, pp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.jk_vjp.restype = ctypes.c_int
        L.jk_vjp.argtypes = [pp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.jk_status_str.restype = ctypes.c_char_p
        L.jk_status_str.argtypes = [ctypes.c_int]
        dp = ctypes.POINTER(ctypes.c_double)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.jk_laplace_quadrature.restype = ctypes.c_int
        L.jk_laplace_quadrature.argtypes = [i32, dbl, dbl, dp, dp, dp, ctypes.POINTER(i32)]
        L.jk_laplace_factors.restype = ctypes.c_int
        L.jk_laplace_factors.argtypes = [i64, i64, i64, i64, i32, vp, vp, vp, dp, dp, dbl, vp, vp]
        lpp = ctypes.POINTER(LaplaceProblem)
        L.jk_laplace_workspace_bytes.restype = sz
        L.jk_laplace_workspace_bytes.argtypes = [lpp]
        L.jk_laplace_build.restype = ctypes.c_int
        L.jk_laplace_build.argtypes = [lpp, vp, vp, vp, vp, vp, vp, dp, dp, dbl, vp, vp, vp, sz, vp]
        tp = ctypes.POINTER(Tuning)
        L.jk_autotune.restype = ctypes.c_int
        L.jk_autotune.argtypes = [pp, vp, vp, vp, vp, vp, vp, sz, vp, ctypes.c_int32, tp]
        L.jk_tuning_get.restype = ctypes.c_int
        L.jk_tuning_get.argtypes = [pp, tp]
        L.jk_tuning_set.restype = ctypes.c_int
        L.jk_tuning_set.argtypes = [pp, tp]
        L.jk_tuning_clear.restype = None
        L.jk_tuning_clear.argtypes = []
        L.jk_tuning_save.restype = sz
        L.jk_tuning_save.argtypes = [ctypes.c_char_p, sz]
        L.jk_tuning_load.restype = ctypes.c_int
        L.jk_tuning_load.argtypes = [ctypes.c_char_p]
        L.jk_plan_describe.restype = ctypes.c_int
        L.jk_plan_describe.argtypes = [pp, tp, ctypes.POINTER(PlanInfo)]
        L.jk_prof_enable.restype = ctypes.c_int
        L.jk_prof_enable.argtypes = [ctypes.c_int32]
        L.jk_prof_reset.restype = None
        L.jk_prof_reset.argtypes = []
        L.jk_prof_collect.restype = ctypes.c_int32
        L.jk_prof_collect.argtypes = []
        L.jk_prof_entry.restype = ctypes.c_int
        L.jk_prof_entry.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.jk_prof_dropped.restype = ctypes.c_int64
        L.jk_prof_dropped.argtypes = []
        L.jk_peak_mfma.restype = ctypes.c_double
        L.jk_peak_mfma.argtypes = [ctypes.c_int32, ctypes.c_int32]
        _lib = L
    return _lib


def status_str(s: int) -> str:
    return lib().jk_status_str(int(s)).decode()


def check(status: int, what: str) -> None:
    if status != JK_OK:
        raise JKError(status, what)


def prof_enable(capacity: int) -> None:
    """Start recording per-launch HIP events (see include/jk_prof.h)."""
    if lib().jk_prof_enable(int(capacity)) != 0:
        raise RuntimeError("jk_prof_enable failed")


def prof_disable() -> None:
    lib().jk_prof_enable(0)


def prof_reset() -> None:
    lib().jk_prof_reset()


def prof_collect() -> dict:
    """{kernel name: (total ms, launches)} of the recorded launches."""
    L = lib()
    n = L.jk_prof_collect()
    if n < 0:
        raise RuntimeError("jk_prof_collect failed")
    out = {}
    for i in range(n):
        name = ctypes.c_char_p()
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        L.jk_prof_entry(i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(cnt))
        out[name.value.decode()] = (ms.value, cnt.value)
    return out


def prof_dropped() -> int:
    return int(lib().jk_prof_dropped())


def peak_mfma(kind: str, random: bool = True) -> float:
    """Measured matrix-core rate: kind "int8" (int8 ops/s in the slice
    engine's pattern) or "fp64" (flop/s); random per-lane operands or
    constants (include/jk_prof.h)."""
    v = float(lib().jk_peak_mfma({"int8": 0, "fp64": 1}[kind], 1 if random else 0))
    if v < 0:
        raise RuntimeError("jk_peak_mfma failed")
    return v
