"""ctypes binding of libfockmi.so (argument marshalling only).

The library is loaded from this package directory. There is no fallback: if
the shared object is missing or cannot be loaded, `lib()` raises.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfockmi.so")

FOCK_OK = 0
FOCK_WARN_NORM = 1
FOCK_WARN_CONV = 2
FOCK_ERR_ARG = -1
FOCK_ERR_SIZE = -2
FOCK_ERR_HIP = -3
FOCK_ERR_NOMEM = -4
FOCK_ERR_STATE = -5
STATUS_NAMES = {0: "FOCK_OK", 1: "FOCK_WARN_NORM", 2: "FOCK_WARN_CONV", -1: "FOCK_ERR_ARG", -2: "FOCK_ERR_SIZE", -3: "FOCK_ERR_HIP",
                -4: "FOCK_ERR_NOMEM", -5: "FOCK_ERR_STATE"}

FOCK_FP64 = 0
FOCK_FP32_COMP = 1
FOCK_FP64_FUSED = 2

EXPORTS = ["fock_plan_create", "fock_plan_destroy", "fock_apply", "fock_apply_krange", "fock_energy", "fock_energy_vjp",
           "fock_vjp", "taylor_step", "taylor_step_pc", "taylor_step_vjp", "taylor_energy", "taylor_energy_vjp", "taylor_excitation_energy",
           "taylor_current", "fock_orthonormalize", "fock_eigensolve",
           "fock_excited_density", "fock_apply_batched", "fock_apply_noalloc", "fock_profile_enable", "fock_profile_fallbacks",
           "fock_profile_read", "fock_last_error"]


class CellDesc(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("a", (C.c_double * 3) * 3), ("nk", C.c_int),
                ("kpts", C.POINTER(C.c_double)), ("nb", C.c_int), ("omega", C.c_double), ("gs", C.c_double),
                ("nsrc", C.c_int), ("src", C.POINTER(C.c_int))]


class FockError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """Loads libfockmi.so (raises if it is missing: no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_1507_05156_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    pd = C.POINTER(C.c_double)
    L.fock_plan_create.argtypes = [C.POINTER(CellDesc), i, i, C.c_char_p, C.POINTER(vp)]
    L.fock_plan_destroy.argtypes = [vp]
    L.fock_apply.argtypes = [vp, i, vp, vp, i, vp, vp]
    L.fock_apply_krange.argtypes = [vp, i, vp, i, i, vp, i, vp, vp]
    L.fock_energy.argtypes = [vp, i, vp, pd, pd, vp]
    L.fock_energy_vjp.argtypes = [vp, i, vp, d, vp, vp]
    L.fock_vjp.argtypes = [vp, i, vp, vp, i, vp, vp, vp, vp]
    L.taylor_step.argtypes = [vp, i, vp, vp, pd, d, d, i, pd, vp]
    L.taylor_step_pc.argtypes = [vp, i, vp, vp, pd, pd, d, d, i, pd, vp]
    L.taylor_step_vjp.argtypes = [vp, i, vp, vp, pd, d, d, i, vp, vp, pd, vp]
    L.taylor_energy.argtypes = [vp, i, vp, vp, pd, d, pd, vp, pd, vp]
    L.taylor_energy_vjp.argtypes = [vp, i, vp, vp, pd, d, d, vp, pd, vp]
    L.taylor_current.argtypes = [vp, i, vp, pd, pd, vp]
    L.taylor_excitation_energy.argtypes = [vp, i, vp, pd, vp, pd, vp, d, pd, vp]
    L.fock_orthonormalize.argtypes = [vp, i, vp, vp]
    L.fock_eigensolve.argtypes = [vp, i, vp, vp, pd, d, vp, d, i, pd, pd, C.POINTER(i), vp]
    L.fock_excited_density.argtypes = [vp, i, vp, vp, pd, vp]
    L.fock_apply_batched.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(i), C.POINTER(vp), vp]
    L.fock_apply_noalloc.argtypes = [vp, i, vp, vp, i, vp, vp]
    L.fock_profile_enable.argtypes = [vp, i]
    L.fock_profile_read.argtypes = [vp, pd, C.POINTER(C.c_longlong), i]
    L.fock_profile_fallbacks.argtypes = [vp, C.POINTER(C.c_longlong), i]
    L.fock_last_error.argtypes = []
    L.fock_last_error.restype = C.c_char_p
    for name in EXPORTS[:-1]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(status: int) -> int:
    if status < 0:
        raise FockError(status, lib().fock_last_error().decode())
    return status
