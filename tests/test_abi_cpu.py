"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/fockmi.h declares, and rejects bad arguments
with status codes before touching a device."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1507_05156_amd import _native as N
from paper_1507_05156_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fockmi.h")


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:fock_status|const char\*)\s+(\w+)\s*\(", text, re.M)))


def test_header_declares_the_four_calls():
    names = header_functions()
    for f in ["fock_apply", "fock_energy", "fock_vjp", "taylor_step", "fock_plan_create", "fock_last_error"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    lib = N.lib()
    for name in header_functions():
        assert hasattr(lib, name), name
    assert set(header_functions()) == set(N.EXPORTS)


def _desc(n=16, nk=2, nb=2, omega=0.106, kpts=None):
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell, 1, 1) if kpts is None else kpts
    d = N.CellDesc()
    for i in range(3):
        d.n[i] = n if np.isscalar(n) else n[i]
        for j in range(3):
            d.a[i][j] = cell[i, j]
    arr = np.ascontiguousarray(kp, dtype=np.float64)
    d.nk = len(arr)
    d.kpts = arr.ctypes.data_as(C.POINTER(C.c_double))
    d.nb = nb
    d.omega = omega
    d.gs = 2.0
    return d, arr


@pytest.mark.parametrize("kw,status", [
    (dict(n=18), N.FOCK_ERR_SIZE),
    (dict(n=(16, 16, 64)), N.FOCK_ERR_SIZE),
    (dict(omega=0.0), N.FOCK_ERR_ARG),
    (dict(omega=-1.0), N.FOCK_ERR_ARG),
    (dict(nb=0), N.FOCK_ERR_ARG),
])
def test_plan_create_rejects_bad_cells(kw, status):
    lib = N.lib()
    d, keep = _desc(**kw)
    h = C.c_void_p()
    st = lib.fock_plan_create(C.byref(d), 1, N.FOCK_FP64, None, C.byref(h))
    assert st == status
    assert h.value is None
    assert lib.fock_last_error()


@pytest.mark.parametrize("prec", ["FOCK_FP32_COMP", "FOCK_FP64_FUSED"])
def test_other_forms_check_grid_lengths(prec):
    """Every precision form takes the same grid lengths (a grid that is not cubic is
    accepted; it runs the plain stages), and rejects the others before any device call."""
    lib = N.lib()
    d, keep = _desc(n=(16, 20, 18))
    h = C.c_void_p()
    assert lib.fock_plan_create(C.byref(d), 1, getattr(N, prec), None, C.byref(h)) == N.FOCK_ERR_SIZE
    assert h.value is None
    assert b"grid length 18" in lib.fock_last_error()


def test_null_arguments():
    lib = N.lib()
    h = C.c_void_p()
    assert lib.fock_plan_create(None, 1, N.FOCK_FP64, None, C.byref(h)) == N.FOCK_ERR_ARG
    d, keep = _desc()
    assert lib.fock_plan_create(C.byref(d), 1, N.FOCK_FP64, None, None) == N.FOCK_ERR_ARG
    assert lib.fock_apply(None, 0, None, None, 1, None, None) == N.FOCK_ERR_ARG
    assert lib.fock_apply_krange(None, 0, None, 0, 1, None, 1, None, None) == N.FOCK_ERR_ARG
    a = (C.c_double * 3)(0.0, 0.0, 0.0)
    it = C.c_int()
    assert lib.fock_eigensolve(None, 0, None, None, a, 0.25, None, 1e-8, 10, None, None, C.byref(it), None) \
        == N.FOCK_ERR_ARG
    nex = C.c_double()
    assert lib.fock_excited_density(None, 0, None, None, C.byref(nex), None) == N.FOCK_ERR_ARG
    assert lib.fock_energy_vjp(None, 0, None, 1.0, None, None) == N.FOCK_ERR_ARG
    j = (C.c_double * 3)()
    assert lib.taylor_energy_vjp(None, 0, None, None, a, 0.25, 1.0, None, j, None) == N.FOCK_ERR_ARG
    assert lib.taylor_current(None, 0, None, a, j, None) == N.FOCK_ERR_ARG
    assert b"plan is NULL" in lib.fock_last_error()
    assert lib.fock_plan_destroy(None) == N.FOCK_OK


@pytest.mark.parametrize("src,nsrc", [([0, 0], 2), ([0, 5], 2), ([-1], 1), ([0], 3)])
def test_plan_create_rejects_bad_source_sets(src, nsrc):
    """Down-sampled source sets: repeated, out-of-range, or more than nk entries."""
    lib = N.lib()
    d, keep = _desc()
    arr = np.ascontiguousarray(np.asarray(src, dtype=np.int32))
    d.nsrc = nsrc
    d.src = arr.ctypes.data_as(C.POINTER(C.c_int))
    h = C.c_void_p()
    assert lib.fock_plan_create(C.byref(d), 1, N.FOCK_FP64, None, C.byref(h)) == N.FOCK_ERR_ARG
    assert h.value is None
    assert b"source" in lib.fock_last_error() or b"nsrc" in lib.fock_last_error()
