"""fock_apply_noalloc (the allocation-free FP32-form application) through the C ABI,
against fock_apply on the same plan and against the FP64 oracle: two calls in a
row, the second with a smaller input, a 32^3 cell, and the refusals (a cell whose
scratch exceeds the fixed array, a plan of another precision)."""

import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1507_05156_amd import synth

pytestmark = pytest.mark.gpu

OMEGA = synth.OMEGA_HSE


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def noalloc(plan, u, phi, cell=0):
    import torch
    from paper_1507_05156_amd import _native as N
    out = torch.empty_like(phi)
    st = N.lib().fock_apply_noalloc(plan._h, cell, C.c_void_p(u.data_ptr()), C.c_void_p(phi.data_ptr()),
                                    phi.shape[1], C.c_void_p(out.data_ptr()),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, out


def test_noalloc_matches_fock_apply_two_calls(device):
    print("[gpu] no-alloc: 20^3 / 8 k / 4 b, then 16^3 / 2 k / 2 b with 3 targets", flush=True)
    from paper_1507_05156_amd import _native as N
    from paper_1507_05156_amd.api import Plan
    cell = synth.cubic_cell()
    kp1 = synth.gamma_mesh(2, cell)
    u1 = synth.orbitals(20, cell, kp1, 4, seed=701)
    kp2 = synth.gamma_mesh(2, cell, 1, 1)
    u2 = synth.orbitals(16, cell, kp2, 2, seed=702)
    phi2 = synth.random_fields((len(kp2), 3, 16, 16, 16), seed=703)
    plan = Plan([dict(n=20, a=cell, kpts=kp1, nb=4, omega=OMEGA), dict(n=16, a=cell, kpts=kp2, nb=2, omega=OMEGA)],
                prec="fp32")
    d1 = to_dev(u1)
    st, got1 = noalloc(plan, d1, d1, cell=0)
    assert st == N.FOCK_OK, N.lib().fock_last_error()
    d2, p2 = to_dev(u2), to_dev(phi2)
    st, got2 = noalloc(plan, d2, p2, cell=1)
    assert st == N.FOCK_OK, N.lib().fock_last_error()
    ref1 = plan.apply(d1, cell=0)
    ref2 = plan.apply(d2, p2, cell=1)
    # the same kernels on the same inputs: the same bits
    assert bool((got1 == ref1).all()) and bool((got2 == ref2).all())
    o1 = oracle.fock_apply(u1, u1, kp1, cell, OMEGA)
    o2 = oracle.fock_apply(u2, phi2, kp2, cell, OMEGA)
    assert rel(got1.cpu().numpy(), o1) < 1e-6
    assert rel(got2.cpu().numpy(), o2) < 1e-6
    # a third call, larger again, after the smaller one
    st, got3 = noalloc(plan, d1, d1, cell=0)
    assert st == N.FOCK_OK and bool((got3 == ref1).all())


def test_noalloc_32cube_cell(device):
    print("[gpu] no-alloc: 32^3 / 2 k / 2 b", flush=True)
    from paper_1507_05156_amd import _native as N
    from paper_1507_05156_amd.api import Plan
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(32, cell, kp, 2, seed=704)
    plan = Plan(dict(n=32, a=cell, kpts=kp, nb=2, omega=OMEGA), prec="fp32")
    d = to_dev(u)
    st, got = noalloc(plan, d, d)
    assert st == N.FOCK_OK, N.lib().fock_last_error()
    ref = plan.apply(d)  # the split form: the same sum in other FP32 roundings
    assert rel(got.cpu().numpy(), ref.cpu().numpy()) < 1e-6
    assert rel(got.cpu().numpy(), oracle.fock_apply(u, u, kp, cell, OMEGA)) < 1e-6


def test_noalloc_refusals(device):
    print("[gpu] no-alloc: refusals", flush=True)
    import torch
    from paper_1507_05156_amd import _native as N
    from paper_1507_05156_amd.api import Plan
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(4, cell)
    big = Plan(dict(n=24, a=cell, kpts=kp, nb=16, omega=OMEGA), prec="fp32")
    u = torch.zeros((len(kp), 16, 24, 24, 24), dtype=torch.complex128, device="cuda:0")
    st, _ = noalloc(big, u, u)
    assert st == N.FOCK_ERR_SIZE
    assert b"scratch" in N.lib().fock_last_error()
    del u
    kp2 = synth.gamma_mesh(2, cell, 1, 1)
    p64 = Plan(dict(n=16, a=cell, kpts=kp2, nb=2, omega=OMEGA), prec="fp64")
    v = to_dev(synth.orbitals(16, cell, kp2, 2, seed=705))
    st, _ = noalloc(p64, v, v)
    assert st == N.FOCK_ERR_ARG
