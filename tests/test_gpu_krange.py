"""fock_apply_krange: the operator on a contiguous range of output k-points (one
GPU's share of a k-point decomposition, Eqs. (15)-(16)) against the rows of the
full application and the FP64 oracle."""

import numpy as np
import pytest

import oracle
from paper_1507_05156_amd import synth

pytestmark = pytest.mark.gpu

OMEGA = synth.OMEGA_HSE


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def plan(cell, kp, nb, n, prec, src=None):
    from paper_1507_05156_amd.api import Plan
    d = dict(n=n, a=cell, kpts=kp, nb=nb, omega=OMEGA)
    if src is not None:
        d["src"] = src
    return Plan(d, prec=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp64f"])
def test_krange_rows_equal_the_full_application(device, prec):
    """16^3, 8 k, 4 bands: each target's sum is computed the same way, bit for bit."""
    print(f"[gpu] krange 16^3 prec={prec}", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell)
    u = synth.orbitals(16, cell, kp, 4, seed=401)
    phi = synth.random_fields((len(kp), 3, 16, 16, 16), seed=402)
    p = plan(cell, kp, 4, 16, prec)
    ud = to_dev(u)
    full = p.apply(ud, to_dev(phi)).cpu().numpy()
    part = p.apply_krange(ud, 3, 4, to_dev(phi[3:7])).cpu().numpy()
    assert np.array_equal(part, full[3:7])
    ref = oracle.fock_apply(u, phi, kp, cell, OMEGA, rows=[(5, 1)])
    e = np.linalg.norm(part[2, 1] - ref[5, 1]) / np.linalg.norm(ref[5, 1])
    assert e < (1e-10 if prec != "fp32" else 1e-6), e


def test_krange_32cube(device):
    """32^3 default form (the split form). A k-range runs every pair of its targets: its
    rows equal those of the full application that runs every pair (FOCKMI_SPLIT_SYM=0;
    each target's sum is independent of the target count) to 1e-13, and agree to FP32
    rounding with the default full application, which uses the pair symmetry (u as
    targets and sources: each pair of k-points once) and so sums each target's terms in
    another order; and with the oracle."""
    import os
    print("[gpu] krange 32^3", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell)
    u = synth.orbitals(32, cell, kp, 2, seed=403)
    p = plan(cell, kp, 2, 32, "fp32")
    ud = to_dev(u)
    full = p.apply(ud).cpu().numpy()
    part = p.apply_krange(ud, 2, 3).cpu().numpy()
    rel = np.max(np.abs(part - full[2:5])) / np.max(np.abs(full[2:5]))
    assert rel < 1e-6, rel
    os.environ["FOCKMI_SPLIT_SYM"] = "0"
    try:
        every = plan(cell, kp, 2, 32, "fp32")
    finally:
        del os.environ["FOCKMI_SPLIT_SYM"]
    full_every = every.apply(ud).cpu().numpy()
    rel = np.max(np.abs(part - full_every[2:5])) / np.max(np.abs(full_every[2:5]))
    assert rel < 1e-13, rel
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA, rows=[(4, 1)])
    e = np.linalg.norm(part[2, 1] - ref[4, 1]) / np.linalg.norm(ref[4, 1])
    assert e < 1e-6, e


def test_krange_downsampled_and_bad_ranges(device):
    print("[gpu] krange down-sampled, bad ranges", flush=True)
    from paper_1507_05156_amd._native import FockError
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(4, cell, 2, 1)
    src = [i for i in range(len(kp)) if (i // 2) % 2 == 0]
    u = synth.orbitals(16, cell, kp, 2, seed=404)
    p = plan(cell, kp, 2, 16, "fp64", src=src)
    ud = to_dev(u)
    full = p.apply(ud).cpu().numpy()
    part = p.apply_krange(ud, 5, 3).cpu().numpy()
    assert np.array_equal(part, full[5:8])
    import torch
    for k0, n in ((-1, 2), (7, 2), (0, 0)):
        phi = torch.zeros((max(n, 1), 2, 16, 16, 16), dtype=torch.complex128, device="cuda:0")
        with pytest.raises((FockError, ValueError)):
            p.apply_krange(ud, k0, n, phi if n > 0 else None)
