"""The gradient and current calls of the C ABI (every piece of arithmetic in the
library; the binding only passes pointers and scalars), against the FP64 oracle:

* fock_energy_vjp: g_e dE_x/du, full mesh and down-sampled source sub-mesh;
* taylor_energy_vjp: g_e times the energy functional's gradients;
* taylor_current: J = -(1/Omega) dE/d(A/c) (Eqs. (3)-(4));
* k-points that differ by a reciprocal-lattice vector (a finite q + G = 0 slot).
"""

import numpy as np
import pytest

import oracle
from oracle import adjoint as oadjoint
from oracle import taylor as otaylor
from paper_1507_05156_amd import synth

pytestmark = pytest.mark.gpu

OMEGA = synth.OMEGA_HSE
TOL = {"fp64": 1e-10, "fp32": 1e-6, "fp64f": 1e-10}


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def plan_for(cell, kp, nb, n, prec, src=None):
    from paper_1507_05156_amd.api import Plan
    d = dict(n=n, a=cell, kpts=kp, nb=nb, omega=OMEGA)
    if src is not None:
        d["src"] = src
    return Plan(d, prec=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp64f"])
def test_energy_vjp_full_mesh(device, prec):
    print(f"[gpu] energy vjp prec={prec}", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(16, cell, kp, 2, seed=610)
    plan = plan_for(cell, kp, 2, 16, prec)
    g_e = -1.7
    got = plan.energy_vjp(to_dev(u), g_e).cpu().numpy()
    assert rel(got, g_e * oracle.energy_grad(u, kp, cell, OMEGA)) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_energy_vjp_down_sampled(device, prec):
    print(f"[gpu] energy vjp down-sampled prec={prec}", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(4, cell, 2, 1)
    u = synth.orbitals(16, cell, kp, 2, seed=611)
    src = [0, 3, 5]
    plan = plan_for(cell, kp, 2, 16, prec, src)
    g_e = 0.75
    got = plan.energy_vjp(to_dev(u), g_e).cpu().numpy()
    w = 1.0 / len(kp) * oracle.volume(cell) / 16 ** 3
    V = oracle.fock_apply(u, u, kp, cell, OMEGA, src=src)
    gu, _ = oadjoint.fock_vjp(u, u, w * u, kp, cell, OMEGA, src=src)
    assert rel(got, g_e * (2.0 * w * V + gu)) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp64f"])
def test_energy_functional_vjp_and_current(device, prec):
    print(f"[gpu] energy functional vjp and current prec={prec}", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(16, cell, kp, 2, seed=612)
    vloc = np.random.default_rng(613).standard_normal((16, 16, 16)) * 0.05
    avec = np.array([0.01, -0.02, 0.03])
    _, g_ref, ga_ref = otaylor.energy_matfree(u, kp, cell, OMEGA, avec, 0.25, vloc)
    plan = plan_for(cell, kp, 2, 16, prec)
    g_e = 2.5
    g, ga = plan.energy_functional_vjp(to_dev(u), avec, 0.25, g_e, vloc=to_dev(vloc))
    assert rel(g.cpu().numpy(), g_e * g_ref) < TOL[prec]
    assert np.max(np.abs(ga - g_e * ga_ref)) < TOL[prec] * np.max(np.abs(g_e * ga_ref)) + 1e-14
    j = plan.current(to_dev(u), avec)
    j_ref = otaylor.current(u, kp, cell, avec)
    assert np.max(np.abs(j - j_ref)) < 1e-10 * np.max(np.abs(j_ref))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_kpoints_differing_by_a_reciprocal_vector(device, prec):
    """k = 0 and k' = b_1 label the same crystal momentum: the (k, k') table has
    q + G = 0 at G = b_1, which takes the finite value pi/w^2 (no NaN)."""
    print(f"[gpu] reciprocal-lattice shifted k-points prec={prec}", flush=True)
    cell = synth.cubic_cell()
    B = oracle.reciprocal(cell)
    kp = np.array([[0.0, 0.0, 0.0], B[0], [0.0, 0.0, 0.5 * B[2, 2]]])
    u = synth.orbitals(16, cell, kp, 2, seed=614)
    plan = plan_for(cell, kp, 2, 16, prec)
    got = plan.apply(to_dev(u)).cpu().numpy()
    assert np.all(np.isfinite(got))
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA)
    assert rel(got, ref) < TOL[prec]


def test_excitation_energy_double_double(device):
    """taylor_excitation_energy against the oracle's energy functional at both states,
    and its cancellation: the same state twice gives exactly 0, a state against itself
    with a phase gives 0 to rounding."""
    print("[gpu] excitation energy", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(16, cell, kp, 2, seed=615)
    w = synth.orbitals(16, cell, kp, 2, seed=616)
    vloc = np.random.default_rng(617).standard_normal((16, 16, 16)) * 0.05
    at, a0 = np.array([0.0, 0.0, 0.04]), np.array([0.01, 0.0, 0.0])
    plan = plan_for(cell, kp, 2, 16, "fp64")
    e = plan.excitation_energy(to_dev(w), at, to_dev(u), a0, 0.25, vloc=to_dev(vloc))
    ref = otaylor.energy_matfree(w, kp, cell, OMEGA, at, 0.25, vloc)[0] - \
        otaylor.energy_matfree(u, kp, cell, OMEGA, a0, 0.25, vloc)[0]
    assert abs(e - ref) < 1e-11 * abs(otaylor.energy_matfree(u, kp, cell, OMEGA, a0, 0.25, vloc)[0])
    assert plan.excitation_energy(to_dev(u), a0, to_dev(u), a0, 0.25) == 0.0
    z = plan.excitation_energy(to_dev(u * np.exp(0.3j)), a0, to_dev(u), a0, 0.25)
    assert abs(z) < 1e-14
