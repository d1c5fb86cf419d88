"""Down-sampled source sets through the C ABI (Sec. II C, after Eq. (16)): the
pair sum runs over a sub-mesh S of the k-points with weight 1/|S|, compared with
the FP64 oracle evaluating the same sum."""

import numpy as np
import pytest

import oracle
from oracle import adjoint as oadjoint
from oracle import taylor as otaylor
from paper_1507_05156_amd import synth

pytestmark = pytest.mark.gpu

OMEGA = synth.OMEGA_HSE
TOL = {"fp64": 1e-10, "fp32": 1e-6}


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def rel_per_k(got, ref):
    return max(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k]) for k in range(ref.shape[0]))


def case(n=16, nb=2, seed=91):
    """4 x 2 x 1 Gamma-centred mesh; S = the points with even x index (a 2 x 2 x 1 sub-mesh)."""
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(4, cell, 2, 1)
    u = synth.orbitals(n, cell, kp, nb, seed=seed)
    src = [i for i in range(len(kp)) if (i // 2) % 2 == 0]
    return cell, kp, u, src


def plan_for(cell, kp, nb, n, prec, src):
    from paper_1507_05156_amd.api import Plan
    return Plan(dict(n=n, a=cell, kpts=kp, nb=nb, omega=OMEGA, src=src), prec=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_and_energy_on_submesh(device, prec):
    print(f"[gpu] down-sampled apply prec={prec}", flush=True)
    cell, kp, u, src = case()
    phi = synth.random_fields((len(kp), 3, 16, 16, 16), seed=92)
    plan = plan_for(cell, kp, 2, 16, prec, src)
    ref = oracle.fock_apply(u, phi, kp, cell, OMEGA, src=src)
    got = plan.apply(to_dev(u), to_dev(phi)).cpu().numpy()
    assert rel_per_k(got, ref) < TOL[prec]
    e_ref = oracle.exchange_energy(u, kp, cell, OMEGA, src=src)
    e = plan.energy(to_dev(u))
    assert abs(e.real - e_ref.real) < TOL[prec] * abs(e_ref.real)
    # the sub-mesh sum differs from the full one: the plan really down-samples
    full = oracle.fock_apply(u, phi, kp, cell, OMEGA, rows=[(1, 0)])
    assert np.linalg.norm(got[1, 0] - full[1, 0]) > 1e-4 * np.linalg.norm(full[1, 0])


def test_gamma_only_source(device):
    """S = {Gamma} of a 2 x 2 x 2 mesh, FP64 and FP32."""
    print("[gpu] gamma source", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell)
    u = synth.orbitals(16, cell, kp, 2, seed=93)
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA, src=[0])
    for prec in ("fp64", "fp32"):
        got = plan_for(cell, kp, 2, 16, prec, [0]).apply(to_dev(u)).cpu().numpy()
        assert rel_per_k(got, ref) < TOL[prec], prec


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vjp_on_submesh(device, prec):
    print(f"[gpu] down-sampled vjp prec={prec}", flush=True)
    cell, kp, u, src = case(seed=94)
    phi = synth.random_fields((len(kp), 3, 16, 16, 16), seed=95)
    g = synth.random_fields((len(kp), 3, 16, 16, 16), seed=96)
    gu_ref, gp_ref = oadjoint.fock_vjp(u, phi, g, kp, cell, OMEGA, src=src)
    plan = plan_for(cell, kp, 2, 16, prec, src)
    gu, gp = plan.vjp(to_dev(u), to_dev(phi), to_dev(g))
    gu, gp = gu.cpu().numpy(), gp.cpu().numpy()
    assert rel_per_k(gp, gp_ref) < TOL[prec]
    assert rel_per_k(gu[src], gu_ref[src]) < TOL[prec]
    off = [k for k in range(len(kp)) if k not in src]
    assert np.all(gu[off] == 0)


def test_taylor_step_on_submesh(device):
    print("[gpu] down-sampled taylor step", flush=True)
    cell, kp, u, src = case(seed=97)
    avec = np.array([0.01, 0.0, -0.02])
    ref = otaylor.step_matfree(u, kp, cell, OMEGA, avec, 0.02, 0.25, src=src)
    plan = plan_for(cell, kp, 2, 16, "fp64", src)
    psi = to_dev(u)
    plan.taylor_step(psi, avec, 0.02, 0.25)
    assert rel_per_k(psi.cpu().numpy(), ref) < 1e-10


def test_energy_gradient_on_submesh(device):
    """autograd of E_x with S: 2 w V_x u from the targets plus the adjoint through the sources."""
    print("[gpu] down-sampled energy gradient", flush=True)
    import torch
    from paper_1507_05156_amd import autograd as ag
    cell, kp, u, src = case(seed=98)
    plan = plan_for(cell, kp, 2, 16, "fp64", src)
    ud = to_dev(u).requires_grad_(True)
    e = ag.fock_energy(ud, plan)
    e.backward()
    w = 1.0 / len(kp) * oracle.volume(cell) / 16 ** 3
    V = oracle.fock_apply(u, u, kp, cell, OMEGA, src=src)
    gu, _ = oadjoint.fock_vjp(u, u, w * u, kp, cell, OMEGA, src=src)
    ref = 2.0 * w * V + gu
    assert rel_per_k(ud.grad.cpu().numpy(), ref) < 1e-10
    # central difference of the GPU energy along a random direction
    d = synth.random_fields(u.shape, seed=99)
    d *= np.linalg.norm(u) / np.linalg.norm(d)
    h = 1e-5
    ep = plan.energy(to_dev(u + h * d)).real
    em = plan.energy(to_dev(u - h * d)).real
    fd = (ep - em) / (2 * h)
    ad = np.real(np.sum(np.conj(ref) * d))
    assert abs(fd - ad) < 1e-7 * abs(ad)


def test_unsupported_calls_and_batched_route(device):
    """The propagator's gradient calls refuse a down-sampled cell; the batched call runs it per cell."""
    print("[gpu] down-sampled unsupported and batched", flush=True)
    from paper_1507_05156_amd._native import FockError
    from paper_1507_05156_amd.api import Plan
    cell, kp, u, src = case(seed=100)
    plan = plan_for(cell, kp, 2, 16, "fp64", src)
    with pytest.raises(FockError):
        plan.energy_functional(to_dev(u), [0, 0, 0], 0.25)
    with pytest.raises(FockError):
        plan.taylor_step_vjp(to_dev(u), [0, 0, 0], 0.02, 0.25, to_dev(u))
    pb = Plan([dict(n=16, a=cell, kpts=kp, nb=2, omega=OMEGA, src=src),
               dict(n=16, a=cell, kpts=kp, nb=2, omega=OMEGA)], prec="fp32")
    outs = pb.apply_batched([to_dev(u), to_dev(u)])
    ref_ds = oracle.fock_apply(u, u, kp, cell, OMEGA, src=src)
    ref_full = oracle.fock_apply(u, u, kp, cell, OMEGA)
    assert rel_per_k(outs[0].cpu().numpy(), ref_ds) < 1e-6
    assert rel_per_k(outs[1].cpu().numpy(), ref_full) < 1e-6
