"""The persistent lockstep form of the 32^3 fused kernel against the form with one
workgroup per target and against the FP64 oracle, with rounds that leave XCDs
partly filled or idle. The lockstep form splits each target's k' sum into equal
parts when that fills the GPU better (4 parts for 8 k-points and 40 or 24
targets, 3 for 27 k-points and 270 targets), so the two forms differ only in the
order of the FP64 additions. The form is chosen through the plan's tuning cache."""

import json

import numpy as np
import pytest

import oracle
from paper_1507_05156_amd import synth

pytestmark = pytest.mark.gpu

OMEGA = synth.OMEGA_HSE


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def plan_with_variant(tmp_path, cell, kp, nb, variant, nx=None):
    import torch
    from paper_1507_05156_amd.api import Plan
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    nk = len(kp)
    key = f"{arch}/fp32/fused/n32x32x32/nt{nk}/ns{nk}/nb{nb}/nx{nx or nb}"
    path = tmp_path / f"tune_{variant}.json"
    path.write_text(json.dumps({key: {"variant": variant, "xcd_map": 1}}))
    return Plan(dict(n=32, a=cell, kpts=kp, nb=nb, omega=OMEGA), prec="fp32", tune_cache=str(path))


@pytest.mark.parametrize("mesh,nb", [((2, 2, 2), 5), ((3, 3, 3), 10)])
def test_lockstep_matches_grid_form_and_oracle(device, tmp_path, mesh, nb):
    """8 k x 5 bands = 40 targets (one XCD full, one partly, six idle); 27 k x 10
    bands = 270 targets (a full round of 256, then 14 on one XCD)."""
    print(f"[gpu] lockstep 32^3 mesh={mesh} nb={nb}", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(mesh[0], cell, mesh[1], mesh[2])
    u = synth.orbitals(32, cell, kp, nb, seed=300 + nb)
    ud = to_dev(u)
    outs = []
    for variant in (0, 1):
        plan = plan_with_variant(tmp_path, cell, kp, nb, variant)
        outs.append(plan.apply(ud).cpu().numpy())
        plan.close()
    rel = np.max(np.abs(outs[0] - outs[1])) / np.max(np.abs(outs[0]))
    assert rel < 1e-13, rel
    rows = [(0, 0), (len(kp) - 1, nb - 1)]
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA, rows=rows)
    for k, i in rows:
        e = np.linalg.norm(outs[1][k, i] - ref[k, i]) / np.linalg.norm(ref[k, i])
        print(f"  row {(k, i)}: rel err {e:.3e}", flush=True)
        assert e < 1e-6


def test_lockstep_separate_phi_and_repeat(device, tmp_path):
    """phi differs from the sources (3 targets per k), and a second launch on the
    same plan (counters cleared by the launch) gives the same bits."""
    print("[gpu] lockstep 32^3 phi != u, repeat", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell)
    u = synth.orbitals(32, cell, kp, 4, seed=311)
    phi = synth.random_fields((len(kp), 3, 32, 32, 32), seed=312)
    plan = plan_with_variant(tmp_path, cell, kp, 4, 1, nx=3)
    a = plan.apply(to_dev(u), to_dev(phi)).cpu().numpy()
    b = plan.apply(to_dev(u), to_dev(phi)).cpu().numpy()
    assert np.array_equal(a, b)
    ref = oracle.fock_apply(u, phi, kp, cell, OMEGA, rows=[(3, 2)])
    e = np.linalg.norm(a[3, 2] - ref[3, 2]) / np.linalg.norm(ref[3, 2])
    assert e < 1e-6, e


def test_lockstep_adjoint_accumulates_split_parts(device, tmp_path):
    """fock_vjp adds a second pair family into the same output (accumulate), which the
    split sums must honour: 32^3, 8 k, 2 bands against the oracle's adjoint."""
    print("[gpu] lockstep 32^3 vjp", flush=True)
    from oracle import adjoint as oadjoint
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell)
    u = synth.orbitals(32, cell, kp, 2, seed=321)
    phi = synth.random_fields((len(kp), 2, 32, 32, 32), seed=322)
    g = synth.random_fields((len(kp), 2, 32, 32, 32), seed=323)
    plan = plan_with_variant(tmp_path, cell, kp, 2, 1)
    gu, gp = plan.vjp(to_dev(u), to_dev(phi), to_dev(g))
    gu_ref, gp_ref = oadjoint.fock_vjp(u, phi, g, kp, cell, OMEGA)
    for got, ref in ((gu.cpu().numpy(), gu_ref), (gp.cpu().numpy(), gp_ref)):
        e = max(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k]) for k in range(len(kp)))
        assert e < 1e-6, e
