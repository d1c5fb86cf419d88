"""The split 32^3 form of the FP32 fused kernel (each target on two CUs of one XCD,
one exchange per pair) through the C ABI: against the FP64 oracle, bitwise
repeatability, more bands than one FP32 partial sum holds (two folds per k'), a
target count that leaves most CU pairs idle, and its fallback (the host forces
every rendezvous to stop; the lockstep form behind it then gives the result).

With u as targets and sources over a whole mesh of at least 3 k-points the form uses
the pair symmetry (W of source b on target a is the conjugate of W of a on b): each
target runs the source k-points k + d, d = 0 .. N_k/2, and pushes the mirror terms of
d = 1 .. (N_k - 1)/2 into per-XCD copies of the other targets. Those cases are checked
against the oracle and against the form that runs every pair (FOCKMI_SPLIT_SYM=0)."""

import os

import numpy as np
import pytest

import oracle
from paper_1507_05156_amd import synth

pytestmark = pytest.mark.gpu

OMEGA = synth.OMEGA_HSE


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def rel_per_k(got, ref):
    return max(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k]) for k in range(ref.shape[0]))


def plan32(kp, nb, cell, **env):
    from paper_1507_05156_amd.api import Plan
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return Plan(dict(n=32, a=cell, kpts=kp, nb=nb, omega=OMEGA), prec="fp32")
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("mesh,nb", [((2, 1, 1), 3), ((1, 1, 1), 20)])
def test_split_matches_oracle(device, mesh, nb):
    print(f"[gpu] split 32^3 mesh={mesh} nb={nb}", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(mesh[0], cell, mesh[1], mesh[2])
    u = synth.orbitals(32, cell, kp, nb, seed=800 + nb)
    plan = plan32(kp, nb, cell)
    plan.profile(True)
    d = to_dev(u)
    got = plan.apply(d).cpu().numpy()
    again = plan.apply(d).cpu().numpy()
    assert plan.profile_fallbacks() == 0       # the split launches ran to completion
    plan.profile(False)
    assert np.array_equal(got, again)          # bitwise repeatable
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA)
    e = rel_per_k(got, ref)
    print(f"  per-k rel err {e:.3e}", flush=True)
    assert e < 1e-6


def test_split_fallback_when_forced(device):
    """FOCKMI_SPLIT_WAIT_TICKS < 0 makes every rendezvous stop at once: the launch sets its
    abort word and the lockstep form behind it computes the whole application."""
    print("[gpu] split 32^3 forced fallback", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(32, cell, kp, 3, seed=810)
    plan = plan32(kp, 3, cell, FOCKMI_SPLIT_WAIT_TICKS=-1)
    plan.profile(True)
    got = plan.apply(to_dev(u)).cpu().numpy()
    assert plan.profile_fallbacks() == 1
    plan.profile(False)
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA)
    assert rel_per_k(got, ref) < 1e-6


def test_split_several_rounds_phi_and_shard(device):
    """27 k x 10 bands = 270 targets on 128 CU pairs (two full rounds and a partial
    one), in the symmetric form (odd N_k: no antipodal block; mirror copies that take
    more than 16 pushes, so their elements are folded more than once): sampled rows
    against the oracle, every k against the form that runs every pair. Separate targets
    phi (3 per k, no symmetry); one k-range shard (no symmetry either), bitwise equal to
    the rows of the full application that runs every pair (each target's sum does not
    depend on the CU pair that runs it)."""
    print("[gpu] split 32^3 rounds, phi, shard", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(3, cell)
    u = synth.orbitals(32, cell, kp, 10, seed=820)
    plan = plan32(kp, 10, cell)
    plan.profile(True)
    d = to_dev(u)
    full = plan.apply(d).cpu().numpy()
    rows = [(0, 0), (12, 7), (26, 9)]
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA, rows=rows)
    for k, i in rows:
        e = np.linalg.norm(full[k, i] - ref[k, i]) / np.linalg.norm(ref[k, i])
        print(f"  row {(k, i)}: rel err {e:.3e}", flush=True)
        assert e < 1e-6
    every = plan32(kp, 10, cell, FOCKMI_SPLIT_SYM=0)
    full_every = every.apply(d).cpu().numpy()
    e = rel_per_k(full, full_every)
    print(f"  symmetric vs every pair: max per-k rel {e:.3e}", flush=True)
    assert e < 1e-6
    part = plan.apply_krange(d, 12, 5).cpu().numpy()
    assert np.array_equal(part, full_every[12:17])
    phi = synth.random_fields((len(kp), 3, 32, 32, 32), seed=821)
    got = plan.apply(d, to_dev(phi)).cpu().numpy()
    ref = oracle.fock_apply(u, phi, kp, cell, OMEGA, rows=[(20, 2)])
    assert np.linalg.norm(got[20, 2] - ref[20, 2]) / np.linalg.norm(ref[20, 2]) < 1e-6
    assert plan.profile_fallbacks() == 0
    plan.profile(False)


def test_split_vjp_and_energy_gradient(device):
    """The adjoint at 32^3: its forward-shaped families run the split kernel, the family that
    accumulates into an existing output runs the lockstep form; both cotangents against the
    oracle, and the library's E_x gradient against the oracle's."""
    print("[gpu] split 32^3 vjp", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(32, cell, kp, 2, seed=830)
    phi = synth.random_fields((2, 3, 32, 32, 32), seed=831)
    g = synth.random_fields((2, 3, 32, 32, 32), seed=832)
    plan = plan32(kp, 2, cell)
    plan.profile(True)
    gu, gp = plan.vjp(to_dev(u), to_dev(phi), to_dev(g))
    gu_ref, gp_ref = oracle.fock_vjp(u, phi, g, kp, cell, OMEGA)
    assert rel_per_k(gu.cpu().numpy(), gu_ref) < 1e-6
    assert rel_per_k(gp.cpu().numpy(), gp_ref) < 1e-6
    ge = plan.energy_vjp(to_dev(u), 1.0).cpu().numpy()
    assert rel_per_k(ge, oracle.energy_grad(u, kp, cell, OMEGA)) < 1e-6
    assert plan.profile_fallbacks() == 0
    plan.profile(False)


def test_split_in_kernel_timeout_falls_back(device):
    """A real-time limit of one tick (10 ns) on each rendezvous: the waits time out inside
    the kernel (not the host-forced stop), the launch sets its abort word, every
    workgroup leaves at its next wait, and the lockstep form behind it gives the result."""
    print("[gpu] split 32^3 in-kernel timeout", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(32, cell, kp, 3, seed=840)
    plan = plan32(kp, 3, cell, FOCKMI_SPLIT_WAIT_TICKS=1)
    plan.profile(True)
    got = plan.apply(to_dev(u)).cpu().numpy()
    assert plan.profile_fallbacks() == 1
    plan.profile(False)
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA)
    assert rel_per_k(got, ref) < 1e-6


def test_split_single_target_single_pair(device):
    """Gamma only and one band: one target, one pair (no staggered fold at all, the final
    fold takes every element), 127 of the 128 CU pairs without work."""
    print("[gpu] split 32^3 one pair", flush=True)
    cell = synth.cubic_cell()
    kp = np.zeros((1, 3))
    u = synth.orbitals(32, cell, kp, 1, seed=850)
    plan = plan32(kp, 1, cell)
    plan.profile(True)
    got = plan.apply(to_dev(u)).cpu().numpy()
    assert plan.profile_fallbacks() == 0
    plan.profile(False)
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA)
    assert rel_per_k(got, ref) < 1e-6


def test_split_pair_symmetry(device):
    """u over a 2x2x2 mesh, 3 bands: the antipodal block d = 4 runs in both rows, the
    blocks d = 1..3 once with their mirror terms pushed. Every row against the oracle,
    bitwise repeatable, against the form that runs every pair (also what a plan whose
    workspace cap cannot hold the mirror copies runs), and the E_x gradient (the same
    symmetric pair sum) against the oracle."""
    print("[gpu] split 32^3 pair symmetry", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell)
    u = synth.orbitals(32, cell, kp, 3, seed=860)
    plan = plan32(kp, 3, cell)
    plan.profile(True)
    d = to_dev(u)
    got = plan.apply(d).cpu().numpy()
    again = plan.apply(d).cpu().numpy()
    assert plan.profile_fallbacks() == 0
    plan.profile(False)
    assert np.array_equal(got, again)
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA)
    e = rel_per_k(got, ref)
    print(f"  per-k rel err {e:.3e}", flush=True)
    assert e < 1e-6
    every = plan32(kp, 3, cell, FOCKMI_SPLIT_SYM=0).apply(d).cpu().numpy()
    assert rel_per_k(got, every) < 1e-6
    # a workspace cap below the mirror copies (201 MB here) leaves the form that runs
    # every pair, bit for bit
    capped = plan32(kp, 3, cell, FOCKMI_WORKSPACE_CAP=100 << 20).apply(d).cpu().numpy()
    assert np.array_equal(capped, every)
    ge = plan.energy_vjp(d, 1.0).cpu().numpy()
    assert rel_per_k(ge, oracle.energy_grad(u, kp, cell, OMEGA)) < 1e-6


@pytest.mark.parametrize("ticks", [-1, 1])
def test_split_pair_symmetry_falls_back(device, ticks):
    """The symmetric form stopped by the host (every wait stops at once) and by its own
    one-tick wait limit (the waits of the exchange and of the mirror pushes time out
    inside the kernel): the combine of the mirror copies is skipped and the lockstep
    form computes the whole application."""
    print(f"[gpu] split 32^3 pair symmetry fallback, ticks {ticks}", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell)
    u = synth.orbitals(32, cell, kp, 2, seed=870)
    plan = plan32(kp, 2, cell, FOCKMI_SPLIT_WAIT_TICKS=ticks)
    plan.profile(True)
    got = plan.apply(to_dev(u)).cpu().numpy()
    assert plan.profile_fallbacks() == 1
    plan.profile(False)
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA)
    assert rel_per_k(got, ref) < 1e-6


def test_split_pair_symmetry_many_bands(device):
    """3 k-points x 20 bands, u as targets and sources: one pushed block (d = 1), more
    bands than one FP32 partial sum takes in the target's own sum, 60 targets over four
    XCDs. Every k against the form that runs every pair, two rows against the oracle."""
    print("[gpu] split 32^3 pair symmetry, 20 bands", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(3, cell, 1, 1)
    u = synth.orbitals(32, cell, kp, 20, seed=880)
    plan = plan32(kp, 20, cell)
    plan.profile(True)
    d = to_dev(u)
    got = plan.apply(d).cpu().numpy()
    assert plan.profile_fallbacks() == 0
    plan.profile(False)
    every = plan32(kp, 20, cell, FOCKMI_SPLIT_SYM=0).apply(d).cpu().numpy()
    e = rel_per_k(got, every)
    print(f"  symmetric vs every pair: max per-k rel {e:.3e}", flush=True)
    assert e < 1e-6
    rows = [(0, 19), (2, 3)]
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA, rows=rows)
    for k, i in rows:
        e = np.linalg.norm(got[k, i] - ref[k, i]) / np.linalg.norm(ref[k, i])
        print(f"  row {(k, i)}: rel err {e:.3e}", flush=True)
        assert e < 1e-6



@pytest.mark.parametrize("mesh", [2, 3])
def test_split_pair_symmetry_16_bands(device, mesh):
    """16 bands, u as targets and sources, so that the 16 CU pairs of an XCD hold the 16 bands
    of one k-point (as on the 32^3 / 216 k / 16-band workload). 2x2x2 mesh: 128 targets, one
    round; 3x3x3: 432 targets, four rounds, the last on three XCDs. Every k against the form
    that runs every pair, bitwise repeatable, rows against the oracle."""
    print(f"[gpu] split 32^3 pair symmetry, 16 bands, mesh {mesh}", flush=True)
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(mesh, cell)
    u = synth.orbitals(32, cell, kp, 16, seed=890 + mesh)
    plan = plan32(kp, 16, cell)
    plan.profile(True)
    d = to_dev(u)
    got = plan.apply(d).cpu().numpy()
    again = plan.apply(d).cpu().numpy()
    assert plan.profile_fallbacks() == 0
    plan.profile(False)
    assert np.array_equal(got, again)
    plan.close()
    every = plan32(kp, 16, cell, FOCKMI_SPLIT_SYM=0).apply(d).cpu().numpy()
    e = rel_per_k(got, every)
    print(f"  symmetric vs every pair: max per-k rel {e:.3e}", flush=True)
    assert e < 1e-6
    nk = len(kp)
    rows = [(0, 0), (nk // 2, 7), (nk - 1, 15)]
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA, rows=rows)
    for k, i in rows:
        e = np.linalg.norm(got[k, i] - ref[k, i]) / np.linalg.norm(ref[k, i])
        print(f"  row {(k, i)}: rel err {e:.3e}", flush=True)
        assert e < 1e-6
