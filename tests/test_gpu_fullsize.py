"""Parity at the full sizes of the named workloads, in the launch configurations
bench.py times, on outputs the FP64 oracle evaluates one by one.

* 32^3 grid, 6^3 k, 16 bands, FP32 form (the bench workload): sampled output rows,
  each a sum over all 3,456 source orbitals.
* Three uneven cells in one captured launch, in the default form (each cell's kernel on
  a forked stream) and in the persistent kernel's form: one sampled row per cell.
* 24^3 grid, 4^3 k, 16 bands, FP64: one Taylor-4 step, sampled rows.
* The same cell through 20 checkpointed steps in the fused FP64 form: dE_ex/dA0 by
  the adjoint against central finite differences (about 3 minutes of GPU time).
"""

import numpy as np
import pytest

import oracle
from oracle import taylor as otaylor
from paper_1507_05156_amd import synth

pytestmark = pytest.mark.gpu

OMEGA = synth.OMEGA_HSE


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def row_err(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def test_bench_workload_fp32_sampled_rows(device):
    """32^3 / 216 k / 16 bands through the fused FP32 kernel, as bench.py runs it (the
    split form: targets t run on CU pair t mod 128, XCD (t mod 128) / 16, round t / 128;
    each target's two halves hold the even and odd m1 planes). One sampled row per XCD,
    spread over the rounds, the first and the last target among them."""
    print("[gpu] full size 32^3 fp32 rows", flush=True)
    from paper_1507_05156_amd.api import Plan
    from tests.oracle_rows import oracle_rows
    cell, kp, u = synth.workload(2)
    plan = Plan(dict(n=32, a=cell, kpts=kp, nb=16, omega=OMEGA), prec="fp32")
    plan.profile(True)
    got = plan.apply(to_dev(u)).cpu().numpy()
    assert plan.profile_fallbacks() == 0
    plan.profile(False)
    targets = [0, 128 * 5 + 16 + 3, 128 * 9 + 32 + 8, 128 * 13 + 48 + 12, 128 * 17 + 64 + 1, 128 * 21 + 80 + 15,
               128 * 24 + 96 + 6, 3455]
    rows = [(t // 16, t % 16) for t in targets]
    ref = oracle_rows(u, kp, cell, OMEGA, rows)
    for k, i in rows:
        e = row_err(got[k, i], ref[(k, i)])
        print(f"  row {(k, i)}: rel err {e:.3e}", flush=True)
        assert e < 1e-6, (k, i, e)


def test_bench_workload_fp32_every_k_vs_fp64(device):
    """The same application against the plain FP64 GPU path at every one of the 216
    k-points (the per-k error bench.py reports), and E_x."""
    print("[gpu] full size 32^3 fp32 vs fp64 at every k", flush=True)
    from paper_1507_05156_amd.api import Plan
    cell, kp, u = synth.workload(2)
    d = to_dev(u)
    p32 = Plan(dict(n=32, a=cell, kpts=kp, nb=16, omega=OMEGA), prec="fp32")
    o32 = p32.apply(d)
    p32.close()
    p64 = Plan(dict(n=32, a=cell, kpts=kp, nb=16, omega=OMEGA), prec="fp64")
    o64 = p64.apply(d)
    rel = ((o32 - o64).reshape(len(kp), -1).norm(dim=1) / o64.reshape(len(kp), -1).norm(dim=1)).cpu().numpy()
    print(f"  per-k rel err max {rel.max():.3e} median {np.median(rel):.3e}", flush=True)
    assert rel.max() < 1e-6


def _batched_plan(cells, form=None, tmp_path=None):
    """The three-cell plan; with `form`, that batched form forced through a tuning cache."""
    import json

    import torch
    from paper_1507_05156_amd.api import Plan
    if form is None:
        return Plan(cells, prec="fp32")
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = f"{arch}/fp32/batched" + "".join(
        f"/{arch}/fp32/cell/n{c['n']}x{c['n']}x{c['n']}/nt{len(c['kpts'])}/ns{len(c['kpts'])}/nb{c['nb']}/nx{c['nb']}"
        for c in cells)
    path = tmp_path / f"tune_batched_{form}.json"
    path.write_text(json.dumps({key: {"form": form, "wg_per_cu": 1, "ms": 0}}))
    return Plan(cells, prec="fp32", tune_cache=str(path))


@pytest.mark.parametrize("form", [None, 0])
def test_batched_workload_sampled_rows(device, tmp_path, form):
    """16^3/27 k/8 b, 20^3/64 k/12 b and 24^3/125 k/16 b in one captured launch: the
    default form (each cell's kernel on a forked stream) and the persistent kernel
    (form 0, forced through the tuning cache), each against the oracle on one row per
    cell and against each other at every k-point."""
    print(f"[gpu] full size batched rows, form {form}", flush=True)
    from tests.oracle_rows import oracle_rows
    cells, us = [], []
    for ci in range(3):
        a, kp, u = synth.workload(4, ci)
        cells.append(dict(n=u.shape[2], a=a, kpts=kp, nb=u.shape[1], omega=OMEGA))
        us.append(u)
    plan = _batched_plan(cells, form, tmp_path)
    outs = [o.cpu().numpy() for o in plan.apply_batched([to_dev(u) for u in us])]
    for ci, (c, u) in enumerate(zip(cells, us)):
        k, i = c["kpts"].shape[0] - 1, c["nb"] // 2
        ref = oracle_rows(u, c["kpts"], c["a"], OMEGA, [(k, i)], workers=1)[(k, i)]
        e = row_err(outs[ci][k, i], ref)
        print(f"  cell {ci} row {(k, i)}: rel err {e:.3e}", flush=True)
        assert e < 1e-6, (ci, e)
    if form is not None:
        other = [o.cpu().numpy() for o in _batched_plan(cells).apply_batched([to_dev(u) for u in us])]
        for ci in range(3):
            nk = outs[ci].shape[0]
            d = max(np.linalg.norm(outs[ci][k] - other[ci][k]) / np.linalg.norm(other[ci][k]) for k in range(nk))
            print(f"  cell {ci}: persistent vs forked, max per-k {d:.3e}", flush=True)
            assert d < 1e-6


def test_differentiation_workload_taylor_step_rows(device):
    """One FP64 Taylor-4 step at 24^3 / 64 k / 16 bands with a field and alpha = 1/4."""
    print("[gpu] full size 24^3 taylor rows", flush=True)
    from paper_1507_05156_amd.api import Plan
    cell, kp, u = synth.workload(3)
    plan = Plan(dict(n=24, a=cell, kpts=kp, nb=16, omega=OMEGA), prec="fp64")
    avec = np.array([0.0, 0.0, 0.03])
    psi = to_dev(u)
    plan.taylor_step(psi, avec, 0.02, 0.25)
    got = psi.cpu().numpy()
    rows = [(5, 3), (63, 15)]
    ref = otaylor.step_rows(u, kp, cell, OMEGA, avec, 0.02, 0.25, rows)
    for (k, i), r in ref.items():
        e = row_err(got[k, i], r)
        print(f"  row {(k, i)}: rel err {e:.3e}", flush=True)
        assert e < 1e-10, (k, i, e)


class _Progress:
    """Delegates to a Plan and prints a line per Taylor step and per adjoint step, so
    that a long propagation shows it is moving."""

    def __init__(self, plan):
        self._plan = plan
        self.fwd = 0
        self.bwd = 0

    def __getattr__(self, name):
        return getattr(self._plan, name)

    def taylor_step(self, *a, **k):
        self.fwd += 1
        print(f"  taylor step {self.fwd}", flush=True)
        return self._plan.taylor_step(*a, **k)

    def taylor_step_vjp(self, *a, **k):
        self.bwd += 1
        print(f"  adjoint step {self.bwd}", flush=True)
        return self._plan.taylor_step_vjp(*a, **k)


def test_differentiation_workload_a0_gradient_fd(device):
    """dE_ex/dA0 through 20 Taylor-4 steps (dt = 0.02, sin^2 pulse, 1.55 eV, A0 = 0.05,
    checkpoints every 5 steps) at 24^3 / 64 k / 16 bands, in the fused FP64 form: the
    adjoint against the central difference at h = 1e-5 and against a fourth-order
    stencil at h = 1e-2, both to 1e-6 relative.

    E_ex = E(T) - E(0) is a difference of two energies near 86 Ha. The library reduces
    both in double-double and subtracts them before rounding (taylor_excitation_energy),
    so E_ex keeps FP64 relative precision of its own; with one unit in the last place of
    86 Ha as its error the h = 1e-5 quotient would move by 2e-4 of this gradient."""
    print("[gpu] full size 24^3 A0 gradient (fp64f)", flush=True)
    import torch
    from paper_1507_05156_amd import autograd as ag
    from paper_1507_05156_amd.api import Plan
    cell, kp, u = synth.workload(3)
    plan = _Progress(Plan(dict(n=24, a=cell, kpts=kp, nb=16, omega=OMEGA), prec="fp64f"))
    kw = dict(nsteps=20, dt=0.02, alpha=0.25, omega_l=0.0569614, checkpoint_every=5)
    A0 = torch.tensor(0.05, dtype=torch.float64, requires_grad=True)
    _, eex = ag.propagate(plan, to_dev(u), A0, **kw)
    eex.backward()
    ad = float(A0.grad)

    def e_ex(a):
        print(f"  E_ex at A0 = {a:.6f}", flush=True)
        return float(ag.propagate(plan, to_dev(u), torch.tensor(a, dtype=torch.float64), **kw)[1])

    with torch.no_grad():
        h = 1e-5
        fd2 = (e_ex(0.05 + h) - e_ex(0.05 - h)) / (2 * h)
        h4 = 1e-2
        d1 = e_ex(0.05 + h4) - e_ex(0.05 - h4)
        d2 = e_ex(0.05 + 2 * h4) - e_ex(0.05 - 2 * h4)
        fd4 = (8 * d1 - d2) / (12 * h4)
    r2, r4 = abs(fd2 - ad) / abs(ad), abs(fd4 - ad) / abs(ad)
    print(f"  E_ex = {float(eex.detach()):.15e}, adjoint {ad:.12e}, central FD (h=1e-5) {fd2:.12e} rel {r2:.3e}, "
          f"4th-order FD (h=1e-2) {fd4:.12e} rel {r4:.3e}", flush=True)
    assert r2 <= 1e-6 and r4 <= 1e-6
