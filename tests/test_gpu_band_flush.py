"""More bands than one FP32 partial sum holds: the fused FP32 forms add their FP32 band
sums into the Neumaier-compensated FP64 sum after at most 16 bands, so the error does
not grow with the band count. 48 bands per k-point against the FP64 oracle at 16^3
(grid form, every row), 24^3 and 32^3 (split form, sampled rows)."""

import numpy as np
import pytest

import oracle
from paper_1507_05156_amd import synth

pytestmark = pytest.mark.gpu

OMEGA = synth.OMEGA_HSE


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.mark.parametrize("n,mesh,rows", [(16, (2, 1, 1), None), (24, (1, 1, 1), [(0, 0), (0, 47)]),
                                         (32, (1, 1, 1), [(0, 5), (0, 47)])])
def test_48_bands_fp32_form(device, n, mesh, rows):
    print(f"[gpu] 48 bands, {n}^3, mesh {mesh}", flush=True)
    from paper_1507_05156_amd.api import Plan
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(mesh[0], cell, mesh[1], mesh[2])
    u = synth.orbitals(n, cell, kp, 48, seed=900 + n)
    plan = Plan(dict(n=n, a=cell, kpts=kp, nb=48, omega=OMEGA), prec="fp32")
    got = plan.apply(to_dev(u)).cpu().numpy()
    ref = oracle.fock_apply(u, u, kp, cell, OMEGA, rows=rows)
    for k, i in (rows or [(k, i) for k in range(len(kp)) for i in range(48)]):
        e = np.linalg.norm(got[k, i] - ref[k, i]) / np.linalg.norm(ref[k, i])
        assert e < 1e-6, (k, i, e)
    if rows is None:
        e = max(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k]) for k in range(len(kp)))
        print(f"  per-k rel err {e:.3e}", flush=True)
