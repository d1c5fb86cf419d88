"""Pins of the down-sampled exchange operator (Sec. II C, after Eq. (16)): the
sum over occupied orbitals runs over a sub-mesh S of the k-mesh with weight 1/|S|.

* S equal to the whole mesh gives the full operator.
* On a tiny grid the real-space double sum with the same S agrees (a route that
  never transforms the pair density).
* E_x through the pair-density spectra (Parseval) agrees with <u|V_x u>.
* For targets on S itself the operator is the full operator of the mesh S.
* The VJP matches central finite differences.
"""

import numpy as np
import pytest

import oracle
from oracle import fock as ofock
from oracle import taylor as otaylor
from paper_1507_05156_amd import synth

OMEGA = 0.106


def mesh4(n=8, nb=2, seed=81):
    """4 x 2 x 1 Gamma-centred mesh; S = every second point along x (a 2 x 2 x 1 sub-mesh)."""
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(4, cell, 2, 1)
    u = synth.orbitals(n, cell, kp, nb, seed=seed)
    src = [i for i in range(len(kp)) if (i // 2) % 2 == 0]   # x index 0 and 2 (row-major: x slowest)
    return cell, kp, u, src


def test_submesh_is_every_second_x_point():
    cell, kp, u, src = mesh4()
    f = np.round(kp @ cell.T / (2 * np.pi) * 4).astype(int)   # fractional coordinates x 4
    assert len(src) == 4
    assert all(f[i][0] % 2 == 0 for i in src)


def test_full_mesh_reduces_to_the_full_sum():
    cell, kp, u, _ = mesh4()
    a = oracle.fock_apply(u, u, kp, cell, OMEGA)
    b = oracle.fock_apply(u, u, kp, cell, OMEGA, src=list(range(len(kp))))
    assert np.array_equal(a, b)


def test_realspace_route_with_submesh():
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell, 2, 1)
    u = synth.orbitals(6, cell, kp, 2, seed=82)
    phi = synth.random_fields(u.shape, seed=83)
    src = [0, 3]
    f = oracle.fock_apply(u, phi, kp, cell, OMEGA, src=src)
    r = ofock.fock_apply_realspace(u, phi, kp, cell, OMEGA, src=src)
    assert np.linalg.norm(f - r) < 1e-12 * np.linalg.norm(r)


def test_parseval_energy_with_submesh():
    cell, kp, u, src = mesh4()
    e1 = oracle.exchange_energy(u, kp, cell, OMEGA, src=src)
    e2 = ofock.exchange_energy_parseval(u, kp, cell, OMEGA, src=src)
    assert abs(e1.imag) < 1e-13 * abs(e1.real)
    assert abs(e1.real - e2) < 1e-12 * abs(e2)
    # down-sampling changes the value (it is an approximation of the full sum)
    e_full = oracle.exchange_energy(u, kp, cell, OMEGA)
    assert abs(e_full.real - e1.real) > 1e-6 * abs(e_full.real)


def test_targets_on_the_submesh_see_the_submesh_operator():
    cell, kp, u, src = mesh4()
    a = oracle.fock_apply(u, u, kp, cell, OMEGA, src=src)[src]
    b = oracle.fock_apply(u[src], u[src], kp[src], cell, OMEGA)
    assert np.linalg.norm(a - b) < 1e-13 * np.linalg.norm(b)


def test_vjp_with_submesh_matches_central_fd():
    cell, kp, u, src = mesh4(nb=1)
    phi = synth.random_fields(u.shape, seed=85)
    g = synth.random_fields(u.shape, seed=86)
    gu, gp = oracle.adjoint.fock_vjp(u, phi, g, kp, cell, OMEGA, src=src)
    du = synth.random_fields(u.shape, seed=87)
    dp = synth.random_fields(u.shape, seed=88)
    du *= np.linalg.norm(u) / np.linalg.norm(du)       # steps on the scale of the orbitals
    dp *= np.linalg.norm(phi) / np.linalg.norm(dp)

    def loss(uu, pp):
        return np.real(np.sum(np.conj(g) * oracle.fock_apply(uu, pp, kp, cell, OMEGA, src=src)))

    h = 1e-5
    fd = (loss(u + h * du, phi + h * dp) - loss(u - h * du, phi - h * dp)) / (2 * h)
    ad = np.real(np.sum(np.conj(gu) * du)) + np.real(np.sum(np.conj(gp) * dp))
    assert abs(fd - ad) < 1e-8 * abs(ad)
    # no gradient flows to orbitals off the sub-mesh
    off = [i for i in range(len(kp)) if i not in src]
    assert np.all(gu[off] == 0)


def test_taylor_step_rows_with_submesh():
    cell, kp, u, src = mesh4()
    av = np.array([0.0, 0.0, 0.02])
    full = otaylor.step_matfree(u, kp, cell, OMEGA, av, 0.05, 0.25, src=src)
    rows = otaylor.step_rows(u, kp, cell, OMEGA, av, 0.05, 0.25, [(3, 1)], src=src)
    assert np.linalg.norm(rows[(3, 1)] - full[3, 1]) < 1e-13 * np.linalg.norm(full[3, 1])
