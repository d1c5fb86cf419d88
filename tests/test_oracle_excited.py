"""Pins of the excited-electron oracle (Sec. IV B, Eqs. (25)-(26)) on tiny grids,
against closed forms and invariants rather than against itself."""

import numpy as np
import pytest

from oracle import excited, lattice
from paper_1507_05156_amd import synth

OMEGA = synth.OMEGA_HSE
CELL = synth.cubic_cell()
VOL = abs(np.linalg.det(CELL))


def setting(n=8, nkm=(2, 1, 1), nb=4, seed=41):
    kp = synth.gamma_mesh(nkm[0], CELL, nkm[1], nkm[2])
    psi = synth.orbitals(n, CELL, kp, nb, seed=seed)
    return kp, psi


def test_free_electron_eigenvalues_are_the_sorted_kinetic_energies():
    """alpha = 0, no local potential: h_k = T_k, whose eigenvalues are |k+G+a|^2/2."""
    n = 8
    kp = np.array([[0.11, -0.07, 0.23], [0.3, 0.2, -0.1]])
    avec = np.array([0.02, 0.0, -0.05])
    psi = synth.orbitals(n, CELL, kp, 2, seed=1)
    eps, _ = excited.eigenstates_dense(psi, kp, CELL, OMEGA, avec, 0.0, 6)
    G = lattice.gvectors((n, n, n), lattice.reciprocal(CELL)).reshape(-1, 3)
    for k in range(2):
        ref = np.sort(0.5 * np.sum((G + kp[k] + avec) ** 2, axis=1))[:6]
        assert np.max(np.abs(eps[k] - ref)) < 1e-12


def test_model_potential_opens_a_gap_above_sixteen_bands():
    """The silicon model potential makes the lowest 16 states of h a well separated set,
    also with the Fock-like term of random orbitals added."""
    kp, psi = setting(nkm=(2, 1, 1), nb=16, seed=42)
    v = synth.model_vloc(8)
    eps, _ = excited.eigenstates_dense(psi, kp, CELL, OMEGA, np.zeros(3), 0.25, 16, vloc=v, extra=1)
    gaps = eps[:, 16] - eps[:, 15]
    assert np.all(gaps > 0.02), gaps


def test_excited_density_invariants():
    """n_ex = 0 for the eigenstates themselves and any unitary mix of them; n_ex =
    g_s N_b / Omega (all electrons excited) for orbitals from the next N_b states;
    n_ex = g_s N_b sin^2(t) / Omega for a rotation by t towards them."""
    nb = 3
    kp, psi = setting(nb=nb, seed=43)
    v = synth.model_vloc(8)
    eps, phi = excited.eigenstates_dense(psi, kp, CELL, OMEGA, np.zeros(3), 0.25, nb, vloc=v, extra=nb)
    occ, unocc = phi[:, :nb], phi[:, nb:]
    assert abs(excited.excited_density(occ, occ, CELL)) < 1e-12
    rng = np.random.default_rng(7)
    mixed = np.empty_like(occ)
    for k in range(len(kp)):
        q, _ = np.linalg.qr(rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb)))
        mixed[k] = np.tensordot(q, occ[k], axes=(1, 0))
    assert abs(excited.excited_density(occ, mixed, CELL)) < 1e-12
    full = 2.0 * nb / VOL
    assert abs(excited.excited_density(occ, unocc, CELL) - full) < 1e-12 * full
    t = 0.3
    rot = np.cos(t) * occ + np.sin(t) * unocc
    assert abs(excited.excited_density(occ, rot, CELL) - full * np.sin(t) ** 2) < 1e-12 * full


def test_dense_eigenpairs_solve_the_matrix_free_equation():
    """The dense Hamiltonian and the matrix-free h (FFT-style kinetic term, Fourier-space
    exchange operator) describe the same operator: the dense eigenpairs leave
    residuals at rounding level."""
    kp, psi = setting(nb=2, seed=44)
    v = synth.model_vloc(8)
    avec = np.array([0.0, 0.01, 0.03])
    eps, phi = excited.eigenstates_dense(psi, kp, CELL, OMEGA, avec, 0.25, 4, vloc=v)
    r = excited.residuals_matfree(psi, phi, eps, kp, CELL, OMEGA, avec, 0.25, vloc=v)
    assert np.max(r) < 1e-10


def test_eigenstates_are_orthonormal_in_the_cell_inner_product():
    kp, psi = setting(nb=2, seed=45)
    _, phi = excited.eigenstates_dense(psi, kp, CELL, OMEGA, np.zeros(3), 0.25, 5, vloc=synth.model_vloc(8))
    S = excited.overlaps(phi, phi, CELL)
    for k in range(len(kp)):
        assert np.max(np.abs(S[k] - np.eye(5))) < 1e-12


@pytest.mark.parametrize("nkm", [(1, 1, 1), (2, 1, 1)])
def test_density_is_a_k_average(nkm):
    """Duplicating every k-point with the same data leaves n_ex unchanged."""
    kp, psi = setting(nkm=nkm, nb=2, seed=46)
    v = synth.model_vloc(8)
    _, phi = excited.eigenstates_dense(psi, kp, CELL, OMEGA, np.zeros(3), 0.25, 2, vloc=v)
    a = excited.excited_density(phi, psi, CELL)
    b = excited.excited_density(np.concatenate([phi, phi]), np.concatenate([psi, psi]), CELL)
    assert abs(a - b) < 1e-14 * abs(a)
    assert 0.0 < a < 2.0 * 2 / VOL


def test_golden_fixture_is_the_oracle_output():
    """tests/golden/excited_16cube.json holds what its committed script computes from the
    oracle and the seeded inputs (dense eigh of two 4096 x 4096 Hamiltonians, about 1.5 min).
    A change to the oracle, the inputs or the fixture that breaks this agreement fails here."""
    import importlib.util
    import json
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("make_excited", os.path.join(here, "golden", "make_excited_16cube.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    with open(os.path.join(here, "golden", "excited_16cube.json")) as f:
        g = json.load(f)
    assert g["case"] == json.loads(json.dumps(mk.CASE))
    cell, kp, psi, v = mk.inputs()
    eps, phi = excited.eigenstates_dense(psi, kp, cell, mk.CASE["omega"], np.array(mk.CASE["a_over_c"]),
                                         mk.CASE["alpha"], mk.CASE["nb"], vloc=v, extra=1)
    nb = mk.CASE["nb"]
    assert np.max(np.abs(eps - np.array(g["eigenvalues"]))) < 1e-12
    nex = excited.excited_density(phi[:, :nb], psi, cell)
    assert abs(nex - g["n_ex"]) < 1e-12 * abs(g["n_ex"])
