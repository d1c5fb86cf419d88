"""Pins of the oracle's derivative and propagator routines.

Reverse-mode formulas are checked against central finite differences (an
independent route); the Taylor propagator against its exact diagonal form for
a free particle and the closed-form norm amplification; the tangent-linear
A0 derivative against central finite differences of the propagation.
"""

import numpy as np
import pytest

import oracle
from oracle import kernel as okernel
from oracle import fock as ofock
from oracle import taylor as otaylor
from paper_1507_05156_amd import synth

A = 10.26
OMEGA = 0.106


def tiny(n=6, nb=2, seed=21):
    cell = np.eye(3) * A
    kp = synth.gamma_mesh(2, cell, 1, 2)           # 4 k-points, unfolded differences
    u = synth.orbitals(n, cell, kp, nb, seed=seed, ecut=30.0)
    return cell, kp, u


def redot(x, y):
    return float(np.real(np.sum(np.conj(x) * y)))


def test_vjp_matches_central_fd():
    cell, kp, u = tiny()
    phi = synth.random_fields(u.shape, seed=22)
    g = synth.random_fields(u.shape, seed=23)
    du = synth.random_fields(u.shape, seed=24)
    dphi = synth.random_fields(u.shape, seed=25)
    du *= np.linalg.norm(u) / np.linalg.norm(du)
    dphi *= np.linalg.norm(phi) / np.linalg.norm(dphi)

    def L(uu, pp):
        return redot(g, oracle.fock_apply(uu, pp, kp, cell, OMEGA))

    h = 1e-5
    fd = (L(u + h * du, phi + h * dphi) - L(u - h * du, phi - h * dphi)) / (2 * h)
    g_u, g_phi = oracle.fock_vjp(u, phi, g, kp, cell, OMEGA)
    ad = redot(g_u, du) + redot(g_phi, dphi)
    assert abs(fd - ad) / abs(ad) < 1e-8


def test_energy_gradient_matches_fd():
    cell, kp, u = tiny(seed=26)
    d = synth.random_fields(u.shape, seed=27)
    d *= np.linalg.norm(u) / np.linalg.norm(d)
    h = 1e-5
    e = lambda x: oracle.exchange_energy(x, kp, cell, OMEGA).real
    fd = (e(u + h * d) - e(u - h * d)) / (2 * h)
    ad = redot(oracle.energy_grad(u, kp, cell, OMEGA), d)
    assert abs(fd - ad) / abs(ad) < 1e-8


def test_nyquist_average_is_needed_for_the_gradient(monkeypatch):
    """Without the Nyquist average, V_x is no longer the gradient of E_x (the pin is sensitive)."""
    cell, kp, u = tiny(n=6, seed=28)
    d = synth.random_fields(u.shape, seed=29)
    d *= np.linalg.norm(u) / np.linalg.norm(d)
    orig_ft = okernel.screened_coulomb_ft

    def table_no_avg(q, q_is_zero, n, B, w):
        L = [oracle.fftfreq_int(x) for x in n]
        L1, L2, L3 = np.meshgrid(*L, indexing="ij")
        p = q + L1[..., None] * B[0] + L2[..., None] * B[1] + L3[..., None] * B[2]
        with np.errstate(divide="ignore", invalid="ignore"):
            v = orig_ft(np.sum(p * p, -1), w)
        if q_is_zero:
            v = np.where((L1 == 0) & (L2 == 0) & (L3 == 0), np.pi / w ** 2, v)
        return v

    monkeypatch.setattr(ofock, "kernel_table", table_no_avg)
    h = 1e-5
    e = lambda x: ofock.exchange_energy(x, kp, cell, OMEGA).real
    fd = (e(u + h * d) - e(u - h * d)) / (2 * h)
    ad = redot(2.0 * 2.0 / len(kp) * oracle.volume(cell) / 216 * ofock.fock_apply(u, u, kp, cell, OMEGA), d)
    assert abs(fd - ad) / abs(ad) > 1e-7


def test_exchange_matrix_matches_fourier_route():
    cell, kp, u = tiny(n=4, seed=30)
    phi = synth.random_fields(u.shape, seed=31)
    V = oracle.fock_apply(u, phi, kp, cell, OMEGA)
    for k in range(len(kp)):
        M = otaylor.exchange_matrix(u, kp, cell, OMEGA, k)
        for i in range(u.shape[1]):
            got = (M @ phi[k, i].reshape(-1)).reshape(phi.shape[2:])
            assert np.linalg.norm(got - V[k, i]) < 1e-13 * np.linalg.norm(V[k, i])


def test_free_particle_step_is_exact_taylor_polynomial():
    """V_x = v_loc = 0: a plane wave exp(i G.r) is multiplied by T4(-i dt eps), eps = |k+G+a|^2/2."""
    cell = np.eye(3) * A
    n = (4, 4, 4)
    kp = np.array([[0.1, -0.05, 0.2]])
    avec = np.array([0.0, 0.03, -0.02])
    B = oracle.reciprocal(cell)
    G = oracle.gvectors(n, B)
    r = oracle.grid_points(n, cell)
    dt = 0.3
    for l in [(0, 0, 0), (1, 2, 3), (2, 0, 1)]:
        g = G[l]
        psi = np.exp(1j * (r @ g))[None, None]
        eps = 0.5 * np.sum((kp[0] + g + avec) ** 2)
        z = -1j * dt * eps
        t4 = sum(z ** m / [1, 1, 2, 6, 24][m]
                 for m in range(5))
        out = otaylor.step(psi, kp, cell, OMEGA, avec, dt, 0.0)
        assert np.max(np.abs(out - t4 * psi)) < 1e-13


def test_taylor_norm_amplification_formula():
    """|T4(-i x)|^2 = 1 - x^6/72 + x^8/576 for real x (stable iff x <= 2 sqrt 2)."""
    for x in [0.1, 0.7, 1.6, 2.8, 3.0]:
        z = -1j * x
        t4 = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
        assert abs(abs(t4) ** 2 - (1 - x ** 6 / 72 + x ** 8 / 576)) < 1e-13


def test_tangent_linear_a0_gradient_matches_fd():
    cell = np.eye(3) * A
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(4, cell, kp, 1, seed=32, ecut=20.0)
    args = dict(kpts=kp, a=cell, omega=OMEGA, dt=0.02, nsteps=3, alpha=0.25, omega_l=0.0569614)
    A0 = 0.05
    # E_ex is close to quadratic in A0, so a larger step keeps truncation small
    # while lifting the difference far above round-off of the O(1) energies
    h = 1e-3
    ep = otaylor.propagate(u, A0=A0 + h, **args)[1]
    em = otaylor.propagate(u, A0=A0 - h, **args)[1]
    fd = (ep - em) / (2 * h)
    tl = otaylor.propagate_tangent(u, A0=A0, **args)
    assert abs(fd - tl) / abs(tl) < 1e-7


def test_gram_schmidt_is_qr_with_positive_diagonal():
    """MGS in band order equals the Q of a QR factorisation whose R has a positive diagonal."""
    cell = np.eye(3) * A
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(6, cell, kp, 4, seed=33, orthonormal=False)
    out = oracle.gram_schmidt(u, cell)
    w = oracle.volume(cell) / 216
    for k in range(2):
        X = u[k].reshape(4, -1).T * np.sqrt(w)
        Q, R = np.linalg.qr(X)
        d = np.diag(R)
        Q = Q * (np.conj(d) / np.abs(d))
        ref = (Q / np.sqrt(w)).T.reshape(u[k].shape)
        assert np.max(np.abs(out[k] - ref)) < 1e-12 * np.max(np.abs(ref))
        S = w * out[k].reshape(4, -1).conj() @ out[k].reshape(4, -1).T
        assert np.max(np.abs(S - np.eye(4))) < 1e-13


def test_matrix_free_step_matches_dense():
    cell = np.eye(3) * A
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(4, cell, kp, 2, seed=40, ecut=20.0)
    vloc = np.random.default_rng(41).standard_normal((4, 4, 4)) * 0.1
    avec = np.array([0.01, -0.02, 0.03])
    dense = otaylor.step(u, kp, cell, OMEGA, avec, 0.05, 0.25, vloc)
    mf = otaylor.step_matfree(u, kp, cell, OMEGA, avec, 0.05, 0.25, vloc)
    assert np.max(np.abs(dense - mf)) < 1e-13


def test_matrix_free_tangent_matches_fd():
    cell = np.eye(3) * A
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(4, cell, kp, 2, seed=42, ecut=20.0)
    du = synth.random_fields(u.shape, seed=43)
    du *= np.linalg.norm(u) / np.linalg.norm(du)
    da = np.array([0.3, -0.2, 0.5])
    avec = np.array([0.01, -0.02, 0.03])
    args = dict(kpts=kp, a=cell, omega=OMEGA, dt=0.05, alpha=0.25)
    h = 1e-5
    fp = otaylor.step_matfree(u + h * du, avec=avec + h * da, **args)
    fm = otaylor.step_matfree(u - h * du, avec=avec - h * da, **args)
    fd = (fp - fm) / (2 * h)
    tl = otaylor.step_tangent_matfree(u, du, da, avec=avec, **args)
    assert np.linalg.norm(fd - tl) / np.linalg.norm(tl) < 1e-8


def test_energy_matfree_matches_dense_and_fd():
    cell = np.eye(3) * A
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(4, cell, kp, 2, seed=44, ecut=20.0)
    avec = np.array([0.01, -0.02, 0.03])
    e, g, ga = otaylor.energy_matfree(u, kp, cell, OMEGA, avec, 0.25)
    assert abs(e - otaylor.energy(u, kp, cell, OMEGA, avec, 0.25).real) < 1e-13 * abs(e)
    d = synth.random_fields(u.shape, seed=45)
    d *= np.linalg.norm(u) / np.linalg.norm(d)
    h = 1e-5
    f = lambda x, av: otaylor.energy_matfree(x, kp, cell, OMEGA, av, 0.25)[0]
    fd = (f(u + h * d, avec) - f(u - h * d, avec)) / (2 * h)
    assert abs(fd - redot(g, d)) < 1e-8 * abs(fd)
    for ax in range(3):
        da = np.zeros(3)
        da[ax] = 1.0
        fd = (f(u, avec + h * da) - f(u, avec - h * da)) / (2 * h)
        assert abs(fd - ga[ax]) < 1e-7 * max(1.0, abs(fd))


def test_step_rows_matches_full_step():
    """The single-orbital Taylor step equals the rows of the full step (v_loc and V_x on)."""
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(16, cell, kp, 2, seed=71)
    vloc = 0.1 * np.cos(2 * np.pi * np.arange(16 ** 3) / 16 ** 3)
    av = np.array([0.0, 0.01, 0.02])
    full = otaylor.step_matfree(u, kp, cell, OMEGA, av, 0.05, 0.25, vloc=vloc)
    rows = otaylor.step_rows(u, kp, cell, OMEGA, av, 0.05, 0.25, [(1, 0), (0, 1)], vloc=vloc)
    for (k, i), r in rows.items():
        assert np.linalg.norm(r - full[k, i]) < 1e-13 * np.linalg.norm(full[k, i])


def test_predictor_corrector_without_fock_is_the_midpoint_step():
    """alpha = 0: the averaged potentials are just v_loc, so the corrector is the plain step at A(t + dt/2)."""
    cell = np.eye(3) * A
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(4, cell, kp, 2, seed=51, ecut=20.0)
    vloc = 0.05 * np.cos(2 * np.pi * np.arange(64) / 64)
    an, am = np.array([0.0, 0.0, 0.02]), np.array([0.0, 0.01, 0.03])
    pc = otaylor.step_pc_matfree(u, kp, cell, OMEGA, an, am, 0.05, 0.0, vloc=vloc)
    ref = otaylor.step_matfree(u, kp, cell, OMEGA, am, 0.05, 0.0, vloc=vloc)
    assert np.linalg.norm(pc - ref) < 1e-14 * np.linalg.norm(ref)


def test_predictor_corrector_is_second_order_in_time():
    """Under a time-dependent field with the Fock term on, the global error of the
    predictor-corrector falls 4x per halved step, that of the step with h(t) frozen 2x
    (reference: the predictor-corrector at a 16x finer step)."""
    cell = np.eye(3) * A
    kp = synth.gamma_mesh(2, cell, 1, 1)
    u = synth.orbitals(4, cell, kp, 2, seed=52, ecut=12.0)
    T, A0, wl = 0.8, 0.3, 0.0569614

    def run(nsteps, pc):
        dt = T / nsteps
        psi = u.copy()
        for s_ in range(nsteps):
            t = s_ * dt
            an = otaylor.pulse_a_over_c(t, A0, wl, T)
            if pc:
                am = otaylor.pulse_a_over_c(t + 0.5 * dt, A0, wl, T)
                psi = otaylor.step_pc_matfree(psi, kp, cell, OMEGA, an, am, dt, 0.25)
            else:
                psi = otaylor.step_matfree(psi, kp, cell, OMEGA, an, dt, 0.25)
        return psi

    ref = run(160, True)
    e = {(n, pc): np.linalg.norm(run(n, pc) - ref) for n in (10, 20) for pc in (False, True)}
    r_frozen = e[(10, False)] / e[(20, False)]
    r_pc = e[(10, True)] / e[(20, True)]
    assert 1.6 < r_frozen < 2.5, (e, r_frozen)
    assert 3.3 < r_pc < 4.7, (e, r_pc)
    assert e[(20, True)] < 0.2 * e[(20, False)]
