"""Dense-matrix Taylor propagation and its A0 derivative (Eqs. (2), (9)-(10), (21), (22)).

Tiny cells only (N_r up to a few hundred): every operator is an explicit
N_r x N_r matrix per k-point.

Hamiltonian of one step (velocity gauge, Eq. (2); HSE enters through the
Fock-like term with weight alpha = 1/4, Eq. (8)):

    h_k = T_k[A/c] + diag(v_loc) + alpha * V_x[psi(t_n)]
    T_k[a] = IDFT diag( |k + G + a|^2 / 2 ) DFT / N_r        (spectral kinetic operator)

Following the paper, h(t + dt/2) is replaced by h(t_n): A = A(t_n) and V_x is
built from psi(t_n) and frozen for the four Taylor terms. The step is

    psi(t_n + dt) = sum_{m=0}^{4} (-i dt h)^m / m! psi(t_n).

Pulse (Eq. (21)) with A0 the amplitude of A/c:
    A(t)/c = -A0 cos(w_L t) sin^2(pi t / T_d) e_z   for 0 < t < T_d, else 0.

Energy (Eq. (22) without the ionic/Hartree/PBE pieces, E_GS replaced by the
energy of the initial state):
    E[psi; a] = (g_s/N_k)(Omega/N_r) sum conj(psi) (T[a] + v_loc) psi + alpha E_x[psi]
    E_ex = E[psi(t_N); a(t_N)] - E[psi(t_0); a(t_0)].

dE_ex/dA0 is computed by tangent-linear (forward-mode) propagation, a route
independent of any reverse-mode code.
"""

import numpy as np

from .dft import dft3_full
from .kernel import kernel_table
from .lattice import reciprocal, volume, gvectors, grid_points


def _dft_matrix_full(n):
    nr = int(np.prod(n))
    eye = np.eye(nr, dtype=np.complex128).reshape((nr,) + tuple(n))
    return dft3_full(eye, -1).reshape(nr, nr).T        # column m -> spectrum


def kinetic_matrix(n, a, k, avec):
    """T_k[a] as a dense N_r x N_r matrix acting on flattened periodic parts."""
    B = reciprocal(a)
    G = gvectors(n, B).reshape(-1, 3)
    eps = 0.5 * np.sum((G + np.asarray(k) + np.asarray(avec)) ** 2, axis=1)
    F = _dft_matrix_full(n)
    nr = F.shape[0]
    return (np.conj(F).T @ (eps[:, None] * F)) / nr


def kinetic_dmatrix(n, a, k, avec, axis):
    """d T_k[a] / d a_axis (dense)."""
    B = reciprocal(a)
    G = gvectors(n, B).reshape(-1, 3)
    deps = (G + np.asarray(k) + np.asarray(avec))[:, axis]
    F = _dft_matrix_full(n)
    nr = F.shape[0]
    return (np.conj(F).T @ (deps[:, None] * F)) / nr


def exchange_matrix(u, kpts, a, omega, k):
    """Dense V_x[u] for output k-point k: -(1/N_k) sum_{k'j} u_j(m) C_{kk'}(m - m') conj(u_j(m'))."""
    u = np.asarray(u, dtype=np.complex128)
    kpts = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
    nk, nb = u.shape[:2]
    n = u.shape[-3:]
    nr = int(np.prod(n))
    B = reciprocal(a)
    G = gvectors(n, B).reshape(-1, 3)
    r = grid_points(n, a).reshape(-1, 3)
    E = np.exp(1j * (r @ G.T))                            # E[m, l] = exp(i G_l . r_m)
    V = np.zeros((nr, nr), dtype=np.complex128)
    for kp in range(nk):
        K = kernel_table(kpts[k] - kpts[kp], k == kp, n, B, omega).reshape(-1)
        C = (E * K[None, :]) @ np.conj(E).T / nr          # C[m, m'] = (1/N_r) sum_l K_l e^{iG(r_m - r_m')}
        for j in range(nb):
            uj = u[kp, j].reshape(-1)
            V -= (uj[:, None] * C * np.conj(uj)[None, :]) / nk
    return V


def exchange_dmatrix_apply(u, du, kpts, a, omega, k, phi):
    """Directional derivative of V_x[u] phi along du (real-linear in du)."""
    u = np.asarray(u, dtype=np.complex128)
    du = np.asarray(du, dtype=np.complex128)
    kpts = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
    nk, nb = u.shape[:2]
    n = u.shape[-3:]
    nr = int(np.prod(n))
    B = reciprocal(a)
    G = gvectors(n, B).reshape(-1, 3)
    r = grid_points(n, a).reshape(-1, 3)
    E = np.exp(1j * (r @ G.T))
    out = np.zeros(nr, dtype=np.complex128)
    phi = phi.reshape(-1)
    for kp in range(nk):
        K = kernel_table(kpts[k] - kpts[kp], k == kp, n, B, omega).reshape(-1)
        C = (E * K[None, :]) @ np.conj(E).T / nr
        for j in range(nb):
            uj = u[kp, j].reshape(-1)
            duj = du[kp, j].reshape(-1)
            out -= (duj * (C @ (np.conj(uj) * phi)) + uj * (C @ (np.conj(duj) * phi))) / nk
    return out


def pulse_a_over_c(t, A0, omega_l, Td, direction=(0.0, 0.0, 1.0)):
    """A(t)/c of Eq. (21) with A0 the amplitude of A/c."""
    if 0.0 < t < Td:
        s = -A0 * np.cos(omega_l * t) * np.sin(np.pi * t / Td) ** 2
    else:
        s = 0.0
    return s * np.asarray(direction, dtype=np.float64)


def step(psi, kpts, a, omega, avec, dt, alpha, vloc=None, order=4):
    """One Taylor step psi(t_n) -> psi(t_n + dt) with dense h_k (V_x frozen at psi(t_n))."""
    psi = np.asarray(psi, dtype=np.complex128)
    nk, nb = psi.shape[:2]
    n = psi.shape[-3:]
    out = np.empty_like(psi)
    for k in range(nk):
        h = kinetic_matrix(n, a, kpts[k], avec)
        if vloc is not None:
            h = h + np.diag(np.asarray(vloc, dtype=np.float64).reshape(-1))
        if alpha != 0.0:
            h = h + alpha * exchange_matrix(psi, kpts, a, omega, k)
        for b in range(nb):
            x = psi[k, b].reshape(-1)
            term = x.copy()
            acc = x.copy()
            for m in range(1, order + 1):
                term = (-1j * dt / m) * (h @ term)
                acc = acc + term
            out[k, b] = acc.reshape(n)
    return out


def energy(psi, kpts, a, omega, avec, alpha, vloc=None, gs=2.0):
    psi = np.asarray(psi, dtype=np.complex128)
    nk = psi.shape[0]
    n = psi.shape[-3:]
    nr = int(np.prod(n))
    w = gs / nk * volume(a) / nr
    e = 0.0
    for k in range(nk):
        h = kinetic_matrix(n, a, kpts[k], avec)
        if vloc is not None:
            h = h + np.diag(np.asarray(vloc, dtype=np.float64).reshape(-1))
        if alpha != 0.0:
            h = h + 0.5 * alpha * exchange_matrix(psi, kpts, a, omega, k)
        for b in range(psi.shape[1]):
            x = psi[k, b].reshape(-1)
            e += w * np.vdot(x, h @ x)
    return e


def propagate(psi0, kpts, a, omega, A0, dt, nsteps, alpha, omega_l, vloc=None, direction=(0, 0, 1)):
    """Returns (psi_N, E_ex) for nsteps Taylor steps with the pulse of Eq. (21), T_d = nsteps*dt."""
    Td = nsteps * dt
    psi = np.asarray(psi0, dtype=np.complex128)
    e0 = energy(psi, kpts, a, omega, pulse_a_over_c(0.0, A0, omega_l, Td, direction), alpha, vloc).real
    for s in range(nsteps):
        avec = pulse_a_over_c(s * dt, A0, omega_l, Td, direction)
        psi = step(psi, kpts, a, omega, avec, dt, alpha, vloc)
    eN = energy(psi, kpts, a, omega, pulse_a_over_c(nsteps * dt, A0, omega_l, Td, direction), alpha, vloc).real
    return psi, eN - e0


def propagate_tangent(psi0, kpts, a, omega, A0, dt, nsteps, alpha, omega_l, vloc=None, direction=(0, 0, 1),
                      gs=2.0):
    """Forward-mode derivative dE_ex/dA0 through the same propagation."""
    Td = nsteps * dt
    psi = np.asarray(psi0, dtype=np.complex128)
    nk, nb = psi.shape[:2]
    n = psi.shape[-3:]
    nr = int(np.prod(n))
    dpsi = np.zeros_like(psi)
    direction = np.asarray(direction, dtype=np.float64)
    for s in range(nsteps):
        t = s * dt
        avec = pulse_a_over_c(t, A0, omega_l, Td, direction)
        davec = pulse_a_over_c(t, 1.0, omega_l, Td, direction)     # d a / d A0
        new = np.empty_like(psi)
        dnew = np.empty_like(psi)
        for k in range(nk):
            h = kinetic_matrix(n, a, kpts[k], avec)
            dT = sum(davec[d] * kinetic_dmatrix(n, a, kpts[k], avec, d) for d in range(3) if davec[d] != 0.0)
            if isinstance(dT, int):
                dT = np.zeros((nr, nr), dtype=np.complex128)
            if vloc is not None:
                h = h + np.diag(np.asarray(vloc, dtype=np.float64).reshape(-1))
            if alpha != 0.0:
                h = h + alpha * exchange_matrix(psi, kpts, a, omega, k)
            for b in range(nb):
                x = psi[k, b].reshape(-1)
                dx = dpsi[k, b].reshape(-1)
                term, dterm = x.copy(), dx.copy()
                acc, dacc = x.copy(), dx.copy()
                for m in range(1, 5):
                    dh_term = dT @ term
                    if alpha != 0.0:
                        dh_term = dh_term + alpha * exchange_dmatrix_apply(psi, dpsi, kpts, a, omega, k, term)
                    dterm = (-1j * dt / m) * (h @ dterm + dh_term)
                    term = (-1j * dt / m) * (h @ term)
                    acc = acc + term
                    dacc = dacc + dterm
                new[k, b] = acc.reshape(n)
                dnew[k, b] = dacc.reshape(n)
        psi, dpsi = new, dnew
    # dE(t_N): a(t_N) = 0 and da(t_N)/dA0 = 0, so only psi_N varies
    aN = pulse_a_over_c(nsteps * dt, A0, omega_l, Td, direction)
    w = gs / nk * volume(a) / nr
    de = 0.0
    for k in range(nk):
        h = kinetic_matrix(n, a, kpts[k], aN)
        if vloc is not None:
            h = h + np.diag(np.asarray(vloc, dtype=np.float64).reshape(-1))
        if alpha != 0.0:
            h = h + alpha * exchange_matrix(psi, kpts, a, omega, k)   # d(E_x)/dpsi = 2 w V_x psi (x alpha)
        for b in range(nb):
            x = psi[k, b].reshape(-1)
            de += 2.0 * w * np.real(np.vdot(h @ x, dpsi[k, b].reshape(-1)))
    return de


# ----------------------------------------------------------- matrix-free forms
# The same operators applied without forming N_r x N_r matrices (separable naive
# DFTs for the kinetic term, the Fourier-space exchange operator of fock.py), so
# that grids of the supported lengths (16^3 and up) stay affordable.

def kinetic_apply(x, kpts, a, avec):
    """T_k[a] x for x [nk][nb][n1][n2][n3]: IDFT(|k+G+a|^2/2 DFT x)/N_r."""
    from .dft import dft3
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-3:]
    nr = int(np.prod(n))
    B = reciprocal(a)
    G = gvectors(n, B)
    out = np.empty_like(x)
    for k in range(x.shape[0]):
        eps = 0.5 * np.sum((G + np.asarray(kpts[k]) + np.asarray(avec)) ** 2, axis=-1)
        out[k] = dft3(eps * dft3(x[k], -1), +1) / nr
    return out


def kinetic_dapply(x, kpts, a, avec, axis):
    """(d T_k[a] / d a_axis) x."""
    from .dft import dft3
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-3:]
    nr = int(np.prod(n))
    B = reciprocal(a)
    G = gvectors(n, B)
    out = np.empty_like(x)
    for k in range(x.shape[0]):
        d = (G + np.asarray(kpts[k]) + np.asarray(avec))[..., axis]
        out[k] = dft3(d * dft3(x[k], -1), +1) / nr
    return out


def h_apply(u, x, kpts, a, omega, avec, alpha, vloc=None, src=None):
    """h x with h = T[a] + v_loc + alpha V_x[u] (V_x over the source sub-mesh src)."""
    from .fock import fock_apply
    y = kinetic_apply(x, kpts, a, avec)
    if vloc is not None:
        y = y + np.asarray(vloc).reshape(x.shape[-3:]) * x
    if alpha != 0.0:
        y = y + alpha * fock_apply(u, x, kpts, a, omega, src=src)
    return y


def step_matfree(psi, kpts, a, omega, avec, dt, alpha, vloc=None, order=4, src=None):
    psi = np.asarray(psi, dtype=np.complex128)
    term = psi.copy()
    acc = psi.copy()
    for m in range(1, order + 1):
        term = (-1j * dt / m) * h_apply(psi, term, kpts, a, omega, avec, alpha, vloc, src=src)
        acc = acc + term
    return acc


def step_pc_matfree(psi, kpts, a, omega, avec_now, avec_mid, dt, alpha, vloc=None, order=4, src=None):
    """The predictor-corrector step (Sec. II C, Eqs. (11)-(13)) for the HSE functional.

    Predictor: psi_pred = T_order(h(t)) psi with h(t) = T[A(t)/c] + v_loc + alpha V_x[psi].
    The potentials at t + dt/2 are the averages of those at t and at t + dt built
    from psi_pred; for HSE that is alpha (V_x[psi] + V_x[psi_pred]) / 2. The
    field is external and known exactly, so the corrector takes A(t + dt/2).
    Corrector: psi(t + dt) = T_order(h_c) psi with that averaged operator.
    """
    from .fock import fock_apply
    psi = np.asarray(psi, dtype=np.complex128)
    pred = step_matfree(psi, kpts, a, omega, avec_now, dt, alpha, vloc, order, src=src)
    term = psi.copy()
    acc = psi.copy()
    for m in range(1, order + 1):
        y = kinetic_apply(term, kpts, a, avec_mid)
        if vloc is not None:
            y = y + np.asarray(vloc).reshape(psi.shape[-3:]) * term
        if alpha != 0.0:
            y = y + 0.5 * alpha * (fock_apply(psi, term, kpts, a, omega, src=src)
                                   + fock_apply(pred, term, kpts, a, omega, src=src))
        term = (-1j * dt / m) * y
        acc = acc + term
    return acc


def step_rows(psi, kpts, a, omega, avec, dt, alpha, rows, vloc=None, order=4, src=None):
    """The Taylor step of Eqs. (9)-(10) for the listed orbitals (k, i) only.

    Once V_x is built from psi(t_n), h acts on each orbital by itself: the
    kinetic term on its own k, v_loc pointwise, V_x through the pair sum over
    all occupied (k', j). So the terms phi_m = (-i dt/m) h phi_{m-1} of one
    orbital need that orbital alone. Returns {(k, i): psi_ki(t_n + dt)}.
    """
    from .fock import general_apply
    psi = np.asarray(psi, dtype=np.complex128)
    kpts = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
    nk = psi.shape[0]
    n = psi.shape[-3:]
    out = {}
    for k, i in rows:
        term = psi[k, i].copy()
        acc = term.copy()
        for m in range(1, order + 1):
            y = kinetic_apply(term[None, None], kpts[k:k + 1], a, avec)[0, 0]
            if vloc is not None:
                y = y + np.asarray(vloc).reshape(n) * term
            if alpha != 0.0:
                X = np.zeros((nk, 1) + tuple(n), dtype=np.complex128)
                X[k, 0] = term
                y = y + alpha * general_apply(X, psi, psi, kpts, a, omega, rows=[(k, 0)], src=src)[k, 0]
            term = (-1j * dt / m) * y
            acc = acc + term
        out[(k, i)] = acc
    return out


def step_tangent_matfree(psi, dpsi, davec, kpts, a, omega, avec, dt, alpha, vloc=None, order=4):
    """Forward-mode derivative of step_matfree along (dpsi, davec)."""
    from .fock import general_apply
    psi = np.asarray(psi, dtype=np.complex128)
    dpsi = np.asarray(dpsi, dtype=np.complex128)
    term, dterm = psi.copy(), dpsi.copy()
    dacc = dpsi.copy()
    for m in range(1, order + 1):
        dh = sum(davec[d] * kinetic_dapply(term, kpts, a, avec, d) for d in range(3))
        if alpha != 0.0:
            # derivative of V_x[u] term in the occupied orbitals (both occurrences)
            dh = dh + alpha * (general_apply(term, psi, dpsi, kpts, a, omega)
                               + general_apply(term, dpsi, psi, kpts, a, omega))
        dterm = (-1j * dt / m) * (h_apply(psi, dterm, kpts, a, omega, avec, alpha, vloc) + dh)
        term = (-1j * dt / m) * h_apply(psi, term, kpts, a, omega, avec, alpha, vloc)
        dacc = dacc + dterm
    return dacc


def energy_matfree(psi, kpts, a, omega, avec, alpha, vloc=None, gs=2.0):
    """E[psi; a] and its gradient in the PyTorch convention."""
    from .fock import fock_apply
    psi = np.asarray(psi, dtype=np.complex128)
    nk = psi.shape[0]
    nr = int(np.prod(psi.shape[-3:]))
    w = gs / nk * volume(a) / nr
    tv = kinetic_apply(psi, kpts, a, avec)
    if vloc is not None:
        tv = tv + np.asarray(vloc).reshape(psi.shape[-3:]) * psi
    vx = fock_apply(psi, psi, kpts, a, omega) if alpha != 0.0 else np.zeros_like(psi)
    e = w * np.real(np.sum(np.conj(psi) * tv)) + 0.5 * alpha * w * np.real(np.sum(np.conj(psi) * vx))
    grad = 2.0 * w * (tv + alpha * vx)
    grad_a = np.array([w * np.real(np.sum(np.conj(psi) * kinetic_dapply(psi, kpts, a, avec, d))) for d in range(3)])
    return e, grad, grad_a


# ------------------------------------------------- current and work (Eqs. (3)-(4), (23)-(24))
# Velocity gauge, no nonlocal pseudopotential (J_NL = 0), atomic units, electron
# charge -1. For Bloch orbitals psi = exp(i k.r) u, the cell integral of
# Re[psi* (-i grad + A/c) psi] is, by Parseval, (Omega/N_r^2) sum_l (k+G_l+A/c) |DFT(u)_l|^2.

def current(psi, kpts, a, avec, gs=2.0):
    """J(t) = -(1/Omega) (g_s/N_k) sum_{k,b} int_cell Re[psi* (-i grad + A/c) psi] dr."""
    from .dft import dft3
    psi = np.asarray(psi, dtype=np.complex128)
    n = psi.shape[-3:]
    nr = int(np.prod(n))
    nk = psi.shape[0]
    G = gvectors(n, reciprocal(a))
    total = np.zeros(3)
    for k in range(nk):
        p2 = np.sum(np.abs(dft3(psi[k], -1)) ** 2, axis=0)          # sum over bands of |DFT u|^2
        vel = G + np.asarray(kpts[k]) + np.asarray(avec)            # k + G + A/c
        total += np.tensordot(p2, vel, axes=([0, 1, 2], [0, 1, 2]))
    vol = volume(a)
    return -(1.0 / vol) * (gs / nk) * (vol / nr ** 2) * total


def electric_field(t, A0, omega_l, Td, direction=(0.0, 0.0, 1.0)):
    """E(t) = -(1/c) dA/dt for the pulse of Eq. (21) (pulse_a_over_c), differentiated by hand."""
    if 0.0 < t < Td:
        s2 = np.sin(np.pi * t / Td) ** 2
        ds2 = (np.pi / Td) * np.sin(2.0 * np.pi * t / Td)
        da = -A0 * (-omega_l * np.sin(omega_l * t) * s2 + np.cos(omega_l * t) * ds2)
    else:
        da = 0.0
    return -da * np.asarray(direction, dtype=np.float64)


def work_and_energy(psi0, kpts, a, omega, A0, dt, nsteps, alpha, omega_l, vloc=None, direction=(0, 0, 1),
                    gs=2.0):
    """The excitation energy at t_N two ways (the equality of Eq. (23) and Eq. (24) for a
    functional-derived potential): E_ex = E[psi(t_N); A(t_N)] - E[psi(t_0); A(t_0)] and
    Omega * W with W = int J.E dt, J(t_n) from psi(t_n), the trapezoid rule over the steps,
    T_d = nsteps * dt. Returns (E_ex, Omega W, [J(t_n)])."""
    Td = nsteps * dt
    psi = np.asarray(psi0, dtype=np.complex128)
    js, es = [], []
    for s_ in range(nsteps + 1):
        t = s_ * dt
        av = pulse_a_over_c(t, A0, omega_l, Td, direction)
        js.append(current(psi, kpts, a, av, gs))
        es.append(electric_field(t, A0, omega_l, Td, direction))
        if s_ < nsteps:
            psi = step_matfree(psi, kpts, a, omega, av, dt, alpha, vloc)
    jE = np.array([np.dot(j, e) for j, e in zip(js, es)])
    w = dt * (0.5 * jE[0] + jE[1:-1].sum() + 0.5 * jE[-1])
    e0 = energy_matfree(psi0, kpts, a, omega, pulse_a_over_c(0.0, A0, omega_l, Td, direction), alpha, vloc, gs)[0]
    eN = energy_matfree(psi, kpts, a, omega, pulse_a_over_c(Td, A0, omega_l, Td, direction), alpha, vloc, gs)[0]
    return eN - e0, volume(a) * w, np.array(js)
