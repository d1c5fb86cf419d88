"""Current and work of the laser field along a Taylor-propagated trajectory.

For a potential derived from an energy functional (HSE is), the work done by
the field (Eq. (24)), W(t) = int J.E dt, equals the excitation energy of the
functional (Eq. (23)) per unit volume: Omega W(t) = E[psi(t); A(t)] - E[psi(0); A(0)].
On the time grid the two differ by an error linear in the step (the field is
held at A(t_n) over each step), and that difference checks the propagator's
energy consistency. Every operator runs in the library; this module only
steps through time and sums host scalars.
"""

from __future__ import annotations

import math

import numpy as np


def pulse_a_over_c(t, A0, omega_l, Td, direction=(0.0, 0.0, 1.0)):
    """A(t)/c of Eq. (21): -A0 cos(omega_l t) sin^2(pi t/Td) along direction, zero outside (0, Td)."""
    s = -A0 * math.cos(omega_l * t) * math.sin(math.pi * t / Td) ** 2 if 0.0 < t < Td else 0.0
    return s * np.asarray(direction, dtype=np.float64)


def electric_field(t, A0, omega_l, Td, direction=(0.0, 0.0, 1.0)):
    """E(t) = -(1/c) dA/dt for pulse_a_over_c."""
    if 0.0 < t < Td:
        s2 = math.sin(math.pi * t / Td) ** 2
        ds2 = (math.pi / Td) * math.sin(2.0 * math.pi * t / Td)
        da = -A0 * (-omega_l * math.sin(omega_l * t) * s2 + math.cos(omega_l * t) * ds2)
    else:
        da = 0.0
    return -da * np.asarray(direction, dtype=np.float64)


def work_and_energy(plan, psi0, A0, dt, nsteps, alpha=0.25, omega_l=0.0569614, vloc=None,
                    direction=(0.0, 0.0, 1.0), cell=0, predictor_corrector=False):
    """Propagate psi0 through nsteps Taylor steps under the pulse (T_d = nsteps dt), with
    h held at t_n or, with predictor_corrector, by the predictor-corrector step, and return

    (E_ex, Omega W, J) with E_ex the energy-functional difference between t_N and t_0,
    W = int J.E dt by the trapezoid rule over the time grid, and J [nsteps+1][3] the
    current at each t_n (from psi(t_n) and A(t_n))."""
    Td = nsteps * dt
    vol = plan.cells[cell]["vol"]
    psi = psi0.clone()
    js, es = [], []
    for s in range(nsteps + 1):
        t = s * dt
        a = pulse_a_over_c(t, A0, omega_l, Td, direction)
        js.append(plan.current(psi, a, cell))
        es.append(electric_field(t, A0, omega_l, Td, direction))
        if s < nsteps and predictor_corrector:
            a_mid = pulse_a_over_c(t + 0.5 * dt, A0, omega_l, Td, direction)
            plan.taylor_step_pc(psi, a, a_mid, dt, alpha, vloc=vloc, cell=cell, want_norm=False)
        elif s < nsteps:
            plan.taylor_step(psi, a, dt, alpha, vloc=vloc, cell=cell, want_norm=False)
    jE = np.array([float(np.dot(j, e)) for j, e in zip(js, es)])
    w = dt * (0.5 * jE[0] + jE[1:-1].sum() + 0.5 * jE[-1])
    e0 = plan.energy_functional(psi0, pulse_a_over_c(0.0, A0, omega_l, Td, direction), alpha, vloc=vloc, cell=cell)
    eN = plan.energy_functional(psi, pulse_a_over_c(Td, A0, omega_l, Td, direction), alpha, vloc=vloc, cell=cell)
    return eN - e0, vol * w, np.array(js)


def excited_density_after_pulse(plan, psi0, A0, dt, nsteps, alpha=0.25, omega_l=0.0569614, vloc=None,
                                direction=(0.0, 0.0, 1.0), tol=1e-8, maxit=400, cell=0):
    """Propagate psi0 through nsteps Taylor steps under the pulse (T_d = nsteps dt), then
    take the eigenstates of h(t_f) (Sec. IV B, Eq. (25); V_x built from psi(t_f), A(t_f))
    starting from psi(t_f), and n_ex of Eq. (26).

    Returns (n_ex, eigenvalues [nk][nb], iterations, converged, psi(t_f), phi)."""
    psi = psi0.clone()
    Td = nsteps * dt
    for n in range(nsteps):
        plan.taylor_step(psi, pulse_a_over_c(n * dt, A0, omega_l, Td, direction), dt, alpha, vloc=vloc, cell=cell,
                         want_norm=False)
    a_f = pulse_a_over_c(Td, A0, omega_l, Td, direction)
    phi, eps, _, it, conv = plan.eigensolve(psi, phi=psi.clone(), vloc=vloc, a_over_c=a_f, alpha=alpha, tol=tol,
                                            maxit=maxit, cell=cell)
    return plan.excited_density(phi, psi, cell=cell), eps, it, conv, psi, phi
