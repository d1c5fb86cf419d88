"""Excited electrons after the pulse (Sec. IV B, Eqs. (25)-(26)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (25): the eigenstates of the Kohn-Sham Hamiltonian at the end of the
pulse. With the pieces of this package,

    h_k(t_f) = T_k[a(t_f)] + v_loc + alpha V_x[psi(t_f)],

the same operator the propagator applies at t_f (the Fock-like term built from
the time-dependent orbitals and frozen). phi_ik are its nb lowest eigenstates
at each k, normalised as (Omega/N_r) sum |phi|^2 = 1.

Eq. (26): the number density of excited electrons. The paper's sum over
occupied i, j runs over k-points too; written out with the k average and the
spin factor that make g_s N_b / Omega the valence density,

    n_ex = (g_s / (N_k Omega)) sum_k [ N_b - sum_{i,j} |<phi_ik | psi_jk>|^2 ],
    <a | b> = (Omega / N_r) sum_r conj(a) b.

Two routes to the eigenstates:
* eigenstates_dense: explicit N_r x N_r matrices (taylor.kinetic_matrix,
  taylor.exchange_matrix) diagonalised by numpy.linalg.eigh; tiny grids, and the
  16^3 reference values stored under tests/golden;
* residuals_matfree: ||h phi - eps phi|| per state with the matrix-free h
  (taylor.h_apply), usable at any supported grid size.
"""

import numpy as np

from .lattice import volume
from .taylor import exchange_matrix, h_apply, kinetic_matrix


def hamiltonian_matrix(psi, kpts, a, omega, k, avec, alpha, vloc=None):
    """Dense h_k = T_k[avec] + diag(v_loc) + alpha V_x[psi] (N_r x N_r)."""
    psi = np.asarray(psi, dtype=np.complex128)
    n = psi.shape[-3:]
    H = kinetic_matrix(n, a, np.asarray(kpts)[k], avec)
    if vloc is not None:
        H = H + np.diag(np.asarray(vloc, dtype=np.float64).reshape(-1))
    if alpha != 0.0:
        H = H + alpha * exchange_matrix(psi, kpts, a, omega, k)
    return H


def eigenstates_dense(psi, kpts, a, omega, avec, alpha, nb, vloc=None, extra=0):
    """(eps[nk][nb + extra], phi[nk][nb + extra][grid]): the lowest eigenpairs of h_k
    at every k, ascending, phi normalised to (Omega/N_r) sum |phi|^2 = 1."""
    psi = np.asarray(psi, dtype=np.complex128)
    nk = psi.shape[0]
    n = psi.shape[-3:]
    nr = int(np.prod(n))
    m = nb + extra
    eps = np.empty((nk, m))
    phi = np.empty((nk, m) + tuple(n), dtype=np.complex128)
    scale = np.sqrt(nr / volume(a))
    for k in range(nk):
        w, V = np.linalg.eigh(hamiltonian_matrix(psi, kpts, a, omega, k, avec, alpha, vloc))
        eps[k] = w[:m]
        phi[k] = (V[:, :m].T * scale).reshape((m,) + tuple(n))
    return eps, phi


def overlaps(phi, psi, a):
    """S[k][i][j] = <phi_ik | psi_jk> with the cell inner product."""
    phi = np.asarray(phi, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    nk = phi.shape[0]
    nr = int(np.prod(phi.shape[-3:]))
    w = volume(a) / nr
    return np.stack([w * np.conj(phi[k].reshape(phi.shape[1], -1)) @ psi[k].reshape(psi.shape[1], -1).T
                     for k in range(nk)])


def excited_density(phi, psi, a, gs=2.0):
    """n_ex of Eq. (26) (number per bohr^3) for eigenstates phi and orbitals psi,
    both [nk][nb][grid] with the same nb."""
    S = overlaps(phi, psi, a)
    nk, nb = S.shape[0], S.shape[1]
    kept = np.sum(np.abs(S) ** 2)
    return gs / (nk * volume(a)) * (nk * nb - kept)


def residuals_matfree(psi, phi, eps, kpts, a, omega, avec, alpha, vloc=None, src=None):
    """r[k][i] = sqrt(Omega/N_r) ||h phi_ik - eps_ik phi_ik|| with the matrix-free h
    (V_x over the source sub-mesh src when given)."""
    phi = np.asarray(phi, dtype=np.complex128)
    hphi = h_apply(psi, phi, kpts, a, omega, avec, alpha, vloc, src=src)
    nr = int(np.prod(phi.shape[-3:]))
    d = hphi - np.asarray(eps)[:, :, None, None, None] * phi
    return np.sqrt(volume(a) / nr * np.sum(np.abs(d) ** 2, axis=(2, 3, 4)))
