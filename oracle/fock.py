"""The Fock-like exchange operator, energy and real-space brute force (Eqs. (14)-(16)).

Orbitals are the periodic parts u_{jk}(r_m) on the grid, normalised so that
(Omega/N_r) sum_m |u|^2 = 1. With psi = exp(i k.r) u, the Fourier-space form
of Eq. (15) with the band/k decomposition of Eq. (16) becomes, per output
orbital phi_{ik}:

    rho   = conj(u_{jk'}) * phi_{ik}                      (pair density; its
                                                           momentum k-k' enters
                                                           only through K)
    W     = (1/N_r) IDFT( K_{k-k'} * DFT(rho) )          ((2 pi)^-3 int dG ->
                                                           (1/Omega) sum_G; Omega
                                                           cancels)
    (V_x phi)_{ik} = -(1/N_k) sum_{k', j} u_{jk'} * W     (exchange is negative;
                                                           1/N_k = BZ average)

Exchange energy (the E_xc piece of Eq. (22), closed shell, spin degeneracy g_s):

    E_x = (g_s/2) (1/N_k) (Omega/N_r) sum_{ik, m} conj(u_{ik}) (V_x u)_{ik}

Down-sampling (Sec. II C, after Eq. (16)): the sum over the occupied orbitals
runs over the k-points of a sub-mesh S of the orbital mesh only (the paper
samples 4^3 of 12^3), with the Brillouin-zone weight 1/|S| in place of 1/N_k.
`src` lists the indices of S in the k-point array; by default S is the whole
mesh and the operator is the one above.
"""

import numpy as np

from .dft import dft3, dft3_full
from .kernel import kernel_table
from .lattice import reciprocal, volume, grid_points, gvectors


def pair_potential(p_src, x_tgt, K, full_dft=False):
    """W = (1/N_r) IDFT(K * DFT(conj(p_src) * x_tgt)); leading axes broadcast."""
    f = dft3_full if full_dft else dft3
    rho = np.conj(p_src) * x_tgt
    nr = rho.shape[-1] * rho.shape[-2] * rho.shape[-3]
    return f(K * f(rho, -1), +1) / nr


def general_apply(X, P, M, kpts, a, omega, rows=None, full_dft=False, src=None, tgt=None, weight=None):
    """out[t][s] = weight * sum_{ks in src, b} M[ks][b] * W(P[ks][b], X[t][s]; K_{k(t) - k_s}).

    X : [N_t][N_x][n1][n2][n3]   fields the operator acts on (targets)
    P : [N_k][N_b][...]          fields conjugated inside the pair density
    M : [N_k][N_b][...]          fields multiplying the pair potential
    The forward operator is general_apply(phi, u, u); the adjoint uses other
    combinations of the same three roles.
    rows   : optional list of (t, s) to evaluate; the others are left zero.
    src    : k indices of P and M summed over (default: all N_k).
    tgt    : k index of each target X[t] (default: t, so N_t = N_k).
    weight : factor of the sum (default -1/len(src)).
    """
    X = np.asarray(X, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128)
    M = np.asarray(M, dtype=np.complex128)
    kpts = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
    src = list(range(P.shape[0])) if src is None else [int(x) for x in src]
    tgt = list(range(X.shape[0])) if tgt is None else [int(x) for x in tgt]
    weight = -1.0 / len(src) if weight is None else weight
    n = X.shape[-3:]
    B = reciprocal(a)
    out = np.zeros_like(X)
    if rows is None:
        rows = [(t, s) for t in range(X.shape[0]) for s in range(X.shape[1])]
    by_t = {}
    for t, s in rows:
        by_t.setdefault(t, []).append(s)
    for t, slist in by_t.items():
        kt = tgt[t]
        acc = np.zeros((len(slist),) + tuple(n), dtype=np.complex128)
        for ks in src:
            K = kernel_table(kpts[kt] - kpts[ks], kt == ks, n, B, omega)
            for idx, s in enumerate(slist):
                W = pair_potential(P[ks], X[t, s][None], K, full_dft)     # [N_b][n...]
                acc[idx] += np.sum(M[ks] * W, axis=0)
        for idx, s in enumerate(slist):
            out[t, s] = weight * acc[idx]
    return out


def fock_apply(u, phi, kpts, a, omega, rows=None, full_dft=False, src=None):
    """(V_x phi) for every (k, i), or for the listed rows only; sources on the sub-mesh src."""
    return general_apply(phi, u, u, kpts, a, omega, rows=rows, full_dft=full_dft, src=src)


def exchange_energy(u, kpts, a, omega, gs=2.0, V=None, src=None):
    """E_x = (g_s/2)(1/N_k)(Omega/N_r) sum conj(u) V_x u, returned as a complex number.

    The imaginary part is a check (zero for exact arithmetic).
    """
    u = np.asarray(u, dtype=np.complex128)
    if V is None:
        V = fock_apply(u, u, kpts, a, omega, src=src)
    nk = u.shape[0]
    nr = int(np.prod(u.shape[-3:]))
    return (gs / 2.0) / nk * volume(a) / nr * np.sum(np.conj(u) * V)


def exchange_energy_parseval(u, kpts, a, omega, gs=2.0, src=None):
    """E_x written through the pair-density spectra (an independent route):

    E_x = -(g_s/2) Omega / (N_k |S| N_r^2) sum_{k, k' in S, i j} sum_l K_{k-k'}[l] |DFT(conj(u_jk') u_ik)[l]|^2
    """
    u = np.asarray(u, dtype=np.complex128)
    kpts = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
    nk = u.shape[0]
    src = list(range(nk)) if src is None else [int(x) for x in src]
    n = u.shape[-3:]
    nr = int(np.prod(n))
    B = reciprocal(a)
    total = 0.0
    for k in range(nk):
        for kp in src:
            K = kernel_table(kpts[k] - kpts[kp], k == kp, n, B, omega)
            rho_hat = dft3(np.conj(u[kp])[:, None] * u[k][None, :], -1)
            total += np.sum(K * np.abs(rho_hat) ** 2)
    return -(gs / 2.0) * volume(a) / (nk * len(src) * nr * nr) * total


def realspace_kernel(q, q_is_zero, n, a, omega):
    """K_q(r_m) = (1/N_r) sum_l K_q[l] exp(i G_l . r_m), evaluated point by point (tiny grids)."""
    B = reciprocal(a)
    K = kernel_table(q, q_is_zero, n, B, omega)
    G = gvectors(n, B).reshape(-1, 3)
    r = grid_points(n, a).reshape(-1, 3)
    phase = np.exp(1j * (r @ G.T))            # [m, l]
    nr = len(r)
    return (phase @ K.reshape(-1)).reshape(tuple(n)) / nr


def fock_apply_realspace(u, phi, kpts, a, omega, src=None):
    """Eq. (14) on the grid: the O(N_r^2) double sum with the periodic kernel K_q(r - r').

    (V_x phi)_{ik}(r_m) = -(1/N_k) sum_{k'j} u_{jk'}(r_m) sum_{m'} K_{k-k'}(r_m - r_m') conj(u_{jk'}(r_m')) phi_{ik}(r_m')

    Independent of the Fourier route: it never transforms the pair density.
    """
    u = np.asarray(u, dtype=np.complex128)
    phi = np.asarray(phi, dtype=np.complex128)
    kpts = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
    nk, nb = u.shape[:2]
    n = u.shape[-3:]
    n1, n2, n3 = n
    nr = n1 * n2 * n3
    idx = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1).reshape(-1, 3)
    # difference index (m - m') mod n for every pair of points
    d = (idx[:, None, :] - idx[None, :, :]) % np.array(n)
    flat_d = (d[..., 0] * n2 + d[..., 1]) * n3 + d[..., 2]
    src = list(range(nk)) if src is None else [int(x) for x in src]
    out = np.zeros_like(phi)
    for k in range(phi.shape[0]):
        for kp in src:
            Kr = realspace_kernel(kpts[k] - kpts[kp], k == kp, n, a, omega).reshape(-1)
            C = Kr[flat_d]                               # C[m, m'] = K(r_m - r_m')
            for i in range(phi.shape[1]):
                for j in range(nb):
                    rho = (np.conj(u[kp, j]) * phi[k, i]).reshape(-1)
                    W = C @ rho
                    out[k, i] -= (u[kp, j].reshape(-1) * W).reshape(n) / len(src)
    return out
