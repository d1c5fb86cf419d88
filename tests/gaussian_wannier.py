"""Closed-form exchange energy of Gaussian Wannier functions (a pin for the oracle).

One doubly occupied band built from a normalised Gaussian w(r) = (alpha/pi)^{3/4}
exp(-alpha r^2 / 2) centred in the cell, Bloch-summed over a Gamma-centred
k-mesh. When Gaussians on different lattice sites do not overlap, the density
matrix is periodic over the Born-von Karman supercell and the exchange energy
per cell with the erfc(w r)/r interaction is

    E_x = -(g_s/2) sum_{L in BvK lattice} I(L)

where I(L) is the interaction of two unit Gaussian charges (exponent alpha)
at distance L through erfc(w r)/r = 1/r - erf(w r)/r:

    I(L) = [erf(g1 L) - erf(g2 L)] / L,   I(0) = 2 (g1 - g2) / sqrt(pi),
    g1 = sqrt(alpha/2),  g2 = sqrt(alpha c / (alpha + c)),  c = alpha w^2 / (alpha + w^2).

The BvK lattice is (N a) Z^3 for an N x N x N mesh (a Z^3 at Gamma only).
This is textbook Gaussian electrostatics, independent of any Fourier-space code.
"""

import numpy as np
from scipy.special import erf


def closed_form_ex(alpha, omega, a, nkm, gs=2.0, shells=8):
    c = alpha * omega ** 2 / (alpha + omega ** 2)
    g1 = np.sqrt(alpha / 2.0)
    g2 = np.sqrt(alpha * c / (alpha + c))
    L0 = nkm * a
    total = 2.0 * (g1 - g2) / np.sqrt(np.pi)
    rng = range(-shells, shells + 1)
    for i in rng:
        for j in rng:
            for k in rng:
                if i == 0 and j == 0 and k == 0:
                    continue
                L = L0 * np.sqrt(i * i + j * j + k * k)
                total += (erf(g1 * L) - erf(g2 * L)) / L
    return -(gs / 2.0) * total


def bloch_orbitals(n, a, kpts, alpha):
    """u_k(r_m) = sum_R exp(-i k.(r_m - R)) w(r_m - R) on the grid, shape [nk][1][n][n][n]."""
    m = np.arange(n) / n
    M1, M2, M3 = np.meshgrid(m, m, m, indexing="ij")
    r = np.stack([M1, M2, M3], -1) * a                     # cubic cell
    centre = np.array([a / 2, a / 2, a / 2])
    out = np.zeros((len(kpts), 1, n, n, n), dtype=np.complex128)
    pref = (alpha / np.pi) ** 0.75
    for ik, k in enumerate(kpts):
        acc = np.zeros((n, n, n), dtype=np.complex128)
        for R1 in (-1, 0, 1):
            for R2 in (-1, 0, 1):
                for R3 in (-1, 0, 1):
                    R = np.array([R1, R2, R3]) * a
                    d = r - centre - R
                    w = pref * np.exp(-0.5 * alpha * np.sum(d * d, -1))
                    acc += np.exp(-1j * (d @ k)) * w
        out[ik, 0] = acc
    return out
