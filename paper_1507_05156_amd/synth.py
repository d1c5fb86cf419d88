"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module draws the inputs only: lattice, k-mesh, orbitals and a model local
potential. It contains none of the exchange operator's arithmetic, so both the
HIP path and the CPU oracle may take their inputs from it.

Workload recipe (stand-in for the paper's silicon ground-state orbitals, which
need pseudopotential data that is not available):

* cubic cell, a = 10.26 bohr (the 8-atom silicon cell of Sec. II C);
* a Gamma-centred N x N x N k-mesh, fractional coordinates m/N mapped into
  (-1/2, 1/2], row-major order over (m1, m2, m3);
* per k-point, N_b orbitals with random plane-wave coefficients
  c_G = (x0 + i x1)/sqrt(2), x ~ N(0, 1), drawn over the full FFT grid in
  fftfreq storage order, multiplied by exp(-|k+G|^2/8) and cut to
  |k+G|^2/2 <= 8 Ha, then made orthonormal in band order (a QR factorisation
  whose R has a positive diagonal, i.e. the Gram-Schmidt result);
* u(r_m) = Omega^{-1/2} sum_G c_G exp(i G.r_m) on the real-space grid, so that
  (Omega/N_r) sum_m |u(r_m)|^2 = 1.

Seeds: 150705156 + 1000 * config + cell_index, numpy PCG64 (default_rng).
"""

from __future__ import annotations

import numpy as np

SEED_BASE = 150705156
LATTICE_A = 10.26          # bohr
OMEGA_HSE = 0.106          # bohr^-1 (range-separation parameter used by the workloads)
ECUT_HA = 8.0              # plane-wave cut of the generated orbitals (Ha)
ENVELOPE_DIV = 8.0         # envelope exp(-|k+G|^2 / ENVELOPE_DIV)


def seed_for(config: int, cell_index: int = 0) -> int:
    return SEED_BASE + 1000 * int(config) + int(cell_index)


def cubic_cell(a: float = LATTICE_A) -> np.ndarray:
    """Rows are the lattice vectors a_1, a_2, a_3 (bohr)."""
    return np.eye(3) * float(a)


def reciprocal_rows(a: np.ndarray) -> np.ndarray:
    """Rows b_d with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(a, dtype=np.float64)).T


def gamma_mesh(nk1: int, a: np.ndarray, nk2: int | None = None, nk3: int | None = None) -> np.ndarray:
    """Gamma-centred k-mesh, Cartesian bohr^-1, shape [nk][3], row-major order.

    Fractional coordinates f = m/N are mapped into (-1/2, 1/2].
    """
    nk2 = nk1 if nk2 is None else nk2
    nk3 = nk1 if nk3 is None else nk3
    B = reciprocal_rows(a)
    out = []
    for m1 in range(nk1):
        for m2 in range(nk2):
            for m3 in range(nk3):
                f = []
                for m, N in ((m1, nk1), (m2, nk2), (m3, nk3)):
                    x = m / N
                    if x > 0.5:
                        x -= 1.0
                    f.append(x)
                out.append(np.asarray(f) @ B)
    return np.asarray(out, dtype=np.float64)


def _fftfreq_int(n: int) -> np.ndarray:
    return np.rint(np.fft.fftfreq(n) * n).astype(np.int64)


def submesh(nk1: int, stride: int, nk2: int | None = None, nk3: int | None = None) -> list[int]:
    """Indices, in gamma_mesh order, of the Gamma-centred sub-mesh keeping every
    `stride`-th point along each axis (e.g. 4^3 of 12^3 with stride 3)."""
    nk2 = nk1 if nk2 is None else nk2
    nk3 = nk1 if nk3 is None else nk3
    return [(m1 * nk2 + m2) * nk3 + m3 for m1 in range(0, nk1, stride) for m2 in range(0, nk2, stride)
            for m3 in range(0, nk3, stride)]


def orbitals(n, a, kpts, nb, seed, *, orthonormal=True, ecut=ECUT_HA, envelope=ENVELOPE_DIV,
             dtype=np.complex128) -> np.ndarray:
    """Seeded orbitals u[k][b][n1][n2][n3] (periodic parts on the real-space grid)."""
    n1, n2, n3 = (int(n), int(n), int(n)) if np.isscalar(n) else tuple(int(x) for x in n)
    a = np.asarray(a, dtype=np.float64)
    kpts = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
    B = reciprocal_rows(a)
    vol = abs(np.linalg.det(a))
    l1, l2, l3 = np.meshgrid(_fftfreq_int(n1), _fftfreq_int(n2), _fftfreq_int(n3), indexing="ij")
    G = (l1[..., None] * B[0] + l2[..., None] * B[1] + l3[..., None] * B[2])
    rng = np.random.default_rng(seed)
    nr = n1 * n2 * n3
    out = np.empty((len(kpts), nb, n1, n2, n3), dtype=np.complex128)
    for ik, k in enumerate(kpts):
        x = rng.standard_normal((nb, n1, n2, n3, 2))
        c = (x[..., 0] + 1j * x[..., 1]) / np.sqrt(2.0)
        kg2 = np.sum((G + k) ** 2, axis=-1)
        c = c * np.exp(-kg2 / envelope) * (0.5 * kg2 <= ecut)
        if orthonormal:
            C = c.reshape(nb, nr).T            # columns = bands
            Q, R = np.linalg.qr(C)
            d = np.diag(R)
            Q = Q * (np.conj(d) / np.abs(d))   # positive diagonal of R
            c = Q.T.reshape(nb, n1, n2, n3)
        # u(r_m) = Omega^{-1/2} sum_G c_G exp(i G.r_m)  (numpy ifftn carries 1/N_r)
        out[ik] = np.fft.ifftn(c, axes=(1, 2, 3)) * (nr / np.sqrt(vol))
    return out.astype(dtype, copy=False)


def workload(config: int, cell_index: int = 0, *, n=None, nk=None, nb=None, a=LATTICE_A,
             orthonormal=True):
    """Inputs of one seeded workload: (a, kpts, u).

    The shapes default to the named workloads:
      0: 16^3 grid, 2x2x2 k, 4 bands;   1: 24^3, 4x4x4 k, 16 bands;
      2: 32^3, 6x6x6 k, 16 bands;       3: 24^3, 4x4x4 k, 16 bands;
      4: three cells (16^3, 3^3 k, 8 b), (20^3, 4^3 k, 12 b), (24^3, 5^3 k, 16 b).
    """
    table = {0: [(16, 2, 4)], 1: [(24, 4, 16)], 2: [(32, 6, 16)], 3: [(24, 4, 16)],
             4: [(16, 3, 8), (20, 4, 12), (24, 5, 16)]}
    dn, dk, db = table.get(config, [(16, 2, 4)])[cell_index]
    n = dn if n is None else n
    nk = dk if nk is None else nk
    nb = db if nb is None else nb
    cell = cubic_cell(a)
    kpts = gamma_mesh(nk, cell)
    u = orbitals(n, cell, kpts, nb, seed_for(config, cell_index), orthonormal=orthonormal)
    return cell, kpts, u


WORKLOADS = {
    0: dict(n=16, nk=2, nb=4),
    1: dict(n=24, nk=4, nb=16),
    2: dict(n=32, nk=6, nb=16),
    3: dict(n=24, nk=4, nb=16),
    4: [dict(n=16, nk=3, nb=8), dict(n=20, nk=4, nb=12), dict(n=24, nk=5, nb=16)],
}


# Empirical local pseudopotential of bulk silicon (Cohen and Bergstresser,
# Phys. Rev. 141, 789 (1966)): symmetric form factors in Rydberg at
# |G|^2 = 3, 8, 11 in units of (2 pi / a)^2, diamond structure with the two
# atoms of each primitive cell at +-tau, tau = (a/8)(1, 1, 1).
SI_FORM_FACTORS_RY = {3: -0.21, 8: 0.04, 11: 0.08}


def model_vloc(n) -> np.ndarray:
    """A crystal-like local potential v[n1][n2][n3] (Ha) on the grid of the cubic
    8-atom silicon cell (any side a): v(r) = sum_G V(|G|^2) cos(G.tau) cos(G.r)
    over the G = (2 pi / a)(h, k, l) with |G|^2 in the form-factor table. With it the
    lowest 16 bands of T + v_loc are separated from the 17th by a gap of about
    1 eV, as for the valence bands of silicon, so that the occupied subspace
    of the Hamiltonian is well defined (the random orbitals alone give nearly
    free-electron shells)."""
    n1, n2, n3 = (int(n), int(n), int(n)) if np.isscalar(n) else tuple(int(x) for x in n)
    m1, m2, m3 = np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2, np.arange(n3) / n3, indexing="ij")
    v = np.zeros((n1, n2, n3))
    rng3 = range(-3, 4)
    for h in rng3:
        for k in rng3:
            for l in rng3:
                g2 = h * h + k * k + l * l
                if g2 not in SI_FORM_FACTORS_RY or not (h % 2 == k % 2 == l % 2):
                    continue
                structure = np.cos(np.pi / 4.0 * (h + k + l))          # G . tau
                phase = 2.0 * np.pi * (h * m1 + k * m2 + l * m3)       # G . r on the grid
                v += 0.5 * SI_FORM_FACTORS_RY[g2] * structure * np.cos(phase)
    return v


def random_fields(shape, seed, dtype=np.complex128) -> np.ndarray:
    """Plain complex Gaussian fields (directions, cotangents, test vectors)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(tuple(shape) + (2,))
    return ((x[..., 0] + 1j * x[..., 1]) / np.sqrt(2.0)).astype(dtype)
