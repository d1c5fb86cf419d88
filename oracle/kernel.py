"""The screened interaction in Fourier space (v-tilde of Eq. (15), HSE of Eq. (8)).

Short-range Coulomb interaction erfc(w r)/r (the paper calls it short-ranged;
its printed "erf" is read as erfc, since erf(w r)/r is the long-range part).
Its Fourier transform is

    v(p) = 4 pi / |p|^2 * (1 - exp(-|p|^2 / (4 w^2))),     v(0) = pi / w^2,

the p -> 0 value being the finite limit of the same expression (the q + G = 0
term, which the paper leaves implicit). It is used for the l = 0 slot of q = 0
and wherever q + G is exactly zero (k and k' differing by a reciprocal-lattice
vector of the grid). The factor 1 - exp(-x) is evaluated as -expm1(-x) so that
small x keeps its digits.

For the pair density of orbitals at k (output) and k' (occupied) the kernel is
evaluated at q + G with q = k - k' (crystal momentum of the pair density),
never folded back into the first zone.

Nyquist slots: for an even grid length the slot j = n/2 holds l = -n/2, and
+n/2 is the same slot. The table entry there is the average of v over the two
choices (over all 2^|N| choices when several axes sit at Nyquist). This keeps
K_{-q}[-l] = K_q[l], the symmetry that makes the operator the exact gradient
of the exchange energy on the grid.
"""

import itertools

import numpy as np

from .lattice import fftfreq_int


def screened_coulomb_ft(p2, omega):
    """v(p) for |p|^2 = p2 > 0 (array)."""
    p2 = np.asarray(p2, dtype=np.float64)
    return 4.0 * np.pi / p2 * (-np.expm1(-p2 / (4.0 * omega * omega)))


def kernel_table(q, q_is_zero, n, B, omega):
    """K_q[l1, l2, l3] on the FFT grid (no 1/N_r folded in).

    q         : (3,) Cartesian crystal momentum of the pair density, q = k - k'
    q_is_zero : True when k and k' are the same k-point (integer test, not a
                float compare); then the l = 0 slot takes v(0) = pi / w^2
    n         : (n1, n2, n3)
    B         : reciprocal rows b_d
    """
    q = np.asarray(q, dtype=np.float64)
    per_axis = []
    for d in range(3):
        nd = int(n[d])
        base = fftfreq_int(nd)
        choices = [base]
        if nd % 2 == 0:
            alt = base.copy()
            alt[nd // 2] = nd // 2            # the +n/2 reading of the Nyquist slot
            choices.append(alt)
        per_axis.append(choices)
    K = np.zeros(tuple(int(x) for x in n), dtype=np.float64)
    combos = list(itertools.product(*per_axis))
    for l1, l2, l3 in combos:
        L1, L2, L3 = np.meshgrid(l1, l2, l3, indexing="ij")
        p = q + L1[..., None] * B[0] + L2[..., None] * B[1] + L3[..., None] * B[2]
        p2 = np.sum(p * p, axis=-1)
        with np.errstate(divide="ignore", invalid="ignore"):
            v = screened_coulomb_ft(p2, omega)
        if q_is_zero:
            zero = (L1 == 0) & (L2 == 0) & (L3 == 0)
            v = np.where(zero, np.pi / (omega * omega), v)
        v = np.where(p2 == 0.0, np.pi / (omega * omega), v)
        K += v
    # slots off Nyquist get the same value from every combination
    return K / len(combos)
