"""Orthonormalisation of the occupied orbitals of each k-point (FP64).

Modified Gram-Schmidt in band order with the cell inner product
<a|b> = (Omega/N_r) sum_m conj(a_m) b_m, so that every output orbital has
(Omega/N_r) sum |u|^2 = 1 (the normalisation the operator of Eq. (15) assumes
for its occupied orbitals).
"""

import numpy as np

from .lattice import volume


def gram_schmidt(u, a):
    u = np.array(u, dtype=np.complex128, copy=True)
    nr = int(np.prod(u.shape[-3:]))
    w = volume(a) / nr
    for k in range(u.shape[0]):
        for b in range(u.shape[1]):
            v = u[k, b]
            for c in range(b):
                v = v - w * np.sum(np.conj(u[k, c]) * v) * u[k, c]
            u[k, b] = v / np.sqrt(w * np.sum(np.abs(v) ** 2))
    return u
