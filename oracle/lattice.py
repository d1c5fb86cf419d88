"""Cell geometry for the oracle (real-space grid of Sec. II C, Fourier set of Eq. (15)).

Conventions: rows of `a` are the lattice vectors, Omega = |det a|, reciprocal
rows b_d satisfy a_i . b_j = 2 pi delta_ij. Grid points r_m = sum_d (m_d/n_d) a_d.
The reciprocal vector of FFT index j along an axis of length n is l b with
l = j for j < n/2 and l = j - n otherwise (numpy fftfreq order).
"""

import numpy as np


def reciprocal(a):
    a = np.asarray(a, dtype=np.float64)
    return 2.0 * np.pi * np.linalg.inv(a).T


def volume(a):
    return float(abs(np.linalg.det(np.asarray(a, dtype=np.float64))))


def fftfreq_int(n):
    """Integer G index of each FFT slot: 0..ceil(n/2)-1 then -floor(n/2)..-1."""
    n = int(n)
    return np.array([j if j < (n + 1) // 2 else j - n for j in range(n)], dtype=np.int64)


def gvectors(n, B):
    """G_l for every FFT slot, shape (n1, n2, n3, 3)."""
    n1, n2, n3 = n
    L1, L2, L3 = np.meshgrid(fftfreq_int(n1), fftfreq_int(n2), fftfreq_int(n3), indexing="ij")
    return L1[..., None] * B[0] + L2[..., None] * B[1] + L3[..., None] * B[2]


def grid_points(n, a):
    """r_m for every grid point, shape (n1, n2, n3, 3)."""
    n1, n2, n3 = n
    M1, M2, M3 = np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2, np.arange(n3) / n3, indexing="ij")
    a = np.asarray(a, dtype=np.float64)
    return M1[..., None] * a[0] + M2[..., None] * a[1] + M3[..., None] * a[2]
