"""Naive discrete Fourier transforms (the FFT of Eq. (15), written as its definition).

Forward:  f_hat[l] = sum_m f[m] exp(-2 pi i sum_d l_d m_d / n_d)
Inverse (unnormalised): f[m] = sum_l f_hat[l] exp(+2 pi i sum_d l_d m_d / n_d)

The separable form applies the one-dimensional DFT matrix along each axis (a
matrix product per axis); the full form builds the N_r x N_r matrix and is only
used on tiny grids to pin the separable one.
"""

import numpy as np

from .lattice import fftfreq_int


def dft_matrix(n, sign):
    """F[j, m] = exp(sign * 2 pi i * l_j * m / n), l_j the G index of slot j.

    The phase index l*m is reduced mod n before the exponential so that equal
    phases give bit-identical entries.
    """
    n = int(n)
    l = fftfreq_int(n)
    m = np.arange(n)
    ph = np.mod(np.outer(l, m), n).astype(np.float64)
    return np.exp(sign * 2j * np.pi * ph / n)


def _apply_axis(x, F, axis):
    x = np.moveaxis(x, axis, -1)
    y = x @ F.T                       # y[..., j] = sum_m F[j, m] x[..., m]
    return np.moveaxis(y, -1, axis)


def dft3(x, sign=-1):
    """Separable 3D DFT over the last three axes (unnormalised, either sign)."""
    x = np.asarray(x, dtype=np.complex128)
    n1, n2, n3 = x.shape[-3:]
    y = _apply_axis(x, dft_matrix(n3, sign), -1)
    y = _apply_axis(y, dft_matrix(n2, sign), -2)
    y = _apply_axis(y, dft_matrix(n1, sign), -3)
    return y


def dft3_full(x, sign=-1):
    """Full O(N_r^2) 3D DFT over the last three axes (tiny grids only)."""
    x = np.asarray(x, dtype=np.complex128)
    n1, n2, n3 = x.shape[-3:]
    L = np.stack(np.meshgrid(fftfreq_int(n1), fftfreq_int(n2), fftfreq_int(n3), indexing="ij"), -1).reshape(-1, 3)
    M = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1).reshape(-1, 3)
    ph = (np.outer(L[:, 0], M[:, 0]) / n1 + np.outer(L[:, 1], M[:, 1]) / n2 + np.outer(L[:, 2], M[:, 2]) / n3)
    F = np.exp(sign * 2j * np.pi * ph)
    flat = x.reshape(x.shape[:-3] + (-1,))
    return (flat @ F.T).reshape(x.shape)
