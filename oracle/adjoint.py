"""Reverse-mode derivatives of the exchange operator and energy (derived from Eq. (15)).

Gradient convention: for a real loss L of a complex array z the gradient is
dL/dRe z + i dL/dIm z (PyTorch's convention), so a first-order change is
dL = Re sum conj(grad) dz.

For y = V_x[u] phi with cotangent g (the gradient of L with respect to y):

* V_x is Hermitian and block diagonal in k, so  g_phi = V_x[u] g.
* u enters twice in each pair (conjugated in the pair density, plain as the
  multiplier). Differentiating both occurrences gives, with K_{k'-k}:

  g_u[k'][j] = -(1/N_k) sum_{k,i} ( g_{ik}   * W(conj(phi_{ik}) u_{jk'})
                                   + phi_{ik} * W(conj(g_{ik})  u_{jk'}) )

  where W(rho) = (1/N_r) IDFT(K_{k'-k} DFT(rho)). Both families are the
  general operator with the target set to u and the roles of the other two
  arrays swapped. With down-sampling, k' runs over the source sub-mesh only
  and 1/N_k becomes 1/|S|.

For E_x = (g_s/2)(1/N_k)(Omega/N_r) sum conj(u) V_x[u] u (real for exact
arithmetic): grad_u E_x = 2 (g_s/N_k)(Omega/N_r) V_x[u] u.
"""

import numpy as np

from .fock import general_apply, fock_apply
from .lattice import volume


def fock_vjp(u, phi, g, kpts, a, omega, src=None):
    """(g_u, g_phi) for y = V_x[u] phi and cotangent g of y.

    With a down-sampled source set src (weight 1/|src|), u enters only through
    the source k-points: g_u is zero elsewhere, and on a source k' it sums over
    every target k with the same weight.
    """
    u = np.asarray(u, dtype=np.complex128)
    nk = u.shape[0]
    src = list(range(nk)) if src is None else [int(x) for x in src]
    w = -1.0 / len(src)
    g_phi = general_apply(g, u, u, kpts, a, omega, src=src)
    g_u = np.zeros_like(u)
    us = u[src]
    g_u[src] = (general_apply(us, phi, g, kpts, a, omega, tgt=src, weight=w)
                + general_apply(us, g, phi, kpts, a, omega, tgt=src, weight=w))
    return g_u, g_phi


def energy_grad(u, kpts, a, omega, gs=2.0):
    """grad_u of E_x in PyTorch's convention."""
    u = np.asarray(u, dtype=np.complex128)
    nk = u.shape[0]
    nr = int(np.prod(u.shape[-3:]))
    return 2.0 * gs / nk * volume(a) / nr * fock_apply(u, u, kpts, a, omega)
