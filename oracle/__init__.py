"""FP64 CPU oracle for the screened Fock-like exchange operator.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, calls or links
this package: it is used by `tests/`, by the smoke check in `__graft_entry__`
and by the CPU-baseline leg of `bench.py`. It shares no code with the HIP
library (no kernels, headers, tables or helpers); only the seeded input
generator is common to both sides.

Everything here is written from the paper (Sato, Taniguchi, Shinohara, Yabana,
"Nonlinear electronic excitations in crystalline solids using meta-GGA and
hybrid functional in TDDFT"):

* Eq. (14): the Fock-like term in real space, a convolution of the pair
  density psi_j^* psi_i with the short-range Coulomb interaction, multiplied by
  psi_j and summed over occupied j;
* Eq. (15): the same term evaluated in Fourier space with the pair density's
  transform and the transformed interaction;
* Eq. (16): the k-point / band decomposition of the occupied sum;
* Eq. (8): the HSE composition (the Fock-like term enters with weight 1/4);
* Eqs. (9)-(10): the fourth-order Taylor propagator with h(t+dt/2) ~ h(t);
* Eq. (21): the sin^2 vector-potential pulse; Eq. (22): the energy functional.

Readings taken where the paper is silent or garbled (they bind the HIP path
too): the short-range kernel is erfc(w r)/r (the text's "erf" would be the
long-range part), exchange carries a minus sign, the q+G=0 term is the finite
limit pi/w^2, the continuum integral becomes (1/Omega) sum_G, the k' sum has
weight 1/N_k and the kernel is evaluated at |k-k'+G|, Nyquist entries of the
kernel are averaged over +-n/2, and q = k-k' is never folded.

Every function works in float64/complex128 with naive DFTs (DFT matrices
applied axis by axis); no FFT library is used for the method itself.
"""

from .lattice import reciprocal, volume, fftfreq_int, gvectors, grid_points  # noqa: F401
from .dft import dft_matrix, dft3, dft3_full  # noqa: F401
from .kernel import screened_coulomb_ft, kernel_table  # noqa: F401
from .fock import (fock_apply, pair_potential, exchange_energy, exchange_energy_parseval,  # noqa: F401
                   fock_apply_realspace, general_apply)
from .adjoint import fock_vjp, energy_grad  # noqa: F401
from .ortho import gram_schmidt  # noqa: F401
from . import taylor  # noqa: F401
from . import excited  # noqa: F401
