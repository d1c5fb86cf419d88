// Launchers of the propagator / orthonormalisation kernels (prop.hip).
#pragma once

#include "kernels.hpp"

namespace fockmi {

// F[k][f][l] *= scale * |k + G_l + a|^2 / 2 for nk x nf Fourier-space fields
hipError_t launch_kinetic_mul(c128* F, const double* kpts, int nk, int nf, const Geom& g, const double a[3],
                              double scale, hipStream_t st);
// F *= scale / (1 + |k + G + a|^2 / (2 e0)) in Fourier space (eigensolver preconditioner)
hipError_t launch_precond_mul(c128* F, const double* kpts, int nk, int nf, const Geom& g, const double a[3],
                              double e0, double scale, hipStream_t st);
// out = (base ? base : 0) + (cre + i cim) * (kin + vloc .* x + alpha * vx); vloc / vx may be NULL
hipError_t launch_hcombine(c128* out, const c128* base, const c128* kin, const c128* x, const c128* vx,
                           const double* vloc, double alpha, double cre, double cim, long count, int nr,
                           hipStream_t st);
// out[f] = sum_r |psi[f][r]|^2
hipError_t launch_norms(double* out, const c128* psi, int nfields, int nr, hipStream_t st);
// out6 = sum conj(L) * (k+G+a)_d * F, d = 0..2 as (re, im) pairs, over nk*nf Fourier-space fields
hipError_t launch_agrad(double* out6, double* partial, int nblk, const c128* L, const c128* F, const double* kpts,
                        int nf, const Geom& g, const double a[3], long count, hipStream_t st);
// modified Gram-Schmidt per k-point with inner product w * sum conj(a) b
hipError_t launch_mgs(c128* psi, int nk, int nb, int nr, double w, hipStream_t st);

}  // namespace fockmi
