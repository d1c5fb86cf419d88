// Eigenstates of the Hamiltonian after the pulse (Sec. IV B, Eq. (25)) and the
// number density of excited electrons (Eq. (26)).
//
// h_k = T_k[a] + v_loc + alpha V_x[u] is the propagator's Hamiltonian with the
// Fock-like term built from the given orbitals u and held fixed, so Eq. (25) is
// a linear Hermitian eigenproblem per k. Its nb lowest eigenpairs come from a
// block LOBPCG iteration in FP64 (Knyazev's locally optimal block
// preconditioned conjugate gradient), every step on the GPU:
//   X <- Ritz vectors of span(X);  repeat until every residual is below tol:
//     R = h X - X Lambda;  W = T R (kinetic preconditioner in Fourier space);
//     Rayleigh-Ritz on span[X, W, P] (P: the previous step's non-X part);
//     X, P <- the new Ritz vectors and their non-X part, h X and h P updated by
//     the same coefficients (h is applied once per iteration, to W).
// Bands whose residual is already below tol take no further part: their W and
// P columns are zeroed and drop out of the basis (soft locking). Without it the
// converged columns become nearly dependent and the rounding they bring into
// the coefficients, carried by the updated h X, makes the iteration diverge
// once it runs past the attainable residual. h X is also recomputed from X every
// kRefresh iterations. If the basis [X, W, P] is too close to dependent for the
// X block to be kept, the step is redone on [X, W].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "../../include/fockmi.h"
#include "eig.hpp"
#include "plan.hpp"
#include "prop.hpp"

using namespace fockmi;

namespace fockmi {

extern thread_local std::string g_last_error;

namespace {

constexpr double kPrecondE0 = 1.0;  // Ha: plane waves far above this are damped
constexpr int kRefresh = 20;        // iterations between recomputations of h X

ColSet cols(std::initializer_list<std::pair<const c128*, int>> parts) {
  ColSet z{};
  for (const auto& pc : parts) {
    z.p[z.nparts] = pc.first;
    z.cnt[z.nparts] = pc.second;
    ++z.nparts;
  }
  return z;
}

}  // namespace

fock_status Plan::eigensolve(Cell& c, const c128* u, c128* phi, const double* vloc, const double a[3], double alpha,
                             double tol, int maxit, double* eig_host, double* res_host, int* iters_host,
                             hipStream_t st) {
  const int nk = c.nk, nb = c.nb;
  const long nr = c.nr;
  const double w = c.vol / c.nr;
  fock_status s;
  hipError_t e;
  if ((s = field_bufs(c, {&eig.x, &eig.hx, &eig.w, &eig.hw, &eig.p, &eig.hp, &eig.xn, &eig.hxn, &eig.pn, &eig.hpn},
                      nb)) != FOCK_OK)
    return s;
  const int mmax = 3 * nb;
  if ((s = eig.S.ensure((size_t)nk * mmax * mmax * sizeof(c128), workspace_cap, "Rayleigh-Ritz matrices")) != FOCK_OK ||
      (s = eig.A.ensure((size_t)nk * mmax * mmax * sizeof(c128), workspace_cap, "Rayleigh-Ritz matrices")) != FOCK_OK ||
      (s = eig.C.ensure((size_t)nk * mmax * nb * sizeof(c128), workspace_cap, "Ritz coefficients")) != FOCK_OK ||
      (s = eig.lam.ensure((size_t)nk * nb * sizeof(double), 0, "Ritz values")) != FOCK_OK ||
      (s = eig.status.ensure((size_t)nk * sizeof(int), 0, "Ritz status")) != FOCK_OK ||
      (s = norms.ensure((size_t)nk * nb * sizeof(double), 0, "norms")) != FOCK_OK)
    return s;
  const c128* us = nullptr;
  if ((s = sources(c, u, nb, srcbuf, st, &us)) != FOCK_OK) return s;

  c128 *X = (c128*)eig.x.ptr, *HX = (c128*)eig.hx.ptr, *W = (c128*)eig.w.ptr, *HW = (c128*)eig.hw.ptr;
  c128 *P = (c128*)eig.p.ptr, *HP = (c128*)eig.hp.ptr, *Xn = (c128*)eig.xn.ptr, *HXn = (c128*)eig.hxn.ptr;
  c128 *Pn = (c128*)eig.pn.ptr, *HPn = (c128*)eig.hpn.ptr;
  c128* S = (c128*)eig.S.ptr;
  c128* A = (c128*)eig.A.ptr;
  c128* C = (c128*)eig.C.ptr;
  double* lam = (double*)eig.lam.ptr;
  int* status = (int*)eig.status.ptr;
  const size_t bytes = (size_t)nk * nb * nr * sizeof(c128);
  const long count = (long)nk * nb * nr;
  std::vector<int> hstat(nk);
  std::vector<double> hn(nk * nb);

  // Rayleigh-Ritz on the columns Z (h Z in HZ): X <- Z C, h X <- HZ C and, with
  // keep_p, P <- the non-X part of Z C, h P likewise; false if the X block of
  // the basis was dependent
  auto rayleigh_ritz = [&](const ColSet& Z, const ColSet& HZ, bool keep_p, bool* ok) -> fock_status {
    const int m = Z.total();
    hipError_t er;
    if ((er = launch_gram(S, Z, Z, nk, nr, w, st)) != hipSuccess) return hip_fail(er, "Gram matrix");
    if ((er = launch_gram(A, Z, HZ, nk, nr, w, st)) != hipSuccess) return hip_fail(er, "projected Hamiltonian");
    if ((er = launch_rayleigh_ritz(S, A, m, nb, nb, C, lam, status, nk, st)) != hipSuccess)
      return hip_fail(er, "Rayleigh-Ritz");
    if ((er = hipMemcpyAsync(hstat.data(), status, nk * sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(er, "Ritz status");
    if ((er = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(er, "Ritz sync");
    *ok = std::all_of(hstat.begin(), hstat.end(), [](int v) { return v == 0; });
    if (!*ok) return FOCK_OK;
    if ((er = launch_rotate(Xn, Z, C, 0, m, nb, nk, nr, st)) != hipSuccess) return hip_fail(er, "Ritz vectors");
    if ((er = launch_rotate(HXn, HZ, C, 0, m, nb, nk, nr, st)) != hipSuccess) return hip_fail(er, "Ritz vectors");
    if (keep_p) {
      ColSet Zr = Z, HZr = HZ;  // the columns after the X block
      for (int q = 0; q + 1 < Z.nparts; ++q) {
        Zr.p[q] = Z.p[q + 1];
        Zr.cnt[q] = Z.cnt[q + 1];
        HZr.p[q] = HZ.p[q + 1];
        HZr.cnt[q] = HZ.cnt[q + 1];
      }
      Zr.nparts = HZr.nparts = Z.nparts - 1;
      if ((er = launch_rotate(Pn, Zr, C, nb, m, nb, nk, nr, st)) != hipSuccess) return hip_fail(er, "search directions");
      if ((er = launch_rotate(HPn, HZr, C, nb, m, nb, nk, nr, st)) != hipSuccess) return hip_fail(er, "search directions");
      std::swap(P, Pn);
      std::swap(HP, HPn);
    }
    std::swap(X, Xn);
    std::swap(HX, HXn);
    return FOCK_OK;
  };

  // start: orthonormal guess, h X, Ritz vectors of span(X)
  if ((e = hipMemcpyAsync(X, phi, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy guess");
  if ((e = launch_mgs(X, nk, nb, c.nr, w, st)) != hipSuccess) return hip_fail(e, "Gram-Schmidt");
  if ((s = h_apply(c, us, nullptr, X, HX, nullptr, 1.0, 0.0, vloc, a, alpha, st)) != FOCK_OK) return s;
  bool ok = false;
  if ((s = rayleigh_ritz(cols({{X, nb}}), cols({{HX, nb}}), false, &ok)) != FOCK_OK) return s;
  if (!ok) return fail(FOCK_ERR_ARG, "the initial vectors are linearly dependent");

  bool have_p = false;
  int it = 0;
  double maxres = 0.0;
  for (;; ++it) {
    if (it > 0 && it % kRefresh == 0 &&
        (s = h_apply(c, us, nullptr, X, HX, nullptr, 1.0, 0.0, vloc, a, alpha, st)) != FOCK_OK)
      return s;
    if ((e = launch_resid(W, HX, X, lam, nr, count, st)) != hipSuccess) return hip_fail(e, "residuals");
    if ((e = launch_norms((double*)norms.ptr, W, nk * nb, c.nr, st)) != hipSuccess) return hip_fail(e, "residual norms");
    if ((e = hipMemcpyAsync(hn.data(), norms.ptr, nk * nb * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(e, "residual norms");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "residual sync");
    maxres = 0.0;
    for (double& v : hn) {
      v = std::sqrt(w * v);
      maxres = std::max(maxres, v);
    }
    if (maxres <= tol || it >= maxit) break;
    // W = T R
    if ((e = launch_fft3_plain(W, nk * nb, c.geom, -1, st)) != hipSuccess) return hip_fail(e, "preconditioner FFT");
    if ((e = launch_precond_mul(W, (const double*)c.kvec.ptr, nk, nb, c.geom, a, kPrecondE0, 1.0 / c.nr, st)) !=
        hipSuccess)
      return hip_fail(e, "preconditioner");
    if ((e = launch_fft3_plain(W, nk * nb, c.geom, +1, st)) != hipSuccess) return hip_fail(e, "preconditioner FFT");
    // soft locking of the converged bands
    const double* nrm = (const double*)norms.ptr;
    if ((e = launch_lock(W, nrm, w, tol, nr, count, st)) != hipSuccess) return hip_fail(e, "locking");
    if (have_p && ((e = launch_lock(P, nrm, w, tol, nr, count, st)) != hipSuccess ||
                   (e = launch_lock(HP, nrm, w, tol, nr, count, st)) != hipSuccess))
      return hip_fail(e, "locking");
    if ((s = h_apply(c, us, nullptr, W, HW, nullptr, 1.0, 0.0, vloc, a, alpha, st)) != FOCK_OK) return s;
    ok = false;
    if (have_p) {
      if ((s = rayleigh_ritz(cols({{X, nb}, {W, nb}, {P, nb}}), cols({{HX, nb}, {HW, nb}, {HP, nb}}), true, &ok)) !=
          FOCK_OK)
        return s;
    }
    if (!ok) {
      if ((s = rayleigh_ritz(cols({{X, nb}, {W, nb}}), cols({{HX, nb}, {HW, nb}}), true, &ok)) != FOCK_OK) return s;
      if (!ok) return fail(FOCK_ERR_STATE, "eigensolver basis collapsed at iteration %d", it);
    }
    have_p = true;
  }
  if ((e = hipMemcpyAsync(phi, X, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy result");
  if (eig_host &&
      (e = hipMemcpyAsync(eig_host, lam, nk * nb * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(e, "eigenvalues");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "eigensolver sync");
  if (res_host) std::copy(hn.begin(), hn.end(), res_host);
  if (iters_host) *iters_host = it;
  return maxres <= tol ? FOCK_OK : FOCK_WARN_CONV;
}

fock_status Plan::excited_density(Cell& c, const c128* phi, const c128* psi, hipStream_t st, double* nex) {
  const int nk = c.nk, nb = c.nb;
  fock_status s;
  hipError_t e;
  if ((s = eig.S.ensure((size_t)nk * nb * nb * sizeof(c128), workspace_cap, "overlaps")) != FOCK_OK) return s;
  if ((s = dotres.ensure(2 * sizeof(double), 0, "reduction")) != FOCK_OK) return s;
  c128* O = (c128*)eig.S.ptr;
  if ((e = launch_gram(O, cols({{phi, nb}}), cols({{psi, nb}}), nk, c.nr, c.vol / c.nr, st)) != hipSuccess)
    return hip_fail(e, "overlaps");
  if ((e = launch_sum_abs2((double*)dotres.ptr, O, (long)nk * nb * nb, st)) != hipSuccess)
    return hip_fail(e, "overlap sum");
  double kept = 0.0;
  if ((e = hipMemcpyAsync(&kept, dotres.ptr, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(e, "overlap sum");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "overlap sync");
  *nex = c.gs / (nk * c.vol) * ((double)nk * nb - kept);
  return FOCK_OK;
}

void EigState::release() {
  for (DevBuf* b : {&x, &hx, &w, &hw, &p, &hp, &xn, &hxn, &pn, &hpn, &S, &A, &C, &lam, &status}) b->release();
}

}  // namespace fockmi

namespace {

fock_status checks(fockmi_plan plan, int cell, Plan** pp) {
  g_last_error.clear();
  if (!plan) return fail(FOCK_ERR_ARG, "plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  fock_status s = p->check_ready(cell);
  if (s != FOCK_OK) return s;
  *pp = p;
  return FOCK_OK;
}

}  // namespace

extern "C" {

fock_status fock_eigensolve(fockmi_plan plan, int cell, const void* u_occ, const double* vloc, const double A_over_c[3],
                            double alpha, void* phi, double tol, int maxit, double* eig_host, double* res_host,
                            int* iters_host, void* stream) {
  Plan* p = nullptr;
  fock_status s = checks(plan, cell, &p);
  if (s != FOCK_OK) return s;
  Cell& c = p->cells[cell];
  if (!u_occ || !phi || !A_over_c) return fail(FOCK_ERR_ARG, "NULL argument");
  if (!aligned16(u_occ) || !aligned16(phi) || (vloc && ((uintptr_t)vloc & 7u))) return fail(FOCK_ERR_ARG, "misaligned pointer");
  if (c.nb > kRotMaxCols) return fail(FOCK_ERR_SIZE, "the eigensolver takes at most %d bands per k (got %d)", kRotMaxCols, c.nb);
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FOCK_ERR_ARG, "tol must be positive");
  if (maxit < 0) return fail(FOCK_ERR_ARG, "maxit must be >= 0");
  if (!std::isfinite(alpha) || !std::isfinite(A_over_c[0]) || !std::isfinite(A_over_c[1]) || !std::isfinite(A_over_c[2]))
    return fail(FOCK_ERR_ARG, "alpha and A/c must be finite");
  const size_t bytes = (size_t)c.nk * c.nb * c.nr * sizeof(c128);
  if (overlap(u_occ, bytes, phi, bytes)) return fail(FOCK_ERR_ARG, "phi must not alias u_occ");
  return p->eigensolve(c, (const c128*)u_occ, (c128*)phi, vloc, A_over_c, alpha, tol, maxit, eig_host, res_host,
                       iters_host, (hipStream_t)stream);
}

fock_status fock_excited_density(fockmi_plan plan, int cell, const void* phi, const void* psi, double* nex_host,
                                 void* stream) {
  Plan* p = nullptr;
  fock_status s = checks(plan, cell, &p);
  if (s != FOCK_OK) return s;
  if (!phi || !psi || !nex_host) return fail(FOCK_ERR_ARG, "NULL argument");
  if (!aligned16(phi) || !aligned16(psi)) return fail(FOCK_ERR_ARG, "misaligned pointer");
  return p->excited_density(p->cells[cell], (const c128*)phi, (const c128*)psi, (hipStream_t)stream, nex_host);
}

}  // extern "C"
