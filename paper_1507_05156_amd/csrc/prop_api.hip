// Taylor propagation (Eqs. (9)-(10)), its reverse mode, the energy functional
// (Eq. (22) restricted to kinetic + local + Fock-like pieces) and FP64
// orthonormalisation, on top of the exchange operator of api.hip.
//
// One step: psi <- sum_{m=0}^{M} phi_m, phi_0 = psi(t_n),
//           phi_m = (-i dt / m) h phi_{m-1},
//           h = T[a] + v_loc + alpha V_x[psi(t_n)]   (h(t + dt/2) ~ h(t_n), V_x frozen)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/fockmi.h"
#include "plan.hpp"
#include "prop.hpp"

using namespace fockmi;

namespace fockmi {

extern thread_local std::string g_last_error;

fock_status Plan::field_bufs(Cell& c, std::initializer_list<DevBuf*> bufs, int nf) {
  const size_t bytes = (size_t)c.nk * nf * c.nr * sizeof(c128);
  for (DevBuf* b : bufs) {
    fock_status s = b->ensure(bytes, workspace_cap, "propagator work array");
    if (s != FOCK_OK) return s;
  }
  return FOCK_OK;
}

// y = T[a] x (FFT, multiply by |k+G+a|^2/2 / N_r, inverse FFT), x and y distinct
fock_status Plan::kinetic(Cell& c, const c128* x, int nf, c128* y, const double a[3], hipStream_t st) {
  const size_t bytes = (size_t)c.nk * nf * c.nr * sizeof(c128);
  hipError_t e;
  if ((e = hipMemcpyAsync(y, x, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "kinetic copy");
  if ((e = launch_fft3_plain(y, c.nk * nf, c.geom, -1, st)) != hipSuccess) return hip_fail(e, "kinetic FFT");
  if ((e = launch_kinetic_mul(y, (const double*)c.kvec.ptr, c.nk, nf, c.geom, a, 1.0 / c.nr, st)) != hipSuccess)
    return hip_fail(e, "kinetic multiply");
  if ((e = launch_fft3_plain(y, c.nk * nf, c.geom, +1, st)) != hipSuccess) return hip_fail(e, "kinetic inverse FFT");
  return FOCK_OK;
}

// out = (base ? base : 0) + (cre + i cim) * h x, with h = T[a] + v_loc + alpha V_x[u]; out distinct from x.
// us holds the orbitals of the source k-points (Plan::sources of u). With a
// second source set us2, the exchange term is the average alpha (V_x[u] + V_x[u2]) / 2.
fock_status Plan::h_apply(Cell& c, const c128* us, const c128* us2, const c128* x, c128* out, const c128* base,
                          double cre, double cim, const double* vloc, const double a[3], double alpha,
                          hipStream_t st) {
  fock_status s;
  if ((s = field_bufs(c, {&kin}, c.nb)) != FOCK_OK) return s;
  if ((s = kinetic(c, x, c.nb, (c128*)kin.ptr, a, st)) != FOCK_OK) return s;
  const c128* vx = nullptr;
  if (alpha != 0.0) {
    if ((s = field_bufs(c, {&vxb}, c.nb)) != FOCK_OK) return s;
    const double w = (us2 ? 0.5 : 1.0) / c.nsrc;
    if ((s = general(c, c.fwd(), x, c.nb, us, us, c.nb, (c128*)vxb.ptr, -w, false, st)) != FOCK_OK) return s;
    if (us2 && (s = general(c, c.fwd(), x, c.nb, us2, us2, c.nb, (c128*)vxb.ptr, -w, true, st)) != FOCK_OK)
      return s;
    vx = (const c128*)vxb.ptr;
  }
  const long count = (long)c.nk * c.nb * c.nr;
  hipError_t e = launch_hcombine(out, base, (const c128*)kin.ptr, x, vx, vloc, alpha, cre, cim, count, c.nr, st);
  if (e != hipSuccess) return hip_fail(e, "h combine");
  return FOCK_OK;
}

fock_status Plan::taylor_sum(Cell& c, const c128* us, const c128* us2, const c128* x0, c128* acc,
                             const double* vloc, const double a[3], double dt, double alpha, int order,
                             hipStream_t st) {
  fock_status s;
  if ((s = field_bufs(c, {&phiA, &phiB}, c.nb)) != FOCK_OK) return s;
  const size_t bytes = (size_t)c.nk * c.nb * c.nr * sizeof(c128);
  const long count = (long)c.nk * c.nb * c.nr;
  c128* cur = (c128*)phiA.ptr;
  c128* nxt = (c128*)phiB.ptr;
  hipError_t e;
  if ((e = hipMemcpyAsync(cur, x0, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy psi");
  if (acc != x0 && (e = hipMemcpyAsync(acc, x0, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return hip_fail(e, "copy psi");
  for (int m = 1; m <= order; ++m) {
    // phi_m = (-i dt/m) h phi_{m-1}
    if ((s = h_apply(c, us, us2, cur, nxt, nullptr, 0.0, -dt / m, vloc, a, alpha, st)) != FOCK_OK) return s;
    if ((e = launch_scale_add(acc, nxt, 1.0, 0.0, count, st)) != hipSuccess) return hip_fail(e, "accumulate step");
    std::swap(cur, nxt);
  }
  return FOCK_OK;
}

fock_status Plan::norm_dev(Cell& c, const c128* psi, hipStream_t st, double* dev) {
  const int nf = c.nk * c.nb;
  fock_status s;
  hipError_t e;
  if ((s = norms.ensure(nf * sizeof(double), 0, "norms")) != FOCK_OK) return s;
  if ((e = launch_norms((double*)norms.ptr, psi, nf, c.nr, st)) != hipSuccess) return hip_fail(e, "norms");
  host_norms.resize(nf);
  if ((e = hipMemcpyAsync(host_norms.data(), norms.ptr, nf * sizeof(double), hipMemcpyDeviceToHost, st)) !=
      hipSuccess)
    return hip_fail(e, "norm copy");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "norm sync");
  double d = 0.0;
  const double w = c.vol / c.nr;
  for (double n2 : host_norms) d = std::max(d, std::fabs(w * n2 - 1.0));
  *dev = d;
  return FOCK_OK;
}

}  // namespace fockmi

namespace {

fock_status common_checks(fockmi_plan plan, int cell, Plan** pp) {
  g_last_error.clear();
  if (!plan) return fail(FOCK_ERR_ARG, "plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  fock_status s = p->check_ready(cell);
  if (s != FOCK_OK) return s;
  *pp = p;
  return FOCK_OK;
}

fock_status check_step_args(const Cell& c, double dt, int order, const double* A_over_c) {
  if (!A_over_c) return fail(FOCK_ERR_ARG, "A_over_c is NULL");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(A_over_c[d])) return fail(FOCK_ERR_ARG, "A_over_c is not finite");
  if (!std::isfinite(dt) || dt <= 0.0) return fail(FOCK_ERR_ARG, "dt must be > 0");
  if (order < 1 || order > 4) return fail(FOCK_ERR_ARG, "order must be in 1..4 (got %d)", order);
  (void)c;
  return FOCK_OK;
}

}  // namespace

extern "C" {

fock_status taylor_step(fockmi_plan plan, int cell, void* psi, const double* vloc, const double A_over_c[3],
                        double dt, double alpha, int order, double* max_norm_dev, void* stream) {
  Plan* p = nullptr;
  fock_status s = common_checks(plan, cell, &p);
  if (s != FOCK_OK) return s;
  Cell& c = p->cells[cell];
  if (!psi) return fail(FOCK_ERR_ARG, "psi is NULL");
  if (!aligned16(psi) || (vloc && ((uintptr_t)vloc & 7u))) return fail(FOCK_ERR_ARG, "misaligned pointer");
  if ((s = check_step_args(c, dt, order, A_over_c)) != FOCK_OK) return s;
  if (!std::isfinite(alpha)) return fail(FOCK_ERR_ARG, "alpha is not finite");
  hipStream_t st = (hipStream_t)stream;
  if ((s = p->field_bufs(c, {&p->psi0}, c.nb)) != FOCK_OK) return s;
  const size_t bytes = (size_t)c.nk * c.nb * c.nr * sizeof(c128);
  c128* P = (c128*)psi;
  c128* psi0 = (c128*)p->psi0.ptr;
  hipError_t e;
  if ((e = hipMemcpyAsync(psi0, P, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy psi");
  const c128* us = nullptr;  // V_x is built from psi(t_n) on the source k-points
  if ((s = p->sources(c, psi0, c.nb, p->srcbuf, st, &us)) != FOCK_OK) return s;
  if ((s = p->taylor_sum(c, us, nullptr, psi0, P, vloc, A_over_c, dt, alpha, order, st)) != FOCK_OK) return s;
  if (!max_norm_dev) return FOCK_OK;
  if ((s = p->norm_dev(c, P, st, max_norm_dev)) != FOCK_OK) return s;
  return *max_norm_dev > 1e-6 ? FOCK_WARN_NORM : FOCK_OK;
}

fock_status taylor_step_pc(fockmi_plan plan, int cell, void* psi, const double* vloc, const double A_now[3],
                           const double A_mid[3], double dt, double alpha, int order, double* max_norm_dev,
                           void* stream) {
  Plan* p = nullptr;
  fock_status s = common_checks(plan, cell, &p);
  if (s != FOCK_OK) return s;
  Cell& c = p->cells[cell];
  if (!psi) return fail(FOCK_ERR_ARG, "psi is NULL");
  if (!aligned16(psi) || (vloc && ((uintptr_t)vloc & 7u))) return fail(FOCK_ERR_ARG, "misaligned pointer");
  if ((s = check_step_args(c, dt, order, A_now)) != FOCK_OK) return s;
  if ((s = check_step_args(c, dt, order, A_mid)) != FOCK_OK) return s;
  if (!std::isfinite(alpha)) return fail(FOCK_ERR_ARG, "alpha is not finite");
  hipStream_t st = (hipStream_t)stream;
  if ((s = p->field_bufs(c, {&p->psi0, &p->predb}, c.nb)) != FOCK_OK) return s;
  const size_t bytes = (size_t)c.nk * c.nb * c.nr * sizeof(c128);
  c128* P = (c128*)psi;
  c128* psi0 = (c128*)p->psi0.ptr;
  c128* pred = (c128*)p->predb.ptr;
  hipError_t e;
  if ((e = hipMemcpyAsync(psi0, P, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy psi");
  const c128* us = nullptr;
  if ((s = p->sources(c, psi0, c.nb, p->srcbuf, st, &us)) != FOCK_OK) return s;
  // predictor with h(t): A(t_n), V_x[psi(t_n)]
  if ((s = p->taylor_sum(c, us, nullptr, psi0, pred, vloc, A_now, dt, alpha, order, st)) != FOCK_OK) return s;
  // corrector with A(t_n + dt/2) and the exchange potentials of psi(t_n) and psi_pred averaged
  const c128* ups = nullptr;
  if ((s = p->sources(c, pred, c.nb, p->srcbuf2, st, &ups)) != FOCK_OK) return s;
  if ((s = p->taylor_sum(c, us, ups, psi0, P, vloc, A_mid, dt, alpha, order, st)) != FOCK_OK) return s;
  if (!max_norm_dev) return FOCK_OK;
  if ((s = p->norm_dev(c, P, st, max_norm_dev)) != FOCK_OK) return s;
  return *max_norm_dev > 1e-6 ? FOCK_WARN_NORM : FOCK_OK;
}

fock_status taylor_step_vjp(fockmi_plan plan, int cell, const void* psi_n, const double* vloc,
                            const double A_over_c[3], double dt, double alpha, int order, const void* g_next,
                            void* g_psi, double g_a[3], void* stream) {
  Plan* p = nullptr;
  fock_status s = common_checks(plan, cell, &p);
  if (s != FOCK_OK) return s;
  Cell& c = p->cells[cell];
  if (c.ds) return fail(FOCK_ERR_ARG, "taylor_step_vjp is not available for a down-sampled cell");
  if (!psi_n || !g_next || !g_psi || !g_a) return fail(FOCK_ERR_ARG, "NULL pointer");
  if (!aligned16(psi_n) || !aligned16(g_next) || !aligned16(g_psi)) return fail(FOCK_ERR_ARG, "misaligned pointer");
  if ((s = check_step_args(c, dt, order, A_over_c)) != FOCK_OK) return s;
  const size_t bytes = (size_t)c.nk * c.nb * c.nr * sizeof(c128);
  if (overlap(g_psi, bytes, psi_n, bytes) || overlap(g_psi, bytes, g_next, bytes))
    return fail(FOCK_ERR_ARG, "g_psi overlaps an input");
  hipStream_t st = (hipStream_t)stream;
  const long count = (long)c.nk * c.nb * c.nr;
  // forward recomputation: phi_0 .. phi_{M-1}
  if ((s = p->phis.ensure(bytes * order, p->workspace_cap, "stored Taylor terms")) != FOCK_OK) return s;
  if ((s = p->field_bufs(c, {&p->lam, &p->lam2, &p->gtmp, &p->ftmp}, c.nb)) != FOCK_OK) return s;
  c128* phis = (c128*)p->phis.ptr;
  const c128* U = (const c128*)psi_n;
  const c128* G = (const c128*)g_next;
  hipError_t e;
  if ((e = hipMemcpyAsync(phis, U, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy");
  for (int m = 1; m < order; ++m) {
    if ((s = p->h_apply(c, U, nullptr, phis + (size_t)(m - 1) * count, phis + (size_t)m * count, nullptr, 0.0, -dt / m, vloc,
                        A_over_c, alpha, st)) != FOCK_OK)
      return s;
  }
  c128* lam = (c128*)p->lam.ptr;
  c128* lam2 = (c128*)p->lam2.ptr;
  c128* gt = (c128*)p->gtmp.ptr;
  c128* ft = (c128*)p->ftmp.ptr;
  c128* GP = (c128*)g_psi;
  if ((e = hipMemcpyAsync(lam, G, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy");
  if ((e = hipMemsetAsync(GP, 0, bytes, st)) != hipSuccess) return hip_fail(e, "zero g_psi");
  const int nblk = 512;
  if ((s = p->partial.ensure(6 * nblk * sizeof(double), 0, "reduction partials")) != FOCK_OK) return s;
  if ((s = p->red6.ensure(6 * sizeof(double) * order, 0, "reduction results")) != FOCK_OK) return s;
  for (int m = order; m >= 1; --m) {
    const c128* phim1 = phis + (size_t)(m - 1) * count;
    // c_m = -i dt/m ; conj(c_m) = +i dt/m
    // d L / d a: Re[c_m / N_r sum conj(DFT lam_m) (k+G+a) DFT phi_{m-1}]
    if ((e = hipMemcpyAsync(gt, lam, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy");
    if ((e = hipMemcpyAsync(ft, phim1, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy");
    if ((e = launch_fft3_plain(gt, c.nk * c.nb, c.geom, -1, st)) != hipSuccess) return hip_fail(e, "FFT");
    if ((e = launch_fft3_plain(ft, c.nk * c.nb, c.geom, -1, st)) != hipSuccess) return hip_fail(e, "FFT");
    if ((e = launch_agrad((double*)p->red6.ptr + 6 * (m - 1), (double*)p->partial.ptr, nblk, gt, ft,
                          (const double*)c.kvec.ptr, c.nb, c.geom, A_over_c, count, st)) != hipSuccess)
      return hip_fail(e, "A gradient");
    if (alpha != 0.0) {
      // cotangent of V_x[u] phi_{m-1} is conj(c_m) alpha lam_m
      if ((e = hipMemsetAsync(gt, 0, bytes, st)) != hipSuccess) return hip_fail(e, "zero");
      if ((e = launch_scale_add(gt, lam, 0.0, alpha * dt / m, count, st)) != hipSuccess) return hip_fail(e, "scale");
      if ((s = p->general(c, c.rev(), U, c.nb, phim1, gt, c.nb, GP, -1.0 / c.nsrc, true, st)) != FOCK_OK) return s;
      if ((s = p->general(c, c.rev(), U, c.nb, gt, phim1, c.nb, GP, -1.0 / c.nsrc, true, st)) != FOCK_OK) return s;
    }
    // lam_{m-1} = g + conj(c_m) h lam_m
    if ((s = p->h_apply(c, U, nullptr, lam, lam2, G, 0.0, dt / m, vloc, A_over_c, alpha, st)) != FOCK_OK) return s;
    std::swap(lam, lam2);
  }
  if ((e = launch_scale_add(GP, lam, 1.0, 0.0, count, st)) != hipSuccess) return hip_fail(e, "accumulate");
  std::vector<double> red(6 * order);
  if ((e = hipMemcpyAsync(red.data(), p->red6.ptr, red.size() * sizeof(double), hipMemcpyDeviceToHost, st)) !=
      hipSuccess)
    return hip_fail(e, "copy");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "sync");
  for (int d = 0; d < 3; ++d) g_a[d] = 0.0;
  for (int m = 1; m <= order; ++m) {
    // Re[(-i dt/m)(re + i im)] / N_r = (dt/m) im / N_r
    for (int d = 0; d < 3; ++d) g_a[d] += (dt / m) * red[6 * (m - 1) + 2 * d + 1] / c.nr;
  }
  return FOCK_OK;
}

}  // extern "C"

namespace {

// double-double values on the host (hi + lo), for energies whose differences are
// taken: the two-sum keeps the rounding error of every addition
struct hdd {
  double hi, lo;
};
hdd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
hdd dd_add(hdd a, hdd b) {
#pragma clang fp contract(off)
  hdd s = two_sum(a.hi, b.hi);
  return two_sum(s.hi, s.lo + (a.lo + b.lo));
}
hdd dd_scale(hdd a, double c) {
#pragma clang fp contract(off)
  const double p = a.hi * c;
  const double e = std::fma(a.hi, c, -p) + a.lo * c;
  return two_sum(p, e);
}

// E = (g_s/N_k)(Omega/N_r) sum conj(psi) (T[a] + v_loc) psi + alpha E_x[psi] (into *e_out when
// given), and the gradients times the cotangent g_e: grad_psi <- g_e dE/dpsi (PyTorch
// convention, 2 (g_s/N_k)(Omega/N_r) (T + v_loc + alpha V_x[psi]) psi) and grad_a <- g_e dE/d(A/c).
fock_status energy_impl(Plan* p, Cell& c, const void* psi, const double* vloc, const double A_over_c[3], double alpha,
                        double g_e, hdd* e_out, void* grad_psi, double grad_a[3], hipStream_t st) {
  if (c.ds) return fail(FOCK_ERR_ARG, "the energy functional is not available for a down-sampled cell");
  if (!psi || !A_over_c) return fail(FOCK_ERR_ARG, "NULL pointer");
  if (!aligned16(psi) || (grad_psi && !aligned16(grad_psi))) return fail(FOCK_ERR_ARG, "misaligned pointer");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(A_over_c[d])) return fail(FOCK_ERR_ARG, "A_over_c is not finite");
  const size_t bytes = (size_t)c.nk * c.nb * c.nr * sizeof(c128);
  if (grad_psi && overlap(grad_psi, bytes, psi, bytes)) return fail(FOCK_ERR_ARG, "grad_psi overlaps psi");
  const long count = (long)c.nk * c.nb * c.nr;
  const double w = c.gs / c.nk * c.vol / c.nr;
  const c128* P = (const c128*)psi;
  fock_status s;
  hipError_t e;
  if (e_out || grad_psi) {
    if ((s = p->field_bufs(c, {&p->lam}, c.nb)) != FOCK_OK) return s;
    c128* hpsi = (c128*)p->lam.ptr;
    if ((s = p->h_apply(c, P, nullptr, P, hpsi, nullptr, 1.0, 0.0, vloc, A_over_c, alpha, st)) != FOCK_OK) return s;
    if (e_out) {
      // in double-double: sum conj(psi) h psi counts V_x with alpha, the energy
      // counts it with alpha / 2
      double h4[4], x4[4] = {0.0, 0.0, 0.0, 0.0};
      if ((s = p->dot_dd(P, hpsi, count, st, h4)) != FOCK_OK) return s;
      if (alpha != 0.0 && (s = p->dot_dd(P, (const c128*)p->vxb.ptr, count, st, x4)) != FOCK_OK) return s;
      const hdd hx = dd_add(two_sum(h4[0], h4[1]), dd_scale(two_sum(x4[0], x4[1]), -0.5 * alpha));
      *e_out = dd_scale(hx, w);
    }
    if (grad_psi) {
      if ((e = launch_zero((c128*)grad_psi, count, st)) != hipSuccess) return hip_fail(e, "zero");
      if ((e = launch_scale_add((c128*)grad_psi, hpsi, 2.0 * w * g_e, 0.0, count, st)) != hipSuccess)
        return hip_fail(e, "gradient");
    }
  }
  if (grad_a) {
    const int nblk = 512;
    if ((s = p->field_bufs(c, {&p->gtmp}, c.nb)) != FOCK_OK) return s;
    if ((s = p->partial.ensure(6 * nblk * sizeof(double), 0, "reduction partials")) != FOCK_OK) return s;
    if ((s = p->red6.ensure(6 * sizeof(double), 0, "reduction results")) != FOCK_OK) return s;
    c128* F = (c128*)p->gtmp.ptr;
    if ((e = hipMemcpyAsync(F, P, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy");
    if ((e = launch_fft3_plain(F, c.nk * c.nb, c.geom, -1, st)) != hipSuccess) return hip_fail(e, "FFT");
    if ((e = launch_agrad((double*)p->red6.ptr, (double*)p->partial.ptr, nblk, F, F, (const double*)c.kvec.ptr, c.nb,
                          c.geom, A_over_c, count, st)) != hipSuccess)
      return hip_fail(e, "A gradient");
    double red[6];
    if ((e = hipMemcpyAsync(red, p->red6.ptr, sizeof(red), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(e, "copy");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "sync");
    for (int d = 0; d < 3; ++d) grad_a[d] = g_e * w * red[2 * d] / c.nr;
  }
  return FOCK_OK;
}

}  // namespace

extern "C" {

fock_status taylor_energy(fockmi_plan plan, int cell, const void* psi, const double* vloc, const double A_over_c[3],
                          double alpha, double* e_out, void* grad_psi, double grad_a[3], void* stream) {
  Plan* p = nullptr;
  fock_status s = common_checks(plan, cell, &p);
  if (s != FOCK_OK) return s;
  if (!e_out) return fail(FOCK_ERR_ARG, "e_out is NULL");
  hdd e{0.0, 0.0};
  s = energy_impl(p, p->cells[cell], psi, vloc, A_over_c, alpha, 1.0, &e, grad_psi, grad_a, (hipStream_t)stream);
  *e_out = e.hi + e.lo;
  return s;
}

fock_status taylor_excitation_energy(fockmi_plan plan, int cell, const void* psi_t, const double A_t[3],
                                     const void* psi_0, const double A_0[3], const double* vloc, double alpha,
                                     double* e_ex, void* stream) {
  Plan* p = nullptr;
  fock_status s = common_checks(plan, cell, &p);
  if (s != FOCK_OK) return s;
  if (!e_ex) return fail(FOCK_ERR_ARG, "e_ex is NULL");
  hdd et{0.0, 0.0}, e0{0.0, 0.0};
  if ((s = energy_impl(p, p->cells[cell], psi_t, vloc, A_t, alpha, 1.0, &et, nullptr, nullptr, (hipStream_t)stream)) !=
      FOCK_OK)
    return s;
  if ((s = energy_impl(p, p->cells[cell], psi_0, vloc, A_0, alpha, 1.0, &e0, nullptr, nullptr, (hipStream_t)stream)) !=
      FOCK_OK)
    return s;
  const hdd d = dd_add(et, hdd{-e0.hi, -e0.lo});
  *e_ex = d.hi + d.lo;
  return FOCK_OK;
}

fock_status taylor_energy_vjp(fockmi_plan plan, int cell, const void* psi, const double* vloc, const double A_over_c[3],
                              double alpha, double g_e, void* g_psi, double g_a[3], void* stream) {
  Plan* p = nullptr;
  fock_status s = common_checks(plan, cell, &p);
  if (s != FOCK_OK) return s;
  if (!std::isfinite(g_e)) return fail(FOCK_ERR_ARG, "g_e is not finite");
  if (!g_psi && !g_a) return fail(FOCK_ERR_ARG, "both outputs are NULL");
  return energy_impl(p, p->cells[cell], psi, vloc, A_over_c, alpha, g_e, nullptr, g_psi, g_a, (hipStream_t)stream);
}

fock_status taylor_current(fockmi_plan plan, int cell, const void* psi, const double A_over_c[3], double j_out[3],
                           void* stream) {
  Plan* p = nullptr;
  fock_status s = common_checks(plan, cell, &p);
  if (s != FOCK_OK) return s;
  if (!j_out) return fail(FOCK_ERR_ARG, "j_out is NULL");
  Cell& c = p->cells[cell];
  // J = -(1/Omega) dE/d(A/c); V_x does not depend on A in the velocity gauge, so
  // only the kinetic term enters (alpha = 0)
  double ga[3];
  if ((s = energy_impl(p, c, psi, nullptr, A_over_c, 0.0, 1.0, nullptr, nullptr, ga, (hipStream_t)stream)) != FOCK_OK)
    return s;
  for (int d = 0; d < 3; ++d) j_out[d] = -ga[d] / c.vol;
  return FOCK_OK;
}

fock_status fock_orthonormalize(fockmi_plan plan, int cell, void* psi, void* stream) {
  Plan* p = nullptr;
  fock_status s = common_checks(plan, cell, &p);
  if (s != FOCK_OK) return s;
  Cell& c = p->cells[cell];
  if (!psi) return fail(FOCK_ERR_ARG, "psi is NULL");
  if (!aligned16(psi)) return fail(FOCK_ERR_ARG, "misaligned pointer");
  hipError_t e = launch_mgs((c128*)psi, c.nk, c.nb, c.nr, c.vol / c.nr, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "Gram-Schmidt");
  return FOCK_OK;
}

}  // extern "C"
