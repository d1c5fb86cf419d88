// Plan set-up: geometry, the distinct pair momenta q = k_t - k_s of a cell and
// the kernel tables K_q (built on the GPU in FP64, see table.hip).
#include <cmath>
#include <cstdlib>
#include <map>
#include <tuple>

#include "plan.hpp"

namespace fockmi {

namespace {

void reciprocal_rows(const double a[3][3], double B[3][3], double* vol) {
  // B = 2 pi inv(a)^T, rows b_d with a_i . b_j = 2 pi delta_ij
  const double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                     a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                     a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  *vol = std::fabs(det);
  double inv[3][3];
  inv[0][0] = (a[1][1] * a[2][2] - a[1][2] * a[2][1]) / det;
  inv[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / det;
  inv[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / det;
  inv[1][0] = (a[1][2] * a[2][0] - a[1][0] * a[2][2]) / det;
  inv[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / det;
  inv[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / det;
  inv[2][0] = (a[1][0] * a[2][1] - a[1][1] * a[2][0]) / det;
  inv[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) / det;
  inv[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / det;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B[i][j] = 2.0 * M_PI * inv[j][i];
}

}  // namespace

fock_status Plan::init_cell(Cell& c, const fock_cell_desc& d, int index) {
  if (const char* capenv = std::getenv("FOCKMI_WORKSPACE_CAP")) workspace_cap = (size_t)std::strtoull(capenv, 0, 10);
  c.geom.n1 = d.n[0];
  c.geom.n2 = d.n[1];
  c.geom.n3 = d.n[2];
  c.nr = d.n[0] * d.n[1] * d.n[2];
  c.nk = d.nk;
  c.nb = d.nb;
  c.omega = d.omega;
  c.gs = d.gs;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c.a[i][j] = d.a[i][j];
  reciprocal_rows(c.a, c.geom.B, &c.vol);
  if (!(c.vol > 0.0) || !std::isfinite(c.vol)) return fail(FOCK_ERR_ARG, "cell %d: singular lattice", index);
  c.kpts.assign(d.kpts, d.kpts + 3 * (size_t)d.nk);
  for (double v : c.kpts)
    if (!std::isfinite(v)) return fail(FOCK_ERR_ARG, "cell %d: non-finite k-point", index);

  // distinct q = k_t - k_s; q = 0 exactly when t == s (distinct k-points required)
  double bscale = 0.0;
  for (int i = 0; i < 3; ++i)
    bscale = std::fmax(bscale, std::sqrt(c.geom.B[i][0] * c.geom.B[i][0] + c.geom.B[i][1] * c.geom.B[i][1] +
                                         c.geom.B[i][2] * c.geom.B[i][2]));
  const double tol = 1e-13 * bscale;
  std::map<std::tuple<long long, long long, long long>, int> seen;
  std::vector<double> qv;
  std::vector<int> qz;
  c.qidx_host.assign((size_t)c.nk * c.nk, -1);
  for (int t = 0; t < c.nk; ++t) {
    for (int s = 0; s < c.nk; ++s) {
      double q[3];
      for (int dd = 0; dd < 3; ++dd) q[dd] = c.kpts[3 * t + dd] - c.kpts[3 * s + dd];
      if (t != s && std::fabs(q[0]) <= tol && std::fabs(q[1]) <= tol && std::fabs(q[2]) <= tol)
        return fail(FOCK_ERR_ARG, "cell %d: k-points %d and %d coincide", index, t, s);
      auto key = std::make_tuple(std::llround(q[0] / tol), std::llround(q[1] / tol), std::llround(q[2] / tol));
      if (t == s) key = std::make_tuple(0LL, 0LL, 0LL);
      auto it = seen.find(key);
      int id;
      if (it == seen.end()) {
        id = (int)qz.size();
        seen.emplace(key, id);
        for (int dd = 0; dd < 3; ++dd) qv.push_back(t == s ? 0.0 : q[dd]);
        qz.push_back(t == s ? 1 : 0);
      } else {
        id = it->second;
      }
      c.qidx_host[(size_t)t * c.nk + s] = id;
    }
  }
  c.nq = (int)qz.size();

  fock_status s;
  if ((s = c.qidx.ensure(c.qidx_host.size() * sizeof(int), 0, "q index table")) != FOCK_OK) return s;
  if ((s = c.qvec.ensure(qv.size() * sizeof(double), 0, "q vectors")) != FOCK_OK) return s;
  if ((s = c.qzero.ensure(qz.size() * sizeof(int), 0, "q flags")) != FOCK_OK) return s;
  hipError_t e;
  if ((e = hipMemcpy(c.qidx.ptr, c.qidx_host.data(), c.qidx_host.size() * sizeof(int), hipMemcpyHostToDevice)) !=
      hipSuccess)
    return hip_fail(e, "upload q index");
  if ((e = hipMemcpy(c.qvec.ptr, qv.data(), qv.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "upload q vectors");
  if ((e = hipMemcpy(c.qzero.ptr, qz.data(), qz.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "upload q flags");

  // down-sampling: the source sub-mesh S (validated at plan creation) and the
  // table rows of (target, source) pairs in both roles
  c.src.clear();
  if (d.nsrc > 0 && d.src) {
    bool identity = d.nsrc == c.nk;
    for (int i = 0; i < d.nsrc; ++i) {
      identity = identity && d.src[i] == i;
      c.src.push_back(d.src[i]);
    }
    c.ds = !identity;
  }
  if (!c.ds) {
    c.src.resize(c.nk);
    for (int k = 0; k < c.nk; ++k) c.src[k] = k;
  }
  c.nsrc = (int)c.src.size();
  if (c.ds) {
    std::vector<int> ts((size_t)c.nk * c.nsrc), stt((size_t)c.nsrc * c.nk);
    for (int t = 0; t < c.nk; ++t)
      for (int i = 0; i < c.nsrc; ++i) ts[(size_t)t * c.nsrc + i] = c.qidx_host[(size_t)t * c.nk + c.src[i]];
    for (int i = 0; i < c.nsrc; ++i)
      for (int k = 0; k < c.nk; ++k) stt[(size_t)i * c.nk + k] = c.qidx_host[(size_t)c.src[i] * c.nk + k];
    if ((s = c.qidx_ts.ensure(ts.size() * sizeof(int), 0, "q index table (sources)")) != FOCK_OK) return s;
    if ((s = c.qidx_st.ensure(stt.size() * sizeof(int), 0, "q index table (reverse)")) != FOCK_OK) return s;
    if ((e = hipMemcpy(c.qidx_ts.ptr, ts.data(), ts.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "upload q index");
    if ((e = hipMemcpy(c.qidx_st.ptr, stt.data(), stt.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "upload q index");
  }

  if ((s = c.kvec.ensure(c.kpts.size() * sizeof(double), 0, "k-points")) != FOCK_OK) return s;
  if ((e = hipMemcpy(c.kvec.ptr, c.kpts.data(), c.kpts.size() * sizeof(double), hipMemcpyHostToDevice)) !=
      hipSuccess)
    return hip_fail(e, "upload k-points");
  if ((s = c.K64.ensure((size_t)c.nq * c.nr * sizeof(double), 0, "FP64 kernel tables")) != FOCK_OK) return s;
  if ((e = launch_build_table_f64((double*)c.K64.ptr, (const double*)c.qvec.ptr, (const int*)c.qzero.ptr, c.nq,
                                  c.geom, c.omega, 1.0 / c.nr, 0)) != hipSuccess)
    return hip_fail(e, "kernel table");
  if (prec == FOCK_FP32_COMP && !(c.geom.n1 == c.geom.n2 && c.geom.n2 == c.geom.n3)) {
    // the fused kernels take cubic grids; this cell runs the plain stages in FP32
    c.f32plain = true;
  } else if (prec == FOCK_FP32_COMP) {
    if ((s = c.Kt.ensure((size_t)c.nq * c.nr * sizeof(float), 0, "FP32 kernel tables")) != FOCK_OK) return s;
    if ((e = launch_build_table_fused((float*)c.Kt.ptr, (const double*)c.K64.ptr, c.nq, c.geom.n1, 0)) !=
        hipSuccess)
      return hip_fail(e, "FP32 kernel table");
    if (c.geom.n1 == 32) {
      // (S, D) pairs of the split 32^3 form
      if ((s = c.SD.ensure(split32_sd_floats(c.nq) * sizeof(float), 0, "split-form kernel tables")) != FOCK_OK)
        return s;
      if ((e = launch_build_sd32((float*)c.SD.ptr, (const double*)c.K64.ptr, c.nq, 0)) != hipSuccess)
        return hip_fail(e, "split-form kernel table");
    }
  }
  if (prec == FOCK_FP64_FUSED && c.geom.n1 == c.geom.n2 && c.geom.n2 == c.geom.n3 && fused64_supported(c.geom.n1)) {
    if ((s = c.Kt64.ensure((size_t)c.nq * c.nr * sizeof(double), 0, "fused FP64 kernel tables")) != FOCK_OK)
      return s;
    if ((e = launch_build_table_fused64((double*)c.Kt64.ptr, (const double*)c.K64.ptr, c.nq, c.geom.n1,
                                        fused64_phases(c.geom.n1), 0)) != hipSuccess)
      return hip_fail(e, "fused FP64 kernel table");
    c.f64f = true;
  }
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "plan set-up");
  return FOCK_OK;
}

hipError_t Plan::prof_begin(hipStream_t st) {
  if (!profiling) return hipSuccess;
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e != hipSuccess) return e;
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return e;
  }
  prof_events.emplace_back(a, b);
  return hipEventRecord(a, st);
}

hipError_t Plan::prof_end(hipStream_t st) {
  if (!profiling || prof_events.empty()) return hipSuccess;
  return hipEventRecord(prof_events.back().second, st);
}

fock_status Plan::prof_collect() {
  for (auto& ev : prof_events) {
    hipError_t e = hipEventSynchronize(ev.second);
    if (e != hipSuccess) return hip_fail(e, "profile event");
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, ev.first, ev.second)) != hipSuccess) return hip_fail(e, "profile elapsed");
    prof_ms += ms;
    ++prof_launches;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  prof_events.clear();
  return FOCK_OK;
}

void Plan::destroy() {
  for (auto& ev : prof_events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  prof_events.clear();
  for (Cell& c : cells) {
    c.qidx.release();
    c.qidx_ts.release();
    c.qidx_st.release();
    c.qvec.release();
    c.qzero.release();
    c.K64.release();
    c.Kt.release();
    c.SD.release();
    c.Kt64.release();
    c.kvec.release();
  }
  for (DevBuf* b : {&batch, &shadow_x, &shadow_p, &shadow_m, &comp, &accs, &vu, &partial, &dotres, &srcbuf, &srcout,
                    &psi0, &phiA, &phiB, &predb, &srcbuf2, &kin, &vxb, &lam, &lam2, &gtmp, &ftmp, &phis, &norms,
                    &red6, &vloc_buf, &sync, &parts, &xbuf, &sflags, &sstatus, &fallbacks, &mpart, &msum, &mcomp,
                    &mdone, &sym_rank, &sym_cnt})
    b->release();
  bstate.release();
  eig.release();
  if (host_pinned) (void)hipHostFree(host_pinned);
  host_pinned = nullptr;
  magic = 0;
}

fock_status Plan::dot(const c128* a, const c128* b, size_t count, hipStream_t st, double* re, double* im) {
  double r[4];
  fock_status s = dot_dd(a, b, count, st, r);
  if (s != FOCK_OK) return s;
  *re = r[0] + r[1];
  *im = r[2] + r[3];
  return FOCK_OK;
}

fock_status Plan::dot_dd(const c128* a, const c128* b, size_t count, hipStream_t st, double out[4]) {
  const int nblk = 1024;
  fock_status s;
  if ((s = partial.ensure(4 * nblk * sizeof(double), 0, "reduction partials")) != FOCK_OK) return s;
  if ((s = dotres.ensure(4 * sizeof(double), 0, "reduction result")) != FOCK_OK) return s;
  hipError_t e;
  if (!host_pinned) {
    if ((e = hipHostMalloc((void**)&host_pinned, 4 * sizeof(double), 0)) != hipSuccess)
      return hip_fail(e, "pinned host buffer");
  }
  if ((e = launch_dot((double*)dotres.ptr, (double*)partial.ptr, nblk, a, b, (long)count, st)) != hipSuccess)
    return hip_fail(e, "reduction");
  if ((e = hipMemcpyAsync(host_pinned, dotres.ptr, 4 * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(e, "reduction copy");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "reduction sync");
  for (int i = 0; i < 4; ++i) out[i] = host_pinned[i];
  return FOCK_OK;
}

}  // namespace fockmi
