// Plan object behind the opaque fockmi_plan handle (host side only).
#pragma once

#include <hip/hip_runtime.h>

#include <initializer_list>
#include <string>
#include <vector>

#include "../../include/fockmi.h"
#include "kernels.hpp"
#include "tune.hpp"

namespace fockmi {

fock_status fail(fock_status st, const char* fmt, ...);
// looks up the current device's copy of the allocation-free call's scratch array (noalloc.hip)
fock_status noalloc_setup(int device);
fock_status hip_fail(hipError_t e, const char* where);

// device allocation owned by the plan, grown on demand
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  fock_status ensure(size_t need, size_t cap, const char* what);
  void release();
};

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
inline bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}

// The k-points a pair sum runs over: targets X at ntk k-points, sources P and
// M (stored contiguously) at nsk k-points, and qidx[t][s] the kernel-table row
// of that (target, source) pair.
struct PairSet {
  int ntk = 0, nsk = 0;
  const int* qidx = nullptr;  // device [ntk][nsk]
};

struct Cell {
  Geom geom{};
  int nr = 0, nk = 0, nb = 0;
  double a[3][3]{}, vol = 0.0, omega = 0.0, gs = 2.0;
  std::vector<double> kpts;   // [nk][3]
  int nq = 0;                 // distinct q = k_t - k_s
  std::vector<int> qidx_host; // [nk][nk]
  DevBuf qidx, qvec, qzero;   // int[nk*nk], double[nq*3], int[nq]
  DevBuf K64;                 // double[nq][nr], 1/N_r folded, natural slot order
  DevBuf Kt;                  // float[nq][nr], fused-kernel layout (FP32 plans)
  DevBuf SD;                  // float[nq][nr/2][2], (S, D) pairs of the split 32^3 form (FP32 plans, n = 32)
  DevBuf Kt64;                // double[nq][nr], fused FP64 kernel layout (FP64-fused plans)
  bool f64f = false;          // this cell runs the fused FP64 kernel
  bool f32plain = false;      // an FP32-form cell on a grid that is not cubic: the plain stages in FP32
  DevBuf kvec;                // double[nk][3] k-points on the device
  // down-sampling: the source sub-mesh S (all k-points when ds is false)
  bool ds = false;
  std::vector<int> src;       // [nsrc] k indices of S
  int nsrc = 0;
  DevBuf qidx_ts, qidx_st;    // int[nk][nsrc] (target k, source s), int[nsrc][nk] (source s as target, k)
  // forward sums: all k-points as targets, S as sources
  PairSet fwd() const { return {nk, nsrc, (const int*)(ds ? qidx_ts.ptr : qidx.ptr)}; }
  // the reverse role of the adjoint: S as targets, all k-points as sources
  PairSet rev() const { return {nsrc, nk, (const int*)(ds ? qidx_st.ptr : qidx.ptr)}; }
};

// the batched form used when no tuned choice exists: the forked cells (three
// cells 16^3/27 k/8 b, 20^3/64 k/12 b, 24^3/125 k/16 b: 257.5 ms, against 261.8
// in sequence and 282.2 for the persistent kernel)
constexpr int kDefaultBatchForm = 1;

// state of the batched persistent launch (fock_apply_batched): buffers whose
// addresses a captured graph refers to, and the graph itself
struct BatchState {
  std::vector<const void*> key;  // u, phi, vphi pointers and nphi of every cell
  DevBuf shadow_u[kMaxBatchCells], shadow_x[kMaxBatchCells], comp[kMaxBatchCells];
  DevBuf accs, queue, counters;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  BatchArgs args{};
  int nthreads = 0, nwg = 0, entries = 0;
  // form 0: the persistent kernel; form 1: each cell's own fused kernel on a
  // stream of its own, forked from and joined to the caller's stream; form 2:
  // those kernels one after another, costliest cell first
  int form = kDefaultBatchForm;
  hipStream_t side[kMaxBatchCells] = {};
  hipEvent_t fork = nullptr, join[kMaxBatchCells] = {};
  bool ready = false;
  void reset_graph();
  void release();
};

// work arrays of the block eigensolver (eig_api.hip)
struct EigState {
  DevBuf x, hx, w, hw, p, hp, xn, hxn, pn, hpn;  // [nk][nb][N_r] blocks and their images under h
  DevBuf S, A, C, lam, status;                    // Rayleigh-Ritz matrices, coefficients, values, flags
  void release();
};

struct Plan {
  static constexpr unsigned kMagic = 0xF0C4C0DEu;
  unsigned magic = kMagic;
  fock_prec prec = FOCK_FP64;
  int device = 0;
  std::string tune_path;
  std::vector<Cell> cells;
  size_t workspace_cap = 0;                 // 0 = no cap (FOCKMI_WORKSPACE_CAP overrides)
  size_t batch_cap = size_t(16) << 30;      // plain path: bytes per pair batch
  int xcd_map = 1;
  DevBuf batch, shadow_x, shadow_p, shadow_m, comp, accs, vu, partial, dotres, srcbuf, srcout;
  DevBuf psi0, phiA, phiB, predb, srcbuf2, kin, vxb, lam, lam2, gtmp, ftmp, phis, norms, red6, vloc_buf;
  DevBuf sync;                              // lockstep counters of the persistent fused form
  DevBuf parts;                             // FP64 part sums of the lockstep form's k' split
  DevBuf xbuf, sflags, sstatus;             // exchange buffers, rendezvous counters, abort word of the split form
  DevBuf fallbacks;                         // split launches that fell back (counted while profiling)
  long split_wait_ticks = 5000000;          // rendezvous bound of the split form, 50 ms (FOCKMI_SPLIT_WAIT_TICKS)
  // pair symmetry of the split form: mirror copies (FP32 partial, FP64 sum, compensation),
  // their push counters, and the push order and counts for (nwg, nk, nb) = sym_key
  DevBuf mpart, msum, mcomp, mdone, sym_rank, sym_cnt;
  int sym_key[4] = {-1, -1, -1, -1};
  int split_stagger_shift = 1;              // the bands' order of the symmetric form (FOCKMI_SPLIT_STAGGER_SHIFT)
  int split_sym = 1;                        // 0: the split form runs every pair (FOCKMI_SPLIT_SYM=0)
  std::vector<double> host_norms;
  double* host_pinned = nullptr;            // 4 doubles for reductions
  bool profiling = false;
  // autotuning: the cache is read at plan creation when a path is given; missing
  // keys are measured on first use and the file is rewritten
  TuneCache tune;
  bool tuning = false;
  int use_graph = 1;
  BatchState bstate;
  EigState eig;
  int num_cus = 0;

  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
  double prof_ms = 0.0;
  long long prof_launches = 0;
  hipError_t prof_begin(hipStream_t st);
  hipError_t prof_end(hipStream_t st);
  fock_status prof_collect();

  fock_status init_cell(Cell& c, const fock_cell_desc& d, int index);
  fock_status check_ready(int cell) const;
  void destroy();

  // out[t][x] = (accumulate ? out : 0) + scale * sum_{s, b} M[s][b] W(P[s][b], X[t][x]; K_{qidx[t][s]})
  // over the targets and sources of ps
  fock_status general(Cell& c, const PairSet& ps, const c128* X, int nx, const c128* P, const c128* M, int ns,
                      c128* out, double scale, bool accumulate, hipStream_t st);
  fock_status run_plain(Cell& c, const PairSet& ps, const c128* X, int nx, const c128* P, const c128* M, int ns,
                        c128* out, double scale, bool accumulate, hipStream_t st);
  fock_status run_fused(Cell& c, const PairSet& ps, const c128* X, int nx, const c128* P, const c128* M, int ns,
                        c128* out, double scale, bool accumulate, hipStream_t st);
  fock_status run_fused64(Cell& c, const PairSet& ps, const c128* X, int nx, const c128* P, const c128* M,
                          int ns, c128* out, double scale, bool accumulate, hipStream_t st);
  // the orbitals of the source k-points, contiguous: `arr` itself without
  // down-sampling, else a copy of its S blocks ([nsrc][nper][nr]) in buf
  fock_status sources(Cell& c, const c128* arr, int nper, DevBuf& buf, hipStream_t st, const c128** out);
  // V_x[u] phi for the output k-points k0 .. k0 + nkout - 1 only (phi, out: those k-points)
  fock_status apply_krange(Cell& c, const c128* u, int k0, int nkout, const c128* phi, int nphi, c128* out,
                           hipStream_t st);
  // V_x[u] phi into out (forward sums over S, weight 1/|S|)
  fock_status apply_op(Cell& c, const c128* u, const c128* phi, int nphi, c128* out, hipStream_t st);
  fock_status shadow(DevBuf& buf, const c128* src, size_t count, const char* what, hipStream_t st,
                     const c64** out);
  // sum conj(a) b over count elements in FP64 (fixed order); synchronises st
  fock_status dot(const c128* a, const c128* b, size_t count, hipStream_t st, double* re, double* im);
  // the same sum as double-double: out = (re.hi, re.lo, im.hi, im.lo)
  fock_status dot_dd(const c128* a, const c128* b, size_t count, hipStream_t st, double out[4]);

  // propagator pieces (prop_api.hip)
  fock_status kinetic(Cell& c, const c128* x, int nf, c128* y, const double a[3], hipStream_t st);
  fock_status h_apply(Cell& c, const c128* us, const c128* us2, const c128* x, c128* out, const c128* base,
                      double cre, double cim, const double* vloc, const double a[3], double alpha, hipStream_t st);
  // acc <- x0 + sum_{m=1}^{order} phi_m, phi_m = (-i dt/m) h phi_{m-1}, phi_0 = x0 (acc may alias x0)
  fock_status taylor_sum(Cell& c, const c128* us, const c128* us2, const c128* x0, c128* acc, const double* vloc,
                         const double a[3], double dt, double alpha, int order, hipStream_t st);
  // max over (k, b) of |(Omega/N_r) ||psi_kb||^2 - 1|; synchronises st
  fock_status norm_dev(Cell& c, const c128* psi, hipStream_t st, double* dev);
  fock_status field_bufs(Cell& c, std::initializer_list<DevBuf*> bufs, int nfields_per_k);

  // eigenstates of h (Eq. (25)) and the excited-electron density (Eq. (26)) (eig_api.hip)
  fock_status eigensolve(Cell& c, const c128* u, c128* phi, const double* vloc, const double a[3], double alpha,
                         double tol, int maxit, double* eig_host, double* res_host, int* iters_host, hipStream_t st);
  fock_status excited_density(Cell& c, const c128* phi, const c128* psi, hipStream_t st, double* nex);

  // batched persistent launch (batched.hip)
  fock_status run_batched(const void* const* u, const void* const* phi, const int* nphi, void* const* vphi,
                          hipStream_t st);
  std::string key_for(const Cell& c, const PairSet& ps, int nx, const char* what) const;
  void save_tune();
};

}  // namespace fockmi
