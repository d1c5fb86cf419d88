// Launchers of the device kernels (host-callable, stream-ordered).
// Every launcher returns the hipError_t of its launch.
#pragma once

#include <hip/hip_runtime.h>
#include <vector>

#include "fft_reg.hpp"

namespace fockmi {

using c64 = cx<float>;
using c128 = cx<double>;

struct Geom {
  int n1, n2, n3;
  double B[3][3];  // reciprocal rows b_d
};

// ---- kernel tables -------------------------------------------------------
// K[q][l] = scale * Nyquist-averaged v(qvec[q] + G_l) for q < nq, natural slot order.
hipError_t launch_build_table_f64(double* K, const double* qvec, const int* qzero, int nq, const Geom& g,
                                  double omega, double scale, hipStream_t st);
// Fused-layout FP32 copy for a cubic grid of length n (value index l3, thread t).
hipError_t launch_build_table_fused(float* Kt, const double* K, int nq, int n, hipStream_t st);

// ---- plain path (complex128 batches for FP64, complex64 for the FP32 form on non-cubic grids)
// A batch holds the pairs of ntb target k-points (kt0 ..) and nkb source k-points (ks0 ..):
// pair p = ((tb*nkb + kb)*nb + j)*nx + s, each a field of nr values. T is double or float.
// batch[p][r] = conj(P[ks0+kb][j][r]) * X[kt0+tb][s][r] (inputs rounded to T)
template <typename T>
hipError_t launch_pair_product(cx<T>* batch, const c128* X, const c128* P, int kt0, int ntb, int ks0, int nkb, int nb,
                               int nx, int nr, hipStream_t st);
// in-place 3D FFT of nfields fields of shape n1 x n2 x n3 (sign -1 forward, +1 inverse, unnormalised)
template <typename T>
hipError_t launch_fft3_plain(cx<T>* data, int nfields, const Geom& g, int sign, hipStream_t st);
// batch[p][l] *= K[qidx[(kt0+tb)*nk + ks0+kb]][l]
template <typename T>
hipError_t launch_kernel_mul(cx<T>* batch, const double* K, const int* qidx, int kt0, int ntb, int nk, int ks0,
                             int nkb, int per_kb, int nr, hipStream_t st);
// out[kt0+tb][s][r] = (accumulate ? out : 0) + scale * sum_{kb,j} M[ks0+kb][j][r] * batch[((tb*nkb+kb)*nb+j)*nx+s][r]
// (FP64 products and sums)
template <typename T>
hipError_t launch_mac(c128* out, const cx<T>* batch, const c128* M, int kt0, int ntb, int ks0, int nkb, int nb, int nx,
                      int nr, double scale, int accumulate, hipStream_t st);

// ---- fused FP32 path -----------------------------------------------------
struct FusedArgs {
  const c64* X;       // [nk][nx][nr] targets
  const c64* P;       // [nk][nb][nr] conjugated in the pair density
  const c64* M;       // [nk][nb][nr] multiplier
  const float* Kt;    // [nq][nr] fused layout, 1/N_r folded
  const int* qidx;    // [nk][nk] table of (target k, source k')
  c128* out;          // [nk][nx][nr] FP64 result (running sum)
  c64* comp;          // [nk][nx][nr] Neumaier compensation of out, rounded to FP32
  c64* accs;          // per-workgroup FP32 partial sums when they do not fit in registers
  int nk, nx, nb;
  int item0, nitems;  // work items [item0, item0 + nitems) of nk*nx
  double scale;       // -1/N_k
  int accumulate;     // 1: add to the existing out
  int xcd_map;        // 1: map workgroups so that one XCD runs the targets of one k
  int n;              // grid length of this cell (batched launch)
  // k' split of the lockstep form (1 elsewhere): target t's sum runs as ksplit
  // parts over equal k' ranges; part 0 writes out, part p > 0 writes FP64 field
  // part_out[p-1][t] (t < nitems, item0 = 0), and comp holds ksplit fields per target
  int ksplit;
  c128* part_out;
  // when not NULL, the lockstep form (and its part combine) runs only if *gate != 0:
  // the fallback of the split 32^3 kernel, launched behind it on the same stream
  const int* gate;
};
// Persistent lockstep form of the fused kernel, for grid lengths whose FP32
// partial sums live in global memory: nwg workgroups (a multiple of 8, at most
// one per CU) keep pace with the other workgroups of their XCD pair by pair.
// counters: kLockstepInts ints of caller-owned device memory, cleared by the
// launch.
constexpr int kLockstepStride = 32;  // ints between the XCD counters (128 bytes)
constexpr int kLockstepInts = 8 * kLockstepStride;
struct LockstepCfg {
  int* counters;
  int nwg;
};
bool fused_has_lockstep(int n);
int fused_default_variant(int n);  // the variant used when no tuned choice exists
// n in {16, 20, 24, 32}; variant < fused_variants(n) selects the register/occupancy
// target, or (the last variant where fused_has_lockstep(n)) the lockstep form, which needs ls
hipError_t launch_fused_apply(int n, const FusedArgs& a, hipStream_t st, int variant = 0,
                              const LockstepCfg* ls = nullptr);
int fused_variants(int n);
size_t fused_acc_scratch_elems(int n, int nslots);  // c64 elements needed in accs (0 if registers)

// Split 32^3 form (split32.hip): each target on two workgroups of one XCD,
// nwg workgroups (a multiple of 16, at most one per CU), accumulate = 0 only.
// On a timed-out rendezvous or an XCD mismatch the launch stops and leaves
// status[0] != 0; the caller then runs the lockstep form gated on status.
struct SplitArgs {
  FusedArgs f;          // X, P, M, qidx, out, comp, nk, nx, nb, nitems, scale (accumulate must be 0)
  const float* SD;      // [nq][16384][2]: (S, D) = K(l1') +- K(l1' + 16) at (l2 * 512 + 32 l1' + l3), 1/N_r folded
  c64* xbuf;            // [nwg/2 pairs][2 halves][16384] exchange mailboxes
  int* flags;           // split32_flag_ints(nwg) ints: rendezvous counters, then XCD ids
  int* status;          // [0] abort word, cleared by the launch
  long wait_ticks;      // bound of one rendezvous wait (100 MHz ticks); < 0 stops the launch at once
  // Pair symmetry (sym = 1; the targets are the sources u over the whole k mesh, nx = nb):
  // target (k, i) runs the source k-points k + d mod nk, d = 0 .. nk/2 (ndelta blocks of nb
  // bands), and for 1 <= d <= npush = (nk - 1)/2 it also adds conj(W) u_(k,i) to the mirror
  // copy of source (k + d, j): the term of target (k + d, j) from source (k, i).
  int sym;
  int ndelta, npush;
  int stagger_shift;    // target (k, i) takes the bands of a source k-point in the order j = (i >> shift) + m mod nb
  const int* rank;      // [nitems][ndelta * nb]: a push's place in its mirror copy's order
  c64* mpart;           // [8][nitems][32768] FP32 partial sums of the mirror copies (one per XCD)
  c128* msum;           // [8][nitems][32768] their FP64 running sums
  c64* mcomp;           // [8][nitems][32768] and the Neumaier compensation, rounded to FP32
  int* mdone;           // split32_mirror_ctr_ints(nitems) counters, cleared by the launch
};
size_t split32_flag_ints(int nwg);
size_t split32_xbuf_elems(int nwg);   // c64 elements
size_t split32_sd_floats(int nq);
size_t split32_mirror_ctr_ints(int nitems);
// The order of the pushes into every mirror copy (rank, [nitems][ndelta*nb], -1 where a
// pair pushes nothing) and the pushes each copy receives (cnt, [8][nitems]), for nwg
// workgroups, nk k-points and nb bands.
void split32_sym_tables(int nwg, int nk, int nb, int shift, std::vector<int>* rank, std::vector<int>* cnt);
hipError_t launch_build_sd32(float* SD, const double* K, int nq, hipStream_t st);
hipError_t launch_split32(const SplitArgs& s, int nwg, hipStream_t st);
// out[b] += the mirror copies of target b (FP64 sum + compensation + scale * FP32 partial,
// copies in XCD order); does nothing when status[0] != 0
hipError_t launch_split32_sym_combine(c128* out, const c128* msum, const c64* mcomp, const c64* mpart,
                                      const int* cnt, int nitems, double scale, const int* status,
                                      hipStream_t st);
// count[0] += (status[0] != 0); p[0] = 0 (diagnostics of the split form's fallbacks)
hipError_t launch_count_abort(long long* count, const int* status, hipStream_t st);
hipError_t launch_zero_ll(long long* p, hipStream_t st);

// ---- fused FP64 form -------------------------------------------------------
struct Fused64Args {
  const c128* X;      // [ntk][nx][nr] targets
  const c128* P;      // [nk][nb][nr] conjugated in the pair density (sources)
  const c128* M;      // [nk][nb][nr] multiplier (sources)
  const double* Kt;   // [nq][nr] fused layout (FP64 transposes), 1/N_r folded
  const int* qidx;    // [ntk][nk] table row of (target k, source k')
  c128* out;          // [ntk][nx][nr] result
  c128* accs;         // per-workgroup FP64 sums when they do not fit in registers
  int nk, nx, nb;     // sources, targets per k, bands per source
  int item0, nitems;  // work items [item0, item0 + nitems) of ntk*nx
  double scale;       // e.g. -1/|S|
  int accumulate;     // 1: add to the existing out
  int xcd_map;
};
bool fused64_supported(int n);                        // cubic grid lengths with a fused FP64 kernel
int fused64_phases(int n);                            // rounds of the x<->y transpose (table layout)
size_t fused64_acc_scratch_elems(int n, int nslots);  // c128 elements needed in accs (0 if registers)
hipError_t launch_fused64_apply(int n, const Fused64Args& a, hipStream_t st);
// FP64 copy of the tables in the fused FP64 kernel's layout (nph rounds)
hipError_t launch_build_table_fused64(double* Kt, const double* K, int nq, int n, int nph, hipStream_t st);

// Persistent launch over several cells: nwg workgroups of nthreads pop entries
// (queue[3i] = cell, queue[3i+1] = target item, queue[3i+2] = a second target
// of the same 16^3 cell or -1) from kBatchQueues sub-queues; sub-queue x holds
// entries [qoff[x], qoff[x] + qlen[x]) and is counted by counters[x].
constexpr int kMaxBatchCells = 8;
constexpr int kBatchQueues = 8;  // one per XCD
struct BatchArgs {
  FusedArgs cells[kMaxBatchCells];
  const int* queue;
  int* counters;
  int qoff[kBatchQueues];
  int qlen[kBatchQueues];
};
int batched_threads(int nmax);  // workgroup size for a batch whose largest grid length is nmax (0: none)
hipError_t launch_fused_batched(const BatchArgs& b, int nthreads, int nwg, hipStream_t st);

// ---- helpers ---------------------------------------------------------------
hipError_t launch_to_c64(c64* dst, const c128* src, long count, hipStream_t st);
// partial[4b..4b+3] for b < nblk, then dst[0..3] = sum conj(a) b as double-double
// (re.hi, re.lo, im.hi, im.lo), fixed order
hipError_t launch_dot(double* dst, double* partial, int nblk, const c128* a, const c128* b, long count,
                      hipStream_t st);
hipError_t launch_scale_add(c128* y, const c128* x, double sre, double sim, long count, hipStream_t st);
// y[i] = 0 for i < count (a kernel, so that it can sit in a captured graph)
hipError_t launch_zero(c128* y, long count, hipStream_t st);

}  // namespace fockmi
