// Fused FP32 pair kernel: every step of Eq. (15) for one pair without leaving the CU.
//
// One workgroup owns one target field X[kt][s] and runs over all sources
// (k', j). For each pair it forms rho = conj(P_jk') X (the pair density), does
// the forward 3D FFT, multiplies by K_{kt-k'} (1/N_r folded into the table),
// does the inverse FFT and accumulates M_jk' * W. The band sum over j is kept
// in FP32 (in registers for N <= 24; for N = 32, whose working field alone
// fills half the register file, in a per-workgroup global buffer); after every
// 16 bands and at the end of every k' the FP32 partial sum is added to an FP64
// running sum with Neumaier compensation (the compensation term stored in
// FP32), and the final FP64 value is s + c.
//
// At N = 32 a persistent form runs one workgroup per CU and keeps the
// workgroups of each XCD in step pair by pair (fused_lockstep_kernel), so that
// the sources they all read in the same order come from L2.
//
// Layout on chip, cubic grid of length N, N*N threads:
//   x phase : thread holds the line along n1 at fixed (m2, m3) -> global loads
//             and stores of neighbouring lanes hit neighbouring addresses;
//   y phase : the line along n2 at fixed (l1, m3);
//   z phase : the line along n3 at fixed (l1, l2), where the kernel multiply
//             happens (the table is stored in this layout, value-major).
// Each phase transforms its line in registers (fft_reg.hpp); LDS only carries
// the transposes between phases. When a full complex64 field does not fit in
// LDS (N = 32), each transpose runs in two rounds over half of the field, with
// the thread map arranged so that a thread never holds two lines at once.
#include "fused_common.hpp"

namespace fockmi {

template <int N>
constexpr int fused_nph() {
  return ((long)N * N * (N + 1) * 8 > 160L * 1024) ? 2 : 1;
}

int fused_phases(int n) {
  switch (n) {
    case 16: return fused_nph<16>();
    case 20: return fused_nph<20>();
    case 24: return fused_nph<24>();
    case 32: return fused_nph<32>();
    default: return 1;
  }
}

template <int N>
constexpr bool fused_acc_in_regs() {
  return N <= 24;
}

// The target X is loaded once per work item and held in registers (N values per
// thread) where they fit; otherwise it is re-read with every pair's density. At
// 16^3 the kernel keeps four waves per SIMD with X in registers (127 VGPRs), and
// the X re-reads, one private field per workgroup and pair, had filled the L2
// (the paper's down-sampled 16^3 setting: 386.5 -> 242.6 ms). At 20^3 the four-wave
// variant spills and the two-wave one loses a workgroup per CU; at 24^3 the line
// leaves no room.
template <int N>
constexpr bool fused_x_in_regs() {
  return N == 16;
}

// Global loads are issued in groups whose results are consumed only after the
// whole group is in flight, so a pair costs a few memory round trips instead
// of one per line element. Group sizes per grid length: pair-product operands,
// kernel values, multipliers (0: element by element, where the registers are
// full, as for N = 32 whose multiplier loads would spill). At N = 32 the
// pair-product operands go in two groups of 16: one group of 32 (128 VGPRs of
// load results) pushed the allocator into spills that cost more than the
// second round trip.
template <int N>
constexpr int grp_px() { return N == 16 ? 8 : (N <= 24 ? 4 : 16); }
template <int N>
constexpr int grp_k() { return N <= 24 ? N : 8; }
template <int N>
constexpr int grp_m() { return N == 16 ? 8 : (N <= 24 ? 4 : 0); }
// Elements whose loads run ahead of their use in the FP64 flush. Element by element, each
// element's loads would wait behind the previous element's stores (the compiler cannot tell
// the buffers apart): loading 4 ahead took the 24^3 / 64 k / 16-band application from 50.6
// to 50.0 ms and the three-cell batch from 230.7 to 228.4 ms, with the same bits.
template <int N>
constexpr int flush_depth() { return 4; }

// bands per FP32 partial sum before it is folded into the FP64 running sum: the
// FP32 rounding of the band sum stays that of at most 16 terms for any band count
constexpr int kBandFlush = 16;

template <int N>
constexpr int fused_lds_elems() {
  constexpr int NPH = fused_nph<N>();
  constexpr int H = N / NPH, NBK = N / NPH;
  constexpr int A = N * N * H, B = NBK * N * (N + 1);
  return A > B ? A : B;
}

namespace {

// s + c += x, with the rounding error of each addition carried in c. The
// error terms are exact only if every operation rounds on its own: no
// contraction into FMAs here or where x is formed.
__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
#pragma clang fp contract(off)
  const double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

// Pair hooks: called by every thread at the start of each pair of a work item,
// p = (k' - first k' of the item) * nb + j, before the pair's loads.
struct NoPairHook {
  __device__ __forceinline__ void operator()(int) {}
};

// Soft lockstep of the workgroups of one XCD (persistent launch). Before every
// kLockstepPeriod-th pair of its item a workgroup counts itself in on its XCD's
// counter and waits until every workgroup of the XCD that has an item in this
// round has arrived at the same pair. All of them read the sources in the same (k', j) order, so the source
// orbitals (and, for targets of one k, the kernel values) then come from L2
// once per XCD instead of once per workgroup. The wait is bounded: after
// kLockstepPolls polls thread 0 stops taking part, and its peers stop at their
// next wait, so the result never depends on the counter, only the speed does.
// The state lives in LDS (thread 0 alone touches it), so it holds no registers
// across the pair.
constexpr int kLockstepPolls = 4096;
// pairs between waits: pacing every pair cost more in barriers and polls than
// it kept in L2 (C2: 2.47 s every pair, 2.30 s every 4th, 2.27 s every 8th,
// 2.32 s every 16th, 2.56 s never)
constexpr int kLockstepPeriod = 8;
struct LockstepState {
  int* cnt;     // this XCD's arrival counter (zero at launch)
  int target;   // arrivals of the XCD's workgroups up to and including this pair
  int part;     // workgroups of the XCD with an item in this round
  int live;     // 0 once a wait has timed out
};
struct XcdLockstep {
  LockstepState* st;  // in LDS
  __device__ __forceinline__ void operator()(int pair) {
    if (pair % kLockstepPeriod != 0) return;  // uniform: every thread passes the same pair
    if (threadIdx.x == 0 && st->live) {
      int* cnt = st->cnt;
      __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int target = st->target + st->part;
      st->target = target;
      int n = 0;
      while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++n > kLockstepPolls) {
          st->live = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __syncthreads();
  }
};

// One work item (target field X[kt][s]) of the fused pair computation, run by
// the N*N threads t = 0 .. N*N-1 of one thread group, with `lds` its own LDS
// region. Twin threads (twin = true) run the code of thread t of a real group
// (the same global loads, which keeps every wave on the same straight-line
// code) in an LDS region of their own, so their values are meaningless; their
// FP64 stores are steered past the end of the buffer, where raw buffer stores
// are dropped. `item` must be uniform over each wave.
template <int N, class Hook>
__device__ __forceinline__ void fused_item(const FusedArgs& a, int item, int acc_slot, c64* __restrict__ lds,
                                           int t, bool twin, Hook& hook, int part = 0) {
  constexpr int NTI = N * N;
  constexpr int NR = N * N * N;
  constexpr int NPH = fused_nph<N>();
  constexpr int H = N / NPH;       // width of one round of the x<->y transpose (along m3)
  constexpr int TPG = NTI / NPH;   // threads per round
  constexpr int NBK = N / NPH;     // l1 values per round of the y<->z transpose
  constexpr bool ACCREG = fused_acc_in_regs<N>();
  constexpr bool XREG = fused_x_in_regs<N>();
  item = __builtin_amdgcn_readfirstlane(item);
  // round indices are wave-uniform (rounds are whole waves: 512 and 256 threads
  // at N = 32, a single round below); readfirstlane lets the compiler branch on
  // them instead of masking lanes
  static_assert(NPH == 1 || (TPG % 64 == 0 && (NBK * H) % 64 == 0), "rounds must be whole waves");
  const int grp = __builtin_amdgcn_readfirstlane(t / TPG);
  const int tl = t % TPG;
  const int hl = tl % H;
  const int clo = hl + H * grp;  // m3 in the x and y phases, l2 in the z phase
  const int chi = tl / H;        // m2 in the x phase, l1 in the y and z phases
  const int gyz = __builtin_amdgcn_readfirstlane(chi / NBK);  // round of the y<->z transpose
  const int lrow = chi % NBK;

  // LDS byte offsets of this thread's elements in the four transposes:
  //   x side of x<->y : element l1 at lx + l1 * SX
  //   y side of x<->y : element m2 at ly + m2 * SY
  //   y side of y<->z : element l2 at lyz + l2 * (N+1)*8
  //   z side of y<->z : element m3 at lz + m3 * 8
  // With one round (N <= 24) both transposes use one array [l1][m2 or l2][m3]
  // with rows padded to N+1 (SX = N*(N+1)*8, SY = (N+1)*8, and ly = lyz): every
  // phase then writes its values back to the slots it read, a slot is rewritten
  // only by the thread that last read it, and each transpose needs one barrier
  // (twins must therefore work in an LDS region of their own). With two rounds
  // (N = 32) the x<->y array is [l1][m2][m3 of the round]
  // (SX = N*H*8, SY = H*8) and the rounds share it, so each transpose keeps a
  // second barrier before the next round overwrites it. Only the x side spans
  // more than 64 KiB; its elements from L1S on are addressed from a second base.
  constexpr bool INPLACE = NPH == 1;
  constexpr unsigned SX = INPLACE ? (unsigned)(N * (N + 1) * 8) : (unsigned)(N * H * 8);
  constexpr unsigned SY = INPLACE ? (unsigned)((N + 1) * 8) : (unsigned)(H * 8);
  constexpr int L1S = (int)((65535u / SX) + 1) < N ? (int)((65535u / SX) + 1) : N;
  const unsigned lx0 = INPLACE ? (unsigned)((chi * (N + 1) + hl) * 8) : (unsigned)((chi * H + hl) * 8);
  const unsigned ly0 = INPLACE ? (unsigned)((chi * N * (N + 1) + hl) * 8) : (unsigned)((chi * N * H + hl) * 8);
  const unsigned lyz0 = (unsigned)((lrow * N * (N + 1) + clo) * 8);
  const unsigned lz0 = (unsigned)((lrow * N + clo) * (N + 1) * 8);

  const int kt = item / a.nx;
  const int s = item % a.nx;

  // byte offsets: x-phase element (m1, m2=chi, m3=clo) is at voff_x + m1 * N*N*8;
  // table and FP32 partial sums are value-major: (v, t) at (v * NTI + t) * size
  const unsigned voff_x = (unsigned)((chi * N + clo) * 8);
  const unsigned voff_f = twin ? 0xF0000000u : 2u * voff_x;  // FP64 stores of twins are dropped
  const unsigned voff_c = twin ? 0xF0000000u : voff_x;        // so are their compensation stores
  const unsigned voff_t4 = (unsigned)(t * 4);
  const unsigned voff_t8 = (unsigned)(t * 8);
  constexpr unsigned FB64 = NR * 8u;  // bytes of one complex64 field
  constexpr unsigned FB128 = NR * 16u;

  // this part's k' range and output (one part, the whole sum, unless split)
  const long tgt = (long)kt * a.nx + s;
  const int nkp = a.ksplit > 1 ? a.nk / a.ksplit : a.nk;
  const int ks0 = part * nkp, ks1 = ks0 + nkp;
  const int accumulate = part == 0 ? a.accumulate : 0;
  c128* const outp = part == 0 ? a.out + tgt * NR : a.part_out + ((long)(part - 1) * a.nitems + tgt) * NR;

  const rsrc_t rX = make_rsrc(a.X + tgt * NR, FB64);
  const rsrc_t rOut = make_rsrc(outp, FB128);
  const rsrc_t rComp = make_rsrc(a.comp + ((long)part * a.nitems + tgt) * NR, FB64);
  const rsrc_t rAcc = make_rsrc(ACCREG ? a.X : a.accs + (long)acc_slot * NR, ACCREG ? 0u : FB64);

  c64 acc[ACCREG ? N : 1];
  c64 xr[XREG ? N : 1];
  if constexpr (XREG) static_for<N>([&](auto m1) { xr[m1] = ld_c64(rX, voff_x, (unsigned)(decltype(m1)::value * NTI * 8)); });

  for (int ks = ks0; ks < ks1; ++ks) {
    const int qi = __builtin_amdgcn_readfirstlane(a.qidx[kt * a.nk + ks]);
    const rsrc_t rK = make_rsrc(a.Kt + (long)qi * NR, NR * 4u);
    const bool first_ks = (ks == ks0);
    const bool last_ks = (ks == ks1 - 1);
    for (int j = 0; j < a.nb; ++j) {
      // the FP32 band sum runs over at most kBandFlush bands before it is folded
      // into the FP64 sum (every kBandFlush-th band and the last band of each k')
      const bool group_start = j % kBandFlush == 0;
      if constexpr (ACCREG) {
        if (group_start) static_for<N>([&](auto m) { acc[decltype(m)::value] = c64{0.0f, 0.0f}; });
      }
      hook((ks - ks0) * a.nb + j);
      const rsrc_t rP = make_rsrc(a.P + ((long)ks * a.nb + j) * NR, FB64);
      const rsrc_t rM = make_rsrc(a.M + ((long)ks * a.nb + j) * NR, FB64);
      c64 v[N];
      static_for<(N + grp_px<N>() - 1) / grp_px<N>()>([&](auto cc) {
        constexpr int G = grp_px<N>(), C0 = decltype(cc)::value * G, CN = (N - C0 < G) ? N - C0 : G;
        c64 p[CN], x[CN];
        static_for<CN>([&](auto q) {
          const unsigned so = (unsigned)((C0 + decltype(q)::value) * NTI * 8);
          p[q] = ld_c64(rP, voff_x, so);
          if constexpr (XREG) x[q] = xr[C0 + decltype(q)::value];
          else x[q] = ld_c64(rX, voff_x, so);
        });
        __builtin_amdgcn_sched_barrier(0);
        static_for<CN>([&](auto q) { v[C0 + decltype(q)::value] = cmulc(p[q], x[q]); });
      });
      fft<N, -1>(v);
      // x -> y
#pragma unroll
      for (int g = 0; g < NPH; ++g) {
        if (grp == g) {
          const unsigned b0 = opaque(lx0), b1 = opaque(lx0 + L1S * SX);
          static_for<N>([&](auto l1) {
            constexpr int L = decltype(l1)::value;
            if constexpr (L < L1S) lds_at<L * SX>(lds, b0) = v[L];
            else lds_at<(L - L1S) * SX>(lds, b1) = v[L];
          });
        }
        __syncthreads();
        if (grp == g) {
          const unsigned b = opaque(ly0);
          static_for<N>([&](auto m2) { v[m2] = lds_at<decltype(m2)::value * SY>(lds, b); });
        }
        if constexpr (!INPLACE) __syncthreads();
      }
      fft<N, -1>(v);
      // y -> z
#pragma unroll
      for (int g = 0; g < NPH; ++g) {
        if (gyz == g) {
          const unsigned b = opaque(lyz0);
          static_for<N>([&](auto l2) { lds_at<decltype(l2)::value * (N + 1) * 8>(lds, b) = v[l2]; });
        }
        __syncthreads();
        if (gyz == g) {
          const unsigned b = opaque(lz0);
          static_for<N>([&](auto m3) { v[m3] = lds_at<decltype(m3)::value * 8>(lds, b); });
        }
        if constexpr (!INPLACE) __syncthreads();
      }
      fft<N, -1>(v);
      static_for<(N + grp_k<N>() - 1) / grp_k<N>()>([&](auto cc) {
        constexpr int G = grp_k<N>(), C0 = decltype(cc)::value * G, CN = (N - C0 < G) ? N - C0 : G;
        float kv[CN];
        static_for<CN>([&](auto q) { kv[q] = ld_f32(rK, voff_t4, (unsigned)((C0 + decltype(q)::value) * NTI * 4)); });
        __builtin_amdgcn_sched_barrier(0);
        static_for<CN>([&](auto q) { v[C0 + decltype(q)::value] = cscale(v[C0 + decltype(q)::value], kv[q]); });
      });
      fft<N, +1>(v);
      // z -> y
#pragma unroll
      for (int g = 0; g < NPH; ++g) {
        if (gyz == g) {
          const unsigned b = opaque(lz0);
          static_for<N>([&](auto m3) { lds_at<decltype(m3)::value * 8>(lds, b) = v[m3]; });
        }
        __syncthreads();
        if (gyz == g) {
          const unsigned b = opaque(lyz0);
          static_for<N>([&](auto l2) { v[l2] = lds_at<decltype(l2)::value * (N + 1) * 8>(lds, b); });
        }
        if constexpr (!INPLACE) __syncthreads();
      }
      fft<N, +1>(v);
      // y -> x
#pragma unroll
      for (int g = 0; g < NPH; ++g) {
        if (grp == g) {
          const unsigned b = opaque(ly0);
          static_for<N>([&](auto m2) { lds_at<decltype(m2)::value * SY>(lds, b) = v[m2]; });
        }
        __syncthreads();
        if (grp == g) {
          const unsigned b0 = opaque(lx0), b1 = opaque(lx0 + L1S * SX);
          static_for<N>([&](auto l1) {
            constexpr int L = decltype(l1)::value;
            if constexpr (L < L1S) v[L] = lds_at<L * SX>(lds, b0);
            else v[L] = lds_at<(L - L1S) * SX>(lds, b1);
          });
        }
        if constexpr (!INPLACE) __syncthreads();
      }
      fft<N, +1>(v);

      const bool last_j = (j == a.nb - 1);
      const bool flush = last_j || (j + 1) % kBandFlush == 0;
      const bool first_fl = first_ks && j < kBandFlush;  // this target's first fold into FP64
      const bool last_fl = last_ks && last_j;            // and its last
      if constexpr (ACCREG) {
        static_assert(N % grp_m<N>() == 0, "multiplier groups must tile the line");
        static_for<N / grp_m<N>()>([&](auto cc) {
          constexpr int G = grp_m<N>(), C0 = decltype(cc)::value * G;
          c64 mv[G];
          static_for<G>([&](auto q) { mv[q] = ld_c64(rM, voff_x, (unsigned)((C0 + decltype(q)::value) * NTI * 8)); });
          __builtin_amdgcn_sched_barrier(0);
          static_for<G>([&](auto q) {
            constexpr int m1 = C0 + decltype(q)::value;
            acc[m1] = cmac(acc[m1], mv[q], v[m1]);
            v[m1] = acc[m1];
          });
        });
      } else {
        // the position of j in the band loop is uniform: one branch per pair
        // selects the accumulator traffic, none per element. The loads go
        // element by element: with the line in registers, loading ahead (in
        // groups, or a few elements in flight) made the allocator spill more
        // than the overlap gained.
        auto mac = [&](auto load_acc, auto store_acc) {
#pragma unroll
          for (int m1 = 0; m1 < N; ++m1) {
            const unsigned so = (unsigned)(m1 * NTI * 8);
            c64 tot = cmul(ld_c64(rM, voff_x, so), v[m1]);
            if constexpr (decltype(load_acc)::value) tot = ld_c64(rAcc, voff_t8, so) + tot;
            if constexpr (decltype(store_acc)::value) st_c64(tot, rAcc, voff_t8, so);
            v[m1] = tot;
          }
        };
        using T = std::true_type;
        using F = std::false_type;
        if (group_start) {
          if (flush) mac(F{}, F{});
          else mac(F{}, T{});
        } else {
          if (flush) mac(T{}, F{});
          else mac(T{}, T{});
        }
      }
      if (flush) {
#pragma clang fp contract(off)
        // fold the FP32 band sum into the FP64 running sum
        // every element is loaded and stored unconditionally (the buffers are
        // whole fields) and the uniform flags only select values, so the loop
        // is straight-line code whose loads run ahead of their use
        const bool use_out = !first_fl || accumulate;
        const bool use_comp = !first_fl;
        constexpr int D = flush_depth<N>();
        c128 oq[D];
        c64 cq[D];
        auto issue = [&](auto m) {
          constexpr int m1 = decltype(m)::value;
          constexpr unsigned so = (unsigned)(m1 * NTI * 16);
          oq[m1 % D] = ld_c128(rOut, voff_f, so);
          cq[m1 % D] = ld_c64(rComp, voff_c, so / 2);
        };
        static_for<D>([&](auto m) { issue(m); });
        static_for<N>([&](auto m) {
          constexpr int m1 = decltype(m)::value;
          constexpr unsigned so = (unsigned)(m1 * NTI * 16);
          const double xr = a.scale * (double)v[m1].re;
          const double xi = a.scale * (double)v[m1].im;
          double sr = use_out ? oq[m1 % D].re : 0.0;
          double si = use_out ? oq[m1 % D].im : 0.0;
          double cr = use_comp ? (double)cq[m1 % D].re : 0.0;
          double ci = use_comp ? (double)cq[m1 % D].im : 0.0;
          if constexpr (m1 + D < N) issue(std::integral_constant<int, m1 + D>{});
          neumaier(sr, cr, xr);
          neumaier(si, ci, xi);
          // the final value is s + c; before it, s and the compensation (a
          // rounding-error term ~1e-16 |s|, which FP32 keeps)
          st_c128(last_fl ? c128{sr + cr, si + ci} : c128{sr, si}, rOut, voff_f, so);
          st_c64(c64{(float)cr, (float)ci}, rComp, voff_c, so / 2);
        });
      }
    }
  }
}

// one workgroup per target; WPE is the waves-per-SIMD target given to the
// register allocator (a tunable: more waves, or more registers per wave)
template <int N, int WPE>
__global__ void __launch_bounds__(N * N) __attribute__((amdgpu_waves_per_eu(WPE)))
fused_apply_kernel(FusedArgs a) {
  __shared__ c64 lds[fused_lds_elems<N>()];
  int b = blockIdx.x;
  if (a.xcd_map) {
    // workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of targets so that workgroups sharing an L2 share k and K_q
    const int nwg = gridDim.x;
    const int q = nwg / 8, rem = nwg % 8;
    const int x = b % 8, r = b / 8;
    b = x * q + (x < rem ? x : rem) + r;
  }
  NoPairHook nh;
  fused_item<N>(a, a.item0 + b, blockIdx.x, lds, threadIdx.x, false, nh);
}

// Persistent form: gridDim.x = 8 * W workgroups, one per CU, W per XCD
// (workgroups are dispatched round-robin over the XCDs, so workgroup b runs on
// XCD b % 8). In round r, the workgroups of XCD x take the W consecutive items
// from r * 8W + x * W, so that an XCD holds the targets of whole k-points, and
// keep in soft lockstep pair by pair (XcdLockstep). Workgroup b owns FP32
// partial-sum slot b.
template <int N, int WPE>
__global__ void __launch_bounds__(N * N) __attribute__((amdgpu_waves_per_eu(WPE)))
fused_lockstep_kernel(FusedArgs a, int* counters) {
  __shared__ c64 lds[fused_lds_elems<N>()];
  __shared__ LockstepState st;
  if (a.gate && *a.gate == 0) return;  // a fallback whose primary launch completed
  const int G = gridDim.x, W = G / 8;
  const int x = blockIdx.x % 8, rank = x * W + blockIdx.x / 8;
  if (threadIdx.x == 0) {
    st.cnt = counters + x * kLockstepStride;
    st.target = 0;
    st.live = 1;
  }
  XcdLockstep hook{&st};
  // work items q = part * nitems + target: equal k' ranges, so that the
  // workgroups of one XCD-round all run the same number of pairs
  const int h = a.ksplit > 1 ? a.ksplit : 1;
  const int total = a.nitems * h;
  for (int r = 0; r * G + rank < total; ++r) {
    const int q = r * G + rank;
    const int left = total - r * G - x * W;
    if (threadIdx.x == 0) st.part = left < W ? left : W;
    // the first pair's wait orders this write before every use
    fused_item<N>(a, a.item0 + q % a.nitems, blockIdx.x, lds, threadIdx.x, false, hook, q / a.nitems);
  }
}

// out[i] += sum_{p < nparts} parts[p][i], in that order
__global__ void add_parts_kernel(c128* __restrict__ out, const c128* __restrict__ parts, int nparts, long count,
                                 const int* gate) {
  if (gate && *gate == 0) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    c128 v = out[i];
    for (int p = 0; p < nparts; ++p) {
      v.re += parts[(long)p * count + i].re;
      v.im += parts[(long)p * count + i].im;
    }
    out[i] = v;
  }
}

// Persistent workgroups of NT threads pop queue entries (cell, target, second
// target or -1) until every sub-queue is empty. Each XCD has a sub-queue of its
// own (a contiguous share of every cell's targets, so that targets sharing k and
// K_q meet in one L2) and moves on to the other sub-queues when it runs dry.
// An entry runs the code of its cell's grid length: 24^3 on all 576 threads,
// 20^3 on 400 (the rest are twins), and 16^3 on two groups of 256 threads, one
// target each with its own LDS region (a single target leaves the second group
// to twins). Twins work in LDS regions of their own (their values are never
// used), so that the one-barrier transposes of the real groups stay race-free.
template <int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3)))
fused_batched_kernel(BatchArgs B) {
  static_assert(NT == 576, "the persistent kernel serves grid lengths up to 24");
  // regions: 24^3 one; 20^3 real threads and twins; 16^3 two targets and twins
  constexpr int kE24 = fused_lds_elems<24>(), kE20 = 2 * fused_lds_elems<20>(), kE16 = 3 * fused_lds_elems<16>();
  constexpr int kLdsElems = kE24 > kE20 ? (kE24 > kE16 ? kE24 : kE16) : (kE20 > kE16 ? kE20 : kE16);
  static_assert(kLdsElems * 8 <= 160 * 1024, "LDS of the persistent kernel");
  __shared__ c64 lds[kLdsElems];
  __shared__ int it_sh;
  NoPairHook nh;
  int sq = blockIdx.x % kBatchQueues;  // only thread 0 uses these two
  int tried = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      int it = -1;
      while (tried < kBatchQueues) {
        const int idx = atomicAdd(&B.counters[sq], 1);
        if (idx < B.qlen[sq]) {
          it = B.qoff[sq] + idx;
          break;
        }
        ++tried;
        sq = (sq + 1) % kBatchQueues;
      }
      it_sh = it;
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(it_sh);
    __syncthreads();
    if (it < 0) return;
    const int cell = __builtin_amdgcn_readfirstlane(B.queue[3 * it]);
    const int item = __builtin_amdgcn_readfirstlane(B.queue[3 * it + 1]);
    const int item2 = __builtin_amdgcn_readfirstlane(B.queue[3 * it + 2]);
    const FusedArgs& a = B.cells[cell];
    const int tr = threadIdx.x;
    switch (a.n) {
      case 16: {
        const int g = tr / 256;  // groups are whole waves; group g works in LDS region g
        const bool second = item2 >= 0 && g == 1;
        fused_item<16>(a, second ? item2 : item, blockIdx.x, lds + g * fused_lds_elems<16>(), tr % 256,
                       !(g == 0 || second), nh);
        break;
      }
      case 20: {
        const bool twin = tr >= 400;
        fused_item<20>(a, item, blockIdx.x, twin ? lds + fused_lds_elems<20>() : lds, tr % 400, twin, nh);
        break;
      }
      default: fused_item<24>(a, item, blockIdx.x, lds, tr, false, nh); break;
    }
  }
}

__global__ void reset_counters_kernel(int* c, int n) {
  for (int i = 0; i < n; ++i) c[i] = 0;
}

template <int N, int WPE>
hipError_t launch_n(const FusedArgs& a, hipStream_t st) {
  FusedArgs b = a;
  b.ksplit = 1;  // one workgroup per target runs the whole k' sum
  hipLaunchKernelGGL((fused_apply_kernel<N, WPE>), dim3(b.nitems), dim3(N * N), 0, st, b);
  return hipGetLastError();
}

template <int N, int WPE>
hipError_t launch_lockstep_n(const FusedArgs& a, const LockstepCfg& ls, hipStream_t st) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(1), 0, st, ls.counters, kLockstepInts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fused_lockstep_kernel<N, WPE>), dim3(ls.nwg), dim3(N * N), 0, st, a, ls.counters);
  if ((e = hipGetLastError()) != hipSuccess || a.ksplit <= 1) return e;
  const long count = (long)a.nitems * N * N * N;
  long g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(add_parts_kernel, dim3((unsigned)g), dim3(256), 0, st, a.out, a.part_out, a.ksplit - 1, count,
                     a.gate);
  return hipGetLastError();
}

}  // namespace

size_t fused_acc_scratch_elems(int n, int nslots) {
  switch (n) {
    case 32: return fused_acc_in_regs<32>() ? 0 : (size_t)nslots * 32 * 32 * 32;
    default: return 0;
  }
}

// 32^3: 0 the grid form, 1 the lockstep form, 2 the split form (split32.hip),
// which the caller launches itself
int fused_variants(int n) { return n == 32 ? 3 : ((n == 16 || n == 20) ? 2 : 1); }

bool fused_has_lockstep(int n) { return n == 32; }

// without a tuned choice at 32^3: the split form
int fused_default_variant(int n) { return n == 32 ? 2 : 0; }

hipError_t launch_fused_apply(int n, const FusedArgs& a, hipStream_t st, int variant, const LockstepCfg* ls) {
  switch (n) {
    case 16: return variant == 1 ? launch_n<16, 2>(a, st) : launch_n<16, 4>(a, st);
    case 20: return variant == 1 ? launch_n<20, 2>(a, st) : launch_n<20, 4>(a, st);
    case 24: return launch_n<24, 3>(a, st);
    case 32:
      if (variant != 1) return launch_n<32, 4>(a, st);
      if (!ls || !ls->counters || ls->nwg < 8 || ls->nwg % 8 != 0) return hipErrorInvalidValue;
      if (a.ksplit > 1 && (a.item0 != 0 || a.nk % a.ksplit != 0 || !a.part_out)) return hipErrorInvalidValue;
      return launch_lockstep_n<32, 4>(a, *ls, st);
    default: return hipErrorInvalidValue;
  }
}

int batched_threads(int nmax) { return nmax > 24 ? 0 : 576; }

hipError_t launch_fused_batched(const BatchArgs& b, int nthreads, int nwg, hipStream_t st) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(1), 0, st, b.counters, kBatchQueues);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nthreads != 576) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fused_batched_kernel<576>, dim3(nwg), dim3(576), 0, st, b);
  return hipGetLastError();
}

}  // namespace fockmi
