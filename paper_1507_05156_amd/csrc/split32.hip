// Fused FP32 pair kernel for 32^3 cells with each target split over two CUs.
//
// A 32^3 complex64 field (256 KiB) fills half of a CU's register file, so one
// workgroup cannot keep a target's FP32 band sum (another 256 KiB) and the
// target itself on chip next to the working field. Here two workgroups on two
// CUs of one XCD share a target: workgroup c in {0, 1} holds the grid points
// with m1 = 2 m1' + c (m1' < 16), i.e. half of the working field, half of the
// band sum and half of the target, all in registers.
//
// Per pair (source k', j), on each half (decimation in time along m1):
//   rho_c = conj(P) X on the half's points;
//   E_c = the 16-point DFT along m1', then the 32-point DFTs along m3 and m2
//         (E_0 is the transform of the even samples, E_1 of the odd ones);
//   the two halves swap E_c through L2 (one exchange per pair);
//   the 32-point transform along m1 is F(l1') = E_0 + tau E_1 and
//   F(l1' + 16) = E_0 - tau E_1 with tau = exp(-2 pi i l1'/32). The kernel
//   multiply and the first step of the inverse transform along m1, back onto
//   the half's own points, fold into
//     G_0 = S E_0 + D (tau E_1),   G_1 = S E_1 + D (conj(tau) E_0),
//   with S = K(l1') + K(l1' + 16) and D = K(l1') - K(l1' + 16) (table of (S, D)
//   pairs, 1/N_r folded), after which the inverse DFTs along m2, m3 and the
//   16-point inverse along m1' give W at the half's points;
//   acc += M W (the FP32 band sum, in registers). Each element's FP32 partial
//   sum covers at most 16 consecutive pairs before it is added into the FP64
//   running sum with Neumaier compensation; the folds are staggered, a few of a
//   thread's elements every other pair, so that their FP64 loads and stores
//   are spread over the pairs.
//
// Layouts, thread t = 32 hi + lo of 512:
//   A (loads, MAC): (m2, m3) = (hi + 16 s, lo) for s in {0, 1}, 16 values m1' each;
//   B: (l1', m2) = (hi, lo), the line along m3;
//   C: (l1', l3) = (hi, lo), the line along m2 (exchange and kernel layout).
// LDS carries the A <-> B and B <-> C transposes of the half field (132 KiB) in
// one array [l1'][m2][m3 or l3] (rows padded to 33). Every phase writes its
// values back to the very slots it read, so a slot is only ever rewritten by the
// thread that last read it, and each transpose needs one barrier (between its
// writes and the next layout's reads), four per pair.
//
// The two workgroups of a pair are blocks b and b + 8 of the launch (blocks are
// dispatched round-robin over the 8 XCDs, so both run on XCD b mod 8); each
// reads its XCD id from the hardware and the pair checks that they agree. Each
// exchange is a rendezvous of wave w of one half with wave w of the other through
// counters in memory (thread t reads exactly what thread t of the other half
// wrote): the writer waits for its stores, then publishes the pair number; the
// reader polls it and reads the other half with device-coherent loads (below). Each half
// has one mailbox; a wave rewrites it only after the other half's wave has
// published that it read the previous contents. Every wait is bounded by a
// real-time limit: on a timeout, or on an
// XCD mismatch, the launch sets an abort word and every workgroup stops; the
// host then runs the one-CU lockstep kernel, gated on that word, over the whole
// application (it rewrites every output element).
//
// Pair symmetry (SYM). When the targets are the sources u over the whole k mesh,
// the pair (target b, source a) has the pair density conj of that of (a, b) and
// the kernel table at -q on the reflected grid (Nyquist planes averaged over both
// signs), so its W is the conjugate of W(a, b). Target (k, i) then runs only the
// source k-points k + d mod N_k, d = 0 .. N_k/2 (the bands of each in a staggered
// order), and for 1 <= d <= (N_k - 1)/2 also adds conj(W) u_(k,i) into a mirror
// copy of target (k + d, j): half the FFT work. Every XCD has its own copy of each
// target (the XCDs' L2s are not coherent within a launch), written only by its
// workgroups, which check at the start that they share one XCD. The pushes into a
// copy follow an order fixed on the host (round, pair, CU pair: a push waits only
// for pushes of smaller keys, so the order cannot deadlock); each push adds into
// the copy's FP32 partial sum and folds one element pair of it into the copy's
// FP64 sums with Neumaier compensation, so no FP32 partial covers more than 16
// pushes. A combine kernel adds the copies to the output in XCD order: the result
// is bitwise repeatable.
//
// Data that another CU wrote during the launch (the other half's mailbox, a mirror
// copy's sums) is read with device-scope coherent loads (the SC1 cache policy), which
// never return a line of this CU's L1 that those stores have made stale. An L1
// invalidate at workgroup scope (buffer_inv sc0) does not give that: a timing copy
// that touched a copy's lines a few microseconds before the other CU pair rewrote
// them read the stale lines after its wait and gave wrong sums. A device-scope
// invalidate (buffer_inv sc1) after every wait gave the right sums but took 2.19 s
// per application on the 32^3 / 216 k / 16-band workload, against 1.82 s.
#include <algorithm>

#include "fused_common.hpp"

namespace fockmi {

namespace {

constexpr int kN = 32;
constexpr int kT = 512;                    // threads per workgroup
constexpr int kHalfElems = kN * kN * kN / 2;  // 16384 points per half
constexpr int kCtr = 4;                    // ints between rendezvous counters (16 bytes)
constexpr int kHalfBlock = (1 + 2 * (kT / 64)) * kCtr;  // counters of one half of a pair
constexpr unsigned kPairBytes = kHalfElems * 8u;
// staggered FP64 fold: kFoldW of a thread's 32 band-sum elements are folded at
// every kFoldSp-th pair, so each element is folded once every 16 pairs (4 at
// every other pair measured 1.5% faster than 2 at every pair on the 32^3 / 216 k
// / 16-band workload; 8 at every 4th spills)
constexpr int kFoldW = 4;
constexpr int kFoldSp = kFoldW / 2;
static_assert(kFoldW == 2 || kFoldW == 4 || kFoldW == 8, "fold width");

// Loads at device scope (cache policy SC1) of data another CU of the XCD has stored:
// they read L2, never a stale line of this CU's L1.
constexpr int kDeviceCoherent = 16;
__device__ __forceinline__ c64 ld_c64_dev(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(c64, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kDeviceCoherent));
}
__device__ __forceinline__ c128 ld_c128_dev(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(c128, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, kDeviceCoherent));
}

// s + c += x with the rounding error of each addition carried in c (no contraction).
__device__ __forceinline__ void neumaier2(double& s, double& c, double x) {
#pragma clang fp contract(off)
  const double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

// LDS access at a per-thread byte base plus a compile-time offset of any size:
// offsets past the 16-bit immediate use a second base formed at the use.
template <unsigned C>
__device__ __forceinline__ c64& lds_far(c64* lds, unsigned base) {
  if constexpr (C < 65536u) {
    return lds_at<C>(lds, base);
  } else {
    constexpr unsigned hi = C & ~0xFFFFu;
    return lds_at<C - hi>(lds, opaque(base + hi));
  }
}

}  // namespace

namespace {

template <bool SYM>
__global__ void __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(2)))
split32_kernel(SplitArgs S) {
  constexpr int NN = kN * kN;
  __shared__ c64 lds[16 * kN * (kN + 1)];
  __shared__ int sh_go, sh_stop;
  const FusedArgs& a = S.f;
  const int t = threadIdx.x;
  const int hi = t >> 5, lo = t & 31;
  const int b = blockIdx.x;
  const int G = gridDim.x;       // a multiple of 16
  const int W = G / 8;           // workgroups per XCD
  const int x = b % 8, wi = b / 8;
  const int c = wi & 1;          // this half holds m1 = 2 m1' + c
  const int pp = wi >> 1;        // pair index within the XCD
  const int npairs = G / 2;
  const int slot = x * (W / 2) + pp;
  // counters of each half (kCtr ints apart): [0] the start handshake, then for each
  // wave w, [1 + 2w] pairs whose data wave w has written to the mailbox and
  // [2 + 2w] pairs whose mailbox data from the other half wave w has read. In layout
  // C thread t reads exactly the element that thread t of the other half wrote, so
  // the exchange is a rendezvous of wave w with wave w of the other half.
  int* mine = S.flags + (slot * 2 + c) * kHalfBlock;
  int* theirs = S.flags + (slot * 2 + (1 - c)) * kHalfBlock;
  int* xcc = S.flags + npairs * 2 * kHalfBlock;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int first = slot;  // target of round 0
  if (first >= a.nitems) return;  // a pair without work takes no part

  // tau_c = exp(-+2 pi i l1'/32) of this thread's l1' in layout C (hi)
  float tr, ti;
  sincospif((float)hi / 16.0f, &ti, &tr);
  ti = c == 0 ? -ti : ti;

  // the calling wave waits until the other half's counter k reaches n (bounded; the
  // loop runs on uniform values); returns 0 when the launch stops (timeout, another
  // pair stopped it, or the host asked)
  auto wait_on = [&](int* ctr, int n) -> int {
    if (S.wait_ticks < 0) {
      __hip_atomic_store(S.status, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 0;
    }
    const unsigned long t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
      const int got = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (got >= n) return 1;
      const int st = __builtin_amdgcn_readfirstlane(__hip_atomic_load(S.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (st != 0) return 0;
      if ((long)(__builtin_amdgcn_s_memrealtime() - t0) > S.wait_ticks) {
        __hip_atomic_store(S.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  };
  auto wait_for = [&](int k, int n) -> int { return wait_on(theirs + k * kCtr, n); };

  // start: the pair checks that both halves run on one XCD (they share its L2)
  if (t == 0) {
    __hip_atomic_store(xcc + b, (int)(__builtin_amdgcn_s_getreg((15 << 11) | 20) & 0xF), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_store(mine, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int go = wait_for(0, 1);
    if (go) {
      const int xm = __hip_atomic_load(xcc + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int xo = __hip_atomic_load(xcc + (c ? b - 8 : b + 8), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (xm != xo) {
        __hip_atomic_store(S.status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        go = 0;
      }
    }
    if constexpr (SYM) {
      // the mirror copies of class x are shared by every workgroup b = x mod 8 through one
      // L2: each checks that it runs on the XCD of block x, the class's first workgroup (it
      // has work whenever any workgroup of its class has)
      if (go) go = wait_on(S.flags + (x * (W / 2) * 2) * kHalfBlock, 1);
      if (go) {
        const int xl = __hip_atomic_load(xcc + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int xm = __hip_atomic_load(xcc + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (xl != xm) {
          __hip_atomic_store(S.status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          go = 0;
        }
      }
    }
    sh_go = go;
    sh_stop = 0;
  }
  __syncthreads();
  if (!sh_go) return;
  int npub = 0;  // pairs exchanged so far

  // per-thread LDS bases (bytes) into the array [l1'][m2][m3 or l3] (33 per row);
  // layouts as in the header
  //   A: element (s, m1') at ((m1' 32 + hi + 16 s) 33 + lo) 8
  //   B: element m3 or l3 at (t 33 + m3) 8
  //   C: element m2 at ((hi 32 + m2) 33 + lo) 8
  const unsigned la = (unsigned)((hi * 33 + lo) * 8);
  const unsigned lb = (unsigned)(t * 33 * 8);
  const unsigned lbc = (unsigned)((hi * 32 * 33 + lo) * 8);
  const unsigned voff8 = (unsigned)(t * 8), voff16 = (unsigned)(t * 16);
  const int nkp = a.nk, nb = a.nb;
  // the exchange mailboxes of this pair (one per half)
  const rsrc_t rMine = make_rsrc(S.xbuf + (long)(slot * 2 + c) * kHalfElems, kPairBytes);
  const rsrc_t rTheirs = make_rsrc(S.xbuf + (long)(slot * 2 + (1 - c)) * kHalfElems, kPairBytes);

  // element (m1', s) of layout A sits at c NN + m1' 2NN + s NN/2 + t of its field;
  // byte offset of element E beyond t (8-byte elements)
  auto offA8 = [](auto e) constexpr { constexpr int E = decltype(e)::value; return (unsigned)(((E % 16) * 2 * NN + (E / 16) * NN / 2) * 8); };
  const int npair_tg = SYM ? S.ndelta * nb : nkp * nb;  // pairs of one target
  for (int tg = first; tg < a.nitems; tg += npairs) {
    const int kt = tg / a.nx, it = tg - kt * a.nx;
    // source orbital of pair s: (k', j) = (s / nb, s mod nb); with the pair symmetry
    // (k', j) = (kt + d mod nk, j) for s = d nb + j
    auto source = [&](int s) -> int {
      if constexpr (SYM) {
        const int d = s / nb, m = s - d * nb;
        const int ks = kt + d < nkp ? kt + d : kt + d - nkp;
        const int i0 = it >> S.stagger_shift;
        const int j = i0 + m < nb ? i0 + m : i0 + m - nb;
        return ks * nb + j;
      } else {
        return s;
      }
    };
    const rsrc_t rX = make_rsrc(a.X + (long)tg * 2 * kHalfElems + c * NN, 2 * kHalfElems * 8u);
    const rsrc_t rOut = make_rsrc(a.out + (long)tg * 2 * kHalfElems + c * NN, 2 * kHalfElems * 16u);
    const rsrc_t rComp = make_rsrc(a.comp + (long)tg * 2 * kHalfElems + c * NN, 2 * kHalfElems * 8u);
    c64 X[32], acc[32], v[32];
    // this half of the target, and the pair density of the first pair
    {
      const rsrc_t rP0 = make_rsrc(a.P + (long)source(0) * 2 * kHalfElems + c * NN, 2 * kHalfElems * 8u);
      static_for<32>([&](auto e) {
        X[decltype(e)::value] = ld_c64(rX, voff8, offA8(e));
        v[decltype(e)::value] = ld_c64(rP0, voff8, offA8(e));
      });
      static_for<32>([&](auto e) {
        v[decltype(e)::value] = cmulc(v[decltype(e)::value], X[decltype(e)::value]);
        acc[decltype(e)::value] = c64{0.0f, 0.0f};
      });
    }
    for (int src = 0; src < npair_tg; ++src) {
      const int sb = source(src);  // source orbital (k', j) = (sb / nb, sb mod nb)
      const int ks = sb / nb;
      const int qi = __builtin_amdgcn_readfirstlane(a.qidx[kt * a.nk + ks]);
      const rsrc_t rSD = make_rsrc(S.SD + (long)qi * kHalfElems * 2, kHalfElems * 8u);
      const rsrc_t rM = make_rsrc(a.M + (long)sb * 2 * kHalfElems + c * NN, 2 * kHalfElems * 8u);
      const bool has_next = src + 1 < npair_tg;
      const rsrc_t rPn = make_rsrc(a.P + (long)source(has_next ? src + 1 : src) * 2 * kHalfElems + c * NN,
                                   2 * kHalfElems * 8u);
      // ---- layout A: 16-point DFTs along m1' of the pair density in v
      static_for<2>([&](auto g) {
        constexpr int G0 = decltype(g)::value * 16;
        c64 w[16];
        static_for<16>([&](auto e) { w[decltype(e)::value] = v[G0 + decltype(e)::value]; });
        fft<16, -1>(w);
        static_for<16>([&](auto e) { v[G0 + decltype(e)::value] = w[decltype(e)::value]; });
      });
      // ---- A -> B
      static_for<32>([&](auto e) {
        constexpr int E = decltype(e)::value, s = E / 16, m = E % 16;
        lds_far<(unsigned)((m * 32 * 33 + s * 16 * 33) * 8)>(lds, la) = v[E];
      });
      __syncthreads();
      {
        const unsigned bb = opaque(lb);
        static_for<32>([&](auto e) { v[decltype(e)::value] = lds_at<decltype(e)::value * 8>(lds, bb); });
      }
      fft<32, -1, true>(v);
      // ---- B -> C: B writes back to the slots it read; meanwhile each wave checks
      // that the other half's wave has read this wave's previous mailbox contents
      // (usually long done), before it rewrites them
      {
        const unsigned bb = opaque(lb);
        static_for<32>([&](auto e) { lds_at<decltype(e)::value * 8>(lds, bb) = v[decltype(e)::value]; });
      }
      ++npub;
      if (!wait_for(2 + 2 * w, npub - 1)) sh_stop = 1;
      __syncthreads();
      {
        const unsigned bb = opaque(lbc);
        static_for<32>([&](auto e) { v[decltype(e)::value] = lds_at<decltype(e)::value * 33 * 8>(lds, bb); });
      }
      fft<32, -1, true>(v);
      // ---- exchange: this half's E_c out, the other half's in. The first group
      // of (S, D) values is loaded ahead: it does not depend on the other half.
      constexpr int GC = 8;  // elements per combine group
      c64 sd0[GC];
      static_for<GC>([&](auto e) { sd0[decltype(e)::value] = ld_c64(rSD, voff8, (unsigned)(decltype(e)::value * kT * 8)); });
      static_for<32>([&](auto e) { st_c64(v[decltype(e)::value], rMine, voff8, (unsigned)(decltype(e)::value * kT * 8)); });
      __builtin_amdgcn_sched_barrier(0);
      // wave-level rendezvous: this wave's stores are in L2; publish, wait for the
      // other half's wave (a failed wait stops the workgroup at the next barrier)
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      // (every lane stores the same value: a branch on the lane would split the
      // live ranges of the resident field across a divergent region)
      __hip_atomic_store(mine + (1 + 2 * w) * kCtr, npub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!wait_for(1 + 2 * w, npub)) sh_stop = 1;
      // no load of the other half's data moves above the wait (those loads are
      // device-coherent)
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      // ---- combine: G_c = S own + D (tau_c other), group by group
      static_for<32 / GC>([&](auto g) {
        constexpr int G0 = decltype(g)::value * GC;
        c64 o[GC], sd[GC];
        static_for<GC>([&](auto e) {
          constexpr int E = G0 + decltype(e)::value;
          o[decltype(e)::value] = ld_c64_dev(rTheirs, voff8, (unsigned)(E * kT * 8));
          if constexpr (G0 == 0) sd[decltype(e)::value] = sd0[decltype(e)::value];
          else sd[decltype(e)::value] = ld_c64(rSD, voff8, (unsigned)(E * kT * 8));
        });
        __builtin_amdgcn_sched_barrier(0);
        static_for<GC>([&](auto e) {
          constexpr int E = G0 + decltype(e)::value;
          const c64 q = o[decltype(e)::value];
          const float sS = sd[decltype(e)::value].re, sD = sd[decltype(e)::value].im;
          const float qr = tr * q.re - ti * q.im, qi2 = tr * q.im + ti * q.re;
          v[E] = c64{fmadd(sD, qr, sS * v[E].re), fmadd(sD, qi2, sS * v[E].im)};
        });
      });
      // every value this wave read from the mailbox is used: it is free again
      __hip_atomic_store(mine + (2 + 2 * w) * kCtr, npub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_sched_barrier(0);
      fft<32, +1, true>(v);
      // ---- C -> B (after its barrier, a stop requested by any wave is seen by all)
      {
        const unsigned bb = opaque(lbc);
        static_for<32>([&](auto e) { lds_at<decltype(e)::value * 33 * 8>(lds, bb) = v[decltype(e)::value]; });
      }
      __syncthreads();
      if (sh_stop) return;
      {
        const unsigned bb = opaque(lb);
        static_for<32>([&](auto e) { v[decltype(e)::value] = lds_at<decltype(e)::value * 8>(lds, bb); });
      }
      fft<32, +1, true>(v);
      // ---- B -> A
      {
        const unsigned bb = opaque(lb);
        static_for<32>([&](auto e) { lds_at<decltype(e)::value * 8>(lds, bb) = v[decltype(e)::value]; });
      }
      __syncthreads();
      static_for<32>([&](auto e) {
        constexpr int E = decltype(e)::value, s = E / 16, m = E % 16;
        v[E] = lds_far<(unsigned)((m * 32 * 33 + s * 16 * 33) * 8)>(lds, la);
      });
      static_for<2>([&](auto g) {
        constexpr int G0 = decltype(g)::value * 16;
        c64 w[16];
        static_for<16>([&](auto e) { w[decltype(e)::value] = v[G0 + decltype(e)::value]; });
        fft<16, +1>(w);
        static_for<16>([&](auto e) { v[G0 + decltype(e)::value] = w[decltype(e)::value]; });
      });
      // ---- acc += M W into the FP32 band sums, and, in the same memory phase, the
      // next pair's density conj(P) X into v as each W element is consumed.
      // Staggered fold into FP64: at the last pair of every kFoldSp (not the last
      // pair of the target), elements kFoldW f .. kFoldW f + kFoldW - 1,
      // f = (src / kFoldSp) mod (32 / kFoldW), add their FP32 partial sums (at most
      // 16 pairs each) to the FP64 running sum with Neumaier compensation; the last
      // pair's partials go into the final fold.
      const int f = (src / kFoldSp) % (32 / kFoldW);
      const bool fold = has_next && src % kFoldSp == kFoldSp - 1;
      const bool fold_prev = src >= 16;  // these elements were folded before
      // element kFoldW f + k: m1' = (kFoldW f) mod 16 + k, s = (kFoldW f) / 16
      const unsigned fo0 = (unsigned)((((kFoldW * f) % 16) * 2 * NN + ((kFoldW * f) / 16) * NN / 2) * 8);
      c128 fq[kFoldW];
      c64 fc[kFoldW];
      // ---- pair symmetry: this pair's push into the mirror copy of source sb held for
      // this XCD (x), in the order the rank table fixes: the push of rank r waits until the
      // copy has taken r pushes. The counters are per half and wave: a wave touches only
      // its own elements of the copy.
      const bool push = SYM && src >= nb && src / nb <= S.npush;
      int rank = 0;
      const long cp = SYM ? (long)x * a.nitems + sb : 0;  // mirror copy (XCD, target sb)
      int* const mctr = SYM ? S.mdone + ((cp * 2 + c) * 8 + w) * kCtr : nullptr;
      if constexpr (SYM) {
        if (push) {
          rank = __builtin_amdgcn_readfirstlane(S.rank[(long)tg * npair_tg + src]);
          if (rank > 0) {
            if (!wait_on(mctr, rank)) sh_stop = 1;
            // the copy was last written by another CU of this XCD: its loads below are
            // device-coherent and stay below the wait
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
          }
        }
      }
      // ---- mirror pass (pair symmetry): the copy's FP32 partial sum += conj(W) X, the fold
      // of one element pair of it into the copy's FP64 sums, and the publish, ahead of the
      // multiply-accumulate, so that the copy's next push waits for this part only. One
      // code path for every pair (branching between forms of these loops makes the
      // allocator spill): the partial sum is read through a resource of size 0 at the copy's
      // first push (loads return zero), and every resource has size 0 when the pair pushes
      // nothing (stores are dropped). The push of rank r folds the element pair (E0, E0 + 1),
      // E0 = 2 g, g = r mod 16, so each element of a copy is folded at every 16th push.
      if constexpr (SYM) {
#pragma clang fp contract(off)
        const int mg = rank & 15;
        const unsigned fm0 = (unsigned)(((2 * (mg & 7)) * 2 * NN + (mg >> 3) * NN / 2) * 8);
        const bool prev = push && rank >= 16;  // the pair's FP64 sums were written before
        const c64* mp_base = S.mpart + cp * 2 * kHalfElems + c * NN;
        const c128* ms_base = S.msum + cp * 2 * kHalfElems + c * NN;
        const c64* mc_base = S.mcomp + cp * 2 * kHalfElems + c * NN;
        const rsrc_t rMPl = make_rsrc(mp_base, push && rank > 0 ? 2 * kHalfElems * 8u : 0u);
        const rsrc_t rMPs = make_rsrc(mp_base, push ? 2 * kHalfElems * 8u : 0u);
        constexpr int GP = 16;  // partial sums loaded per group (16: 1,819 against 1,836 ms for 8 on C2)
        static_for<32 / GP>([&](auto g) {
          constexpr int G0 = decltype(g)::value * GP;
          c64 qv[GP];
          static_for<GP>([&](auto e) {
            constexpr auto E = std::integral_constant<int, G0 + decltype(e)::value>{};
            qv[decltype(e)::value] = ld_c64_dev(rMPl, voff8, offA8(E));
          });
          __builtin_amdgcn_sched_barrier(0);
          static_for<GP>([&](auto e) {
            constexpr auto E = std::integral_constant<int, G0 + decltype(e)::value>{};
            const c64 wv = v[E], xv = X[E], q0 = qv[decltype(e)::value];
            st_c64(c64{fmadd(wv.im, xv.im, fmadd(wv.re, xv.re, q0.re)), fmadd(-wv.im, xv.re, fmadd(wv.re, xv.im, q0.im))},
                   rMPs, voff8, offA8(E));
          });
        });
        // the folded pair's partial sums and FP64 values
        c128 msq[2];
        c64 mq[2], mcq[2];
        {
          const rsrc_t rMSl = make_rsrc(ms_base, prev ? 2 * kHalfElems * 16u : 0u);
          const rsrc_t rMCl = make_rsrc(mc_base, prev ? 2 * kHalfElems * 8u : 0u);
          static_for<2>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            mq[k] = ld_c64_dev(rMPs, voff8, fm0 + k * 2 * NN * 8);  // the partial sum this thread has just stored
            msq[k] = ld_c128_dev(rMSl, voff16, 2 * (fm0 + k * 2 * NN * 8));
            mcq[k] = ld_c64_dev(rMCl, voff8, fm0 + k * 2 * NN * 8);
          });
        }
        const rsrc_t rMSs = make_rsrc(ms_base, push ? 2 * kHalfElems * 16u : 0u);
        const rsrc_t rMCs = make_rsrc(mc_base, push ? 2 * kHalfElems * 8u : 0u);
        static_for<2>([&](auto kk) {
          constexpr int k = decltype(kk)::value;
          const unsigned fo = fm0 + k * 2 * NN * 8;
          double sr = msq[k].re, si = msq[k].im, cr = mcq[k].re, ci = mcq[k].im;
          neumaier2(sr, cr, a.scale * (double)mq[k].re);
          neumaier2(si, ci, a.scale * (double)mq[k].im);
          st_c128(c128{sr, si}, rMSs, voff16, 2 * fo);
          st_c64(c64{(float)cr, (float)ci}, rMCs, voff8, fo);
          st_c64(c64{0.0f, 0.0f}, rMPs, voff8, fo);  // the pair's partial sum starts again
        });
        if (push) {
          // every store of this push is in L2: publish it to the copy's next push
          asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
          __hip_atomic_store(mctr, rank + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      // ---- the multiply-accumulate acc += M W, and v = conj(P_next) X
      constexpr int GM = 8;
      static_for<32 / GM>([&](auto g) {
        constexpr int G0 = decltype(g)::value * GM;
        c64 mv[GM], pv[GM];
        static_for<GM>([&](auto e) {
          constexpr auto E = std::integral_constant<int, G0 + decltype(e)::value>{};
          mv[decltype(e)::value] = ld_c64(rM, voff8, offA8(E));
          pv[decltype(e)::value] = ld_c64(rPn, voff8, offA8(E));
        });
        __builtin_amdgcn_sched_barrier(0);
        static_for<GM>([&](auto e) {
          constexpr int E = G0 + decltype(e)::value;
          acc[E] = cmac(acc[E], mv[decltype(e)::value], v[E]);
          v[E] = cmulc(pv[decltype(e)::value], X[E]);
        });
      });
      if (fold) {
        static_for<kFoldW>([&](auto kk) {
          constexpr int k = decltype(kk)::value;
          if (fold_prev) {
            fq[k] = ld_c128(rOut, voff16, 2 * (fo0 + k * 2 * NN * 8));
            fc[k] = ld_c64(rComp, voff8, fo0 + k * 2 * NN * 8);
          } else {
            fq[k] = c128{0.0, 0.0};
            fc[k] = c64{0.0f, 0.0f};
          }
        });
      }
      if (fold) {
#pragma clang fp contract(off)
        static_for<32 / kFoldW>([&](auto ff) {
          constexpr int F = decltype(ff)::value;
          if (f == F) {
            static_for<kFoldW>([&](auto kk) {
              constexpr int k = decltype(kk)::value, E = kFoldW * F + k;
              const unsigned fo = fo0 + k * 2 * NN * 8;
              double sr = fq[k].re, si = fq[k].im, cr = fc[k].re, ci = fc[k].im;
              neumaier2(sr, cr, a.scale * (double)acc[E].re);
              neumaier2(si, ci, a.scale * (double)acc[E].im);
              st_c128(c128{sr, si}, rOut, voff16, 2 * fo);
              st_c64(c64{(float)cr, (float)ci}, rComp, voff8, fo);
              acc[E] = c64{0.0f, 0.0f};
            });
          }
        });
      }
    }
    // ---- final fold of every element: s + c into the output
    {
#pragma clang fp contract(off)
      constexpr int GF = 4;
      static_for<32 / GF>([&](auto g) {
        constexpr int G0 = decltype(g)::value * GF;
        c128 oq[GF];
        c64 cq[GF];
        static_for<GF>([&](auto e) {
          constexpr auto E = std::integral_constant<int, G0 + decltype(e)::value>{};
          // folded before iff its first fold pair came before the last pair
          if ((E / kFoldW) * kFoldSp + kFoldSp - 1 < npair_tg - 1) {
            oq[decltype(e)::value] = ld_c128(rOut, voff16, 2 * offA8(E));
            cq[decltype(e)::value] = ld_c64(rComp, voff8, offA8(E));
          } else {
            oq[decltype(e)::value] = c128{0.0, 0.0};
            cq[decltype(e)::value] = c64{0.0f, 0.0f};
          }
        });
        static_for<GF>([&](auto e) {
          constexpr auto E = std::integral_constant<int, G0 + decltype(e)::value>{};
          double sr = oq[decltype(e)::value].re, si = oq[decltype(e)::value].im;
          double cr = cq[decltype(e)::value].re, ci = cq[decltype(e)::value].im;
          neumaier2(sr, cr, a.scale * (double)acc[E].re);
          neumaier2(si, ci, a.scale * (double)acc[E].im);
          st_c128(c128{sr + cr, si + ci}, rOut, voff16, 2 * offA8(E));
        });
      });
    }
  }
}

// flags, XCD ids, mirror counters and the abort word to zero (a kernel, so that a
// captured graph holds no memset)
__global__ void split_reset_kernel(int* flags, int nflags, int* mdone, long nmdone, int* status) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nflags; i += gridDim.x * blockDim.x) flags[i] = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nmdone; i += (long)gridDim.x * blockDim.x)
    mdone[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) status[0] = 0;
}

// out[b] += the mirror copies of target b, in XCD order. In a copy that took n pushes,
// the element pair g is folded at the pushes of rank g, g + 16, ... (so at least once iff
// g < n): its FP64 sum and compensation hold the pushes up to its last fold, its FP32
// partial sum the pushes after that.
__global__ void sym_combine_kernel(c128* __restrict__ out, const c128* __restrict__ msum,
                                   const c64* __restrict__ mcomp, const c64* __restrict__ mpart,
                                   const int* __restrict__ cnt, int nitems, double scale, const int* status) {
  constexpr long NR = (long)kN * kN * kN;
  if (status[0] != 0) return;  // the split launch stopped: the lockstep form rewrites out
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)nitems * NR) return;
  const int tb = (int)(idx / NR);
  const int e = (int)(idx % NR);
  // layout A of the kernel: half c = m1 mod 2, element E = 16 s + m1' with m1' = m1 / 2,
  // s = m2 / 16; the fold pair of E is E / 2
  const int m1 = e >> 10, m2 = (e >> 5) & 31;
  const int g = 8 * (m2 >> 4) + (m1 >> 2);
  double re = out[idx].re, im = out[idx].im;
  for (int xc = 0; xc < 8; ++xc) {
    const int n = cnt[(long)xc * nitems + tb];
    if (n == 0) continue;
    const long o = ((long)xc * nitems + tb) * NR + e;
    double sr = 0.0, si = 0.0;
    if (g < n) {
      sr = msum[o].re + (double)mcomp[o].re;
      si = msum[o].im + (double)mcomp[o].im;
    }
    sr += scale * (double)mpart[o].re;
    si += scale * (double)mpart[o].im;
    re += sr;
    im += si;
  }
  out[idx] = c128{re, im};
}

// (S, D) table: for layout C element (l2 * 512 + t), t = 32 l1' + l3, from the
// FP64 natural-order table K[l1][l2][l3] (1/N_r folded)
__global__ void build_sd_kernel(float* __restrict__ SD, const double* __restrict__ K, int nq) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // l2 * 512 + t
  const int q = blockIdx.y;
  if (idx >= kHalfElems || q >= nq) return;
  const int l2 = idx / kT, t = idx % kT;
  const int l1 = t / 32, l3 = t % 32;
  const double* Kq = K + (long)q * 2 * kHalfElems;
  const double ka = Kq[(l1 * kN + l2) * kN + l3];
  const double kb = Kq[((l1 + 16) * kN + l2) * kN + l3];
  SD[((long)q * kHalfElems + idx) * 2 + 0] = (float)(ka + kb);
  SD[((long)q * kHalfElems + idx) * 2 + 1] = (float)(ka - kb);
}

__global__ void count_abort_kernel(long long* count, const int* status) {
  if (status[0] != 0) count[0] += 1;
}

__global__ void zero_ll_kernel(long long* p) { p[0] = 0; }

}  // namespace

hipError_t launch_count_abort(long long* count, const int* status, hipStream_t st) {
  hipLaunchKernelGGL(count_abort_kernel, dim3(1), dim3(1), 0, st, count, status);
  return hipGetLastError();
}

hipError_t launch_zero_ll(long long* p, hipStream_t st) {
  hipLaunchKernelGGL(zero_ll_kernel, dim3(1), dim3(1), 0, st, p);
  return hipGetLastError();
}

size_t split32_flag_ints(int nwg) { return (size_t)(nwg / 2) * 2 * kHalfBlock + (size_t)nwg; }
size_t split32_mirror_ctr_ints(int nitems) { return (size_t)8 * nitems * 2 * (kT / 64) * kCtr; }

void split32_sym_tables(int nwg, int nk, int nb, int shift, std::vector<int>* rank, std::vector<int>* cnt) {
  // every CU pair runs its targets round by round and the pairs of a target in order; a
  // push's key is (round, pair, CU pair within the XCD), and each copy (XCD, target) takes
  // its pushes in key order. A push waits only for pushes of smaller keys (or for its own
  // pair's exchange partner at the same key), so the order cannot deadlock.
  const int npairs = nwg / 2, per_x = npairs / 8;
  const int nitems = nk * nb, ndelta = nk / 2 + 1, npush = (nk - 1) / 2, ns = ndelta * nb;
  rank->assign((size_t)nitems * ns, -1);
  cnt->assign((size_t)8 * nitems, 0);
  const int rounds = (nitems + npairs - 1) / npairs;
  for (int r = 0; r < rounds; ++r)
    for (int s = nb; s < ns; ++s) {
      const int d = s / nb, j = s % nb;
      if (d > npush) break;
      for (int xc = 0; xc < 8; ++xc)
        for (int pp = 0; pp < per_x; ++pp) {
          const int tg = xc * per_x + pp + r * npairs;
          if (tg >= nitems) continue;
          const int b = ((tg / nb + d) % nk) * nb + (((tg % nb) >> shift) + j) % nb;
          (*rank)[(size_t)tg * ns + s] = (*cnt)[(size_t)xc * nitems + b]++;
        }
    }
}
size_t split32_xbuf_elems(int nwg) { return (size_t)(nwg / 2) * 2 * kHalfElems; }
size_t split32_sd_floats(int nq) { return (size_t)nq * kHalfElems * 2; }

hipError_t launch_build_sd32(float* SD, const double* K, int nq, hipStream_t st) {
  for (int q0 = 0; q0 < nq; q0 += 65535) {
    const int cnt = nq - q0 < 65535 ? nq - q0 : 65535;
    hipLaunchKernelGGL(build_sd_kernel, dim3(kHalfElems / 256, cnt), dim3(256), 0, st,
                       SD + (long)q0 * kHalfElems * 2, K + (long)q0 * 2 * kHalfElems, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_split32(const SplitArgs& s, int nwg, hipStream_t st) {
  if (nwg < 16 || nwg % 16 != 0 || s.f.accumulate) return hipErrorInvalidValue;
  if (s.sym && (s.f.nx != s.f.nb || s.f.nitems != s.f.nk * s.f.nb || s.ndelta != s.f.nk / 2 + 1 ||
                s.npush != (s.f.nk - 1) / 2 || !s.rank || !s.mpart || !s.msum || !s.mcomp || !s.mdone))
    return hipErrorInvalidValue;
  const int nflags = (int)split32_flag_ints(nwg);
  const long nmdone = s.sym ? (long)split32_mirror_ctr_ints(s.f.nitems) : 0;
  const long nreset = std::max<long>(nflags, nmdone);
  const int rblocks = (int)std::min<long>((nreset + 255) / 256, 4096);
  hipLaunchKernelGGL(split_reset_kernel, dim3(rblocks), dim3(256), 0, st, s.flags, nflags, s.mdone, nmdone,
                     s.status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (s.sym) hipLaunchKernelGGL(split32_kernel<true>, dim3(nwg), dim3(kT), 0, st, s);
  else hipLaunchKernelGGL(split32_kernel<false>, dim3(nwg), dim3(kT), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_split32_sym_combine(c128* out, const c128* msum, const c64* mcomp, const c64* mpart,
                                      const int* cnt, int nitems, double scale, const int* status,
                                      hipStream_t st) {
  const long n = (long)nitems * kN * kN * kN;
  hipLaunchKernelGGL(sym_combine_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, msum, mcomp,
                     mpart, cnt, nitems, scale, status);
  return hipGetLastError();
}

}  // namespace fockmi
