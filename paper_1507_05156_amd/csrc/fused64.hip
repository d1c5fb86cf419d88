// Fused FP64 pair kernel: every step of Eq. (15) for one pair in complex128,
// without leaving the CU, for cubic grids of length 16, 20 and 24.
//
// The structure is the FP32 form's: one workgroup of N*N threads owns one
// target field X[kt][s] and runs over all sources (k', j); each thread holds
// one line of the field in registers (x phase: along n1 at fixed (m2, m3);
// y phase: along n2 at fixed (l1, m3); z phase: along n3 at fixed (l1, l2),
// where the kernel multiplies), and LDS carries only the transposes. What
// differs is the arithmetic and where the sum lives:
//   * every product, transform and sum is FP64;
//   * the sum over all (k', j) is one FP64 accumulator per element, in
//     registers for N = 16 and 20, and for N = 24 (a line of 24 complex128
//     values already takes 96 of the 168 VGPRs a 9-wave workgroup may use) in
//     a per-workgroup global buffer;
//   * out = scale * sum (+ out) is written once, at the end.
// A complex128 field of 24^3 does not fit in LDS, so at N = 24 each transpose
// runs in two rounds over half of the field, as the FP32 form does at 32^3.
#include "fused_common.hpp"

namespace fockmi {

template <int N>
constexpr int f64_nph() {
  return ((long)N * N * (N + 1) * 16 > 160L * 1024) ? 2 : 1;
}

template <int N>
constexpr bool f64_acc_in_regs() {
  return N <= 20;
}

// Where the FP64 accumulator is a global buffer (24^3), its first elements of
// each thread's line live in registers and the next ones in LDS (thread-private
// slots beside the transpose array), which takes their read-modify-write off
// device memory: the kernel there is bound by that traffic.
template <int N>
constexpr int f64_acc_regs() {
  return f64_acc_in_regs<N>() ? 0 : 4;
}
template <int N>
constexpr int f64_acc_lds() {
  return f64_acc_in_regs<N>() ? 0 : 4;
}

// the target held in registers for the whole work item (see the FP32 kernel):
// at 16^3 two 256-thread workgroups per CU leave room for it
template <int N>
constexpr bool f64_x_in_regs() {
  return N == 16;
}

template <int N>
constexpr int f64_lds_elems() {
  constexpr int NPH = f64_nph<N>();
  constexpr int H = N / NPH, NBK = N / NPH;
  constexpr int A = N * N * H, B = NBK * N * (N + 1);
  return A > B ? A : B;
}

// group sizes of the global loads (issued together, consumed after the group is in flight)
template <int N>
constexpr int f64_grp() {
  return 4;
}

int fused64_phases(int n) {
  switch (n) {
    case 16: return f64_nph<16>();
    case 20: return f64_nph<20>();
    case 24: return f64_nph<24>();
    default: return 0;
  }
}

bool fused64_supported(int n) { return n == 16 || n == 20 || n == 24; }

size_t fused64_acc_scratch_elems(int n, int nslots) {
  return (fused64_supported(n) && n > 20) ? (size_t)nslots * n * n * n : 0;
}

namespace {

template <int N>
__device__ __forceinline__ void f64_item(const Fused64Args& a, int item, int acc_slot, c128* __restrict__ lds,
                                         c128* __restrict__ lds_acc) {
  constexpr int NTI = N * N;
  constexpr int NR = N * N * N;
  constexpr int NPH = f64_nph<N>();
  constexpr int H = N / NPH;      // width of one round of the x<->y transpose (along m3)
  constexpr int TPG = NTI / NPH;  // threads per round
  constexpr int NBK = N / NPH;    // l1 values per round of the y<->z transpose
  constexpr bool ACCREG = f64_acc_in_regs<N>();
  constexpr bool XREG = f64_x_in_regs<N>();
  constexpr int AR = f64_acc_regs<N>(), AL = f64_acc_lds<N>();  // accumulator elements in registers, in LDS
  constexpr int G = f64_grp<N>();
  static_assert(N % G == 0, "load groups must tile the line");

  // The round of a thread is uniform over its wave only when the rounds are
  // whole waves; at N = 24 (288 threads per x<->y round, 144 per y<->z round)
  // they are not, and each lane takes its own branch.
  constexpr bool XY_WAVES = TPG % 64 == 0;
  constexpr bool YZ_WAVES = XY_WAVES && (NBK * H) % 64 == 0;
  const int t = threadIdx.x;
  const int grp = XY_WAVES ? __builtin_amdgcn_readfirstlane(t / TPG) : t / TPG;
  const int tl = t % TPG;
  const int hl = tl % H;
  const int clo = hl + H * grp;  // m3 in the x and y phases, l2 in the z phase
  const int chi = tl / H;        // m2 in the x phase, l1 in the y and z phases
  const int gyz = YZ_WAVES ? __builtin_amdgcn_readfirstlane(chi / NBK) : chi / NBK;
  const int lrow = chi % NBK;

  // LDS byte offsets of this thread's elements in the four transposes (16-byte elements);
  // the x side of x<->y spans more than 64 KiB and uses a second base from L1S on.
  // With one round (N <= 20) both transposes use one array [l1][m2 or l2][m3] with
  // rows padded to N+1, every phase writes its values back to the slots it read,
  // and each transpose needs one barrier; with two rounds (N = 24) the rounds share
  // the x<->y array and each transpose keeps a second barrier.
  constexpr bool INPLACE = NPH == 1;
  constexpr unsigned SX = INPLACE ? (unsigned)(N * (N + 1) * 16) : (unsigned)(N * H * 16);
  constexpr unsigned SY = INPLACE ? (unsigned)((N + 1) * 16) : (unsigned)(H * 16);
  constexpr int L1S = (int)((65535u / SX) + 1) < N ? (int)((65535u / SX) + 1) : N;
  const unsigned lx0 = INPLACE ? (unsigned)((chi * (N + 1) + hl) * 16) : (unsigned)((chi * H + hl) * 16);
  const unsigned ly0 = INPLACE ? (unsigned)((chi * N * (N + 1) + hl) * 16) : (unsigned)((chi * N * H + hl) * 16);
  const unsigned lyz0 = (unsigned)((lrow * N * (N + 1) + clo) * 16);
  const unsigned lz0 = (unsigned)((lrow * N + clo) * (N + 1) * 16);

  const int kt = item / a.nx;
  const int s = item % a.nx;
  // global byte offsets: x-phase element (m1, m2 = chi, m3 = clo) at voff + m1 * N*N*16;
  // table and accumulator buffer are value-major: (v, t) at (v * NTI + t) * size
  const unsigned voff = (unsigned)((chi * N + clo) * 16);
  const unsigned voff_t8 = (unsigned)(t * 8);
  const unsigned voff_t16 = (unsigned)(t * 16);
  constexpr unsigned FB = NR * 16u;

  const rsrc_t rX = make_rsrc(a.X + ((long)kt * a.nx + s) * NR, FB);
  const rsrc_t rOut = make_rsrc(a.out + ((long)kt * a.nx + s) * NR, FB);
  const rsrc_t rAcc = make_rsrc(ACCREG ? a.out : a.accs + (long)acc_slot * NR, ACCREG ? 0u : FB);

  c128 acc[ACCREG ? N : 1];
  c128 accr[AR > 0 ? AR : 1];
  c128 xr[XREG ? N : 1];
  if constexpr (XREG) static_for<N>([&](auto m1) { xr[m1] = ld_c128(rX, voff, (unsigned)(decltype(m1)::value * NTI * 16)); });
  if constexpr (ACCREG) {
#pragma unroll
    for (int m1 = 0; m1 < N; ++m1) acc[m1] = c128{0.0, 0.0};
  }

  for (int ks = 0; ks < a.nk; ++ks) {
    const int qi = __builtin_amdgcn_readfirstlane(a.qidx[kt * a.nk + ks]);
    const rsrc_t rK = make_rsrc(a.Kt + (long)qi * NR, NR * 8u);
    for (int j = 0; j < a.nb; ++j) {
      const rsrc_t rP = make_rsrc(a.P + ((long)ks * a.nb + j) * NR, FB);
      const rsrc_t rM = make_rsrc(a.M + ((long)ks * a.nb + j) * NR, FB);
      c128 v[N];
      static_for<N / G>([&](auto cc) {
        constexpr int C0 = decltype(cc)::value * G;
        c128 p[G], x[G];
        static_for<G>([&](auto q) {
          const unsigned so = (unsigned)((C0 + decltype(q)::value) * NTI * 16);
          p[q] = ld_c128(rP, voff, so);
          if constexpr (XREG) x[q] = xr[C0 + decltype(q)::value];
          else x[q] = ld_c128(rX, voff, so);
        });
        __builtin_amdgcn_sched_barrier(0);
        static_for<G>([&](auto q) { v[C0 + decltype(q)::value] = cmulc(p[q], x[q]); });
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
          static_for<N>([&](auto l2) { lds_at<decltype(l2)::value * (N + 1) * 16>(lds, b) = v[l2]; });
        }
        __syncthreads();
        if (gyz == g) {
          const unsigned b = opaque(lz0);
          static_for<N>([&](auto m3) { v[m3] = lds_at<decltype(m3)::value * 16>(lds, b); });
        }
        if constexpr (!INPLACE) __syncthreads();
      }
      fft<N, -1>(v);
      static_for<N / G>([&](auto cc) {
        constexpr int C0 = decltype(cc)::value * G;
        double kv[G];
        static_for<G>([&](auto q) { kv[q] = ld_f64(rK, voff_t8, (unsigned)((C0 + decltype(q)::value) * NTI * 8)); });
        __builtin_amdgcn_sched_barrier(0);
        static_for<G>([&](auto q) { v[C0 + decltype(q)::value] = cscale(v[C0 + decltype(q)::value], kv[q]); });
      });
      fft<N, +1>(v);
      // z -> y
#pragma unroll
      for (int g = 0; g < NPH; ++g) {
        if (gyz == g) {
          const unsigned b = opaque(lz0);
          static_for<N>([&](auto m3) { lds_at<decltype(m3)::value * 16>(lds, b) = v[m3]; });
        }
        __syncthreads();
        if (gyz == g) {
          const unsigned b = opaque(lyz0);
          static_for<N>([&](auto l2) { v[l2] = lds_at<decltype(l2)::value * (N + 1) * 16>(lds, b); });
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

      // multiply-accumulate into the FP64 sum over all (k', j)
      if constexpr (ACCREG) {
        static_for<N / G>([&](auto cc) {
          constexpr int C0 = decltype(cc)::value * G;
          c128 mv[G];
          static_for<G>([&](auto q) { mv[q] = ld_c128(rM, voff, (unsigned)((C0 + decltype(q)::value) * NTI * 16)); });
          __builtin_amdgcn_sched_barrier(0);
          static_for<G>([&](auto q) {
            constexpr int m1 = C0 + decltype(q)::value;
            acc[m1] = cmac(acc[m1], mv[q], v[m1]);
          });
        });
      } else {
        // the position of the pair in the (k', j) loop is uniform: one branch per pair
        const bool first = ks == 0 && j == 0;
        // in groups of GA elements, every load of a group issued before any of its stores: the
        // compiler cannot tell the accumulator's stores from the multiplier's loads, so one
        // element at a time would cost two memory round trips each
        auto mac = [&](auto load_acc) {
          constexpr bool LOAD = decltype(load_acc)::value;
          constexpr int GA = 4;
          static_assert(N % GA == 0, "accumulator groups");
          static_for<N / GA>([&](auto gg) {
            constexpr int C0 = decltype(gg)::value * GA;
            c128 mv[GA], av[GA];
            static_for<GA>([&](auto q) {
              constexpr int m1 = C0 + decltype(q)::value;
              mv[decltype(q)::value] = ld_c128(rM, voff, (unsigned)(m1 * NTI * 16));
              if constexpr (LOAD && m1 >= AR + AL) av[decltype(q)::value] = ld_c128(rAcc, voff_t16, (unsigned)(m1 * NTI * 16));
            });
            __builtin_amdgcn_sched_barrier(0);
            static_for<GA>([&](auto q) {
              constexpr int m1 = C0 + decltype(q)::value;
              const unsigned so = (unsigned)(m1 * NTI * 16);
              c128 tot = cmul(mv[decltype(q)::value], v[m1]);
              if constexpr (m1 < AR) {
                accr[m1] = LOAD ? accr[m1] + tot : tot;
              } else if constexpr (m1 < AR + AL) {
                c128& slot = lds_acc[(m1 - AR) * NTI + t];
                slot = LOAD ? slot + tot : tot;
              } else {
                if constexpr (LOAD) tot = av[decltype(q)::value] + tot;
                st_c128(tot, rAcc, voff_t16, so);
              }
            });
          });
        };
        if (first) mac(std::false_type{});
        else mac(std::true_type{});
      }
    }
  }
  // out = scale * sum (+ out)
#pragma unroll
  for (int m1 = 0; m1 < N; ++m1) {
    const unsigned so = (unsigned)(m1 * NTI * 16);
    c128 sum;
    if constexpr (ACCREG) sum = acc[m1];
    else if (m1 < AR) sum = accr[m1 < AR ? m1 : 0];
    else if (m1 < AR + AL) sum = lds_acc[(m1 - AR) * NTI + t];
    else sum = ld_c128(rAcc, voff_t16, so);
    c128 o = cscale(sum, a.scale);
    if (a.accumulate) o = ld_c128(rOut, voff, so) + o;
    st_c128(o, rOut, voff, so);
  }
}

template <int N>
__global__ void __launch_bounds__(N * N) fused64_apply_kernel(Fused64Args a) {
  __shared__ c128 lds[f64_lds_elems<N>()];
  __shared__ c128 lds_acc[f64_acc_lds<N>() > 0 ? f64_acc_lds<N>() * N * N : 1];
  static_assert((f64_lds_elems<N>() + f64_acc_lds<N>() * N * N) * 16 <= 160 * 1024, "LDS of the fused FP64 kernel");
  int b = blockIdx.x;
  if (a.xcd_map) {
    // workgroups go round-robin over the 8 XCDs; give each XCD a contiguous run of targets
    const int nwg = gridDim.x;
    const int q = nwg / 8, rem = nwg % 8;
    const int x = b % 8, r = b / 8;
    b = x * q + (x < rem ? x : rem) + r;
  }
  f64_item<N>(a, a.item0 + b, blockIdx.x, lds, lds_acc);
}

template <int N>
hipError_t launch64(const Fused64Args& a, hipStream_t st) {
  hipLaunchKernelGGL(fused64_apply_kernel<N>, dim3(a.nitems), dim3(N * N), 0, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fused64_apply(int n, const Fused64Args& a, hipStream_t st) {
  switch (n) {
    case 16: return launch64<16>(a, st);
    case 20: return launch64<20>(a, st);
    case 24: return launch64<24>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fockmi
