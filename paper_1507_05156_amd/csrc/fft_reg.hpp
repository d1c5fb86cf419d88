// In-register mixed-radix FFTs for one thread (lengths built from 2, 3, 4, 5).
// Lengths with an odd factor use the prime-factor mapping at the top level.
//
// Every loop below runs over compile-time indices (static_for), so after
// inlining each array element is a named register and every twiddle factor is
// an immediate constant; no twiddle table is read at run time.
//
// Forward transform (SIGN = -1):  X[l] = sum_m x[m] exp(-2 pi i l m / N)
// Inverse transform (SIGN = +1):  x[m] = sum_l X[l] exp(+2 pi i l m / N)  (unnormalised)
// Input and output are both in natural order.
#pragma once

// FOCKMI_FFT_HOST_CHECK builds only the arithmetic (complex type, twiddles,
// transforms) as plain host C++, for the CPU test that compares the
// transforms with a direct DFT; the build of the library never defines it.
#ifdef FOCKMI_FFT_HOST_CHECK
#define __device__
#define __forceinline__ inline
#else
#include <hip/hip_runtime.h>
#endif

#include <type_traits>
#include <utility>

namespace fockmi {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T re, T im) { return cx<T>{re, im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc + a * b with each product term fused into the accumulator: two
// multiply-adds per component, against three for acc + cmul(a, b)
template <typename T>
__device__ __forceinline__ cx<T> cmac(cx<T> acc, cx<T> a, cx<T> b) {
  return {fmadd(-a.im, b.im, fmadd(a.re, b.re, acc.re)), fmadd(a.im, b.re, fmadd(a.re, b.im, acc.im))};
}
// multiply by s * i with s = +-1
template <int S, typename T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a) {
  if constexpr (S > 0) return {-a.im, a.re};
  else return {a.im, -a.re};
}

#ifndef FOCKMI_FFT_HOST_CHECK
// ------------------------------------------------------------ buffer access
// Raw buffer loads/stores: a uniform 128-bit resource (base pointer, size in
// bytes) plus one per-thread byte offset and a uniform byte offset. Every load
// of a thread shares one offset register; accesses past the size read zero and
// stores past it are dropped.
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ cx<float> ld_c64(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void st_c64(cx<float> v, rsrc_t r, unsigned voff, unsigned soff) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, soff, 0);
}
__device__ __forceinline__ float ld_f32(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ cx<double> ld_c128(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
// A complex128 is stored as two 64-bit buffer stores. A 128-bit buffer store
// whose offset comes from an SGPR, with its data VGPRs rewritten by the next
// VALU instructions, was seen to write wrong data now and then (no wait states
// are inserted for that form); 64-bit stores carry no such hazard.
__device__ __forceinline__ void st_c128(cx<double> v, rsrc_t r, unsigned voff, unsigned soff) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v.re), r, voff, soff, 0);
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v.im), r, voff + 8u, soff, 0);
}

#endif  // FOCKMI_FFT_HOST_CHECK

// ---------------------------------------------------------------- static_for
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ------------------------------------------------- compile-time trigonometry
// cos and sin of 2 pi p / q for integers, evaluated in double at compile time.
// The angle is reduced exactly in integers to base * (pi/2) + phi with
// |phi| <= pi/4, and the Taylor series is summed for phi (error < 1e-19).
namespace ct {
constexpr double kQuarterPi = 0.78539816339744830961566084581987572;
constexpr double sin_series(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
struct CS {
  double c, s;
};
constexpr CS cis(long p, long q) {
  p %= q;
  if (p < 0) p += q;
  const long e8 = 8 * p;
  const long oct = e8 / q;        // octant 0..7
  const long rem = e8 - oct * q;  // 0 <= rem < q
  long base = 0;
  double phi = 0.0;
  if (oct % 2 == 0) {
    base = oct / 2;
    phi = kQuarterPi * (double)rem / (double)q;
  } else {
    base = (oct + 1) / 2;
    phi = -kQuarterPi * (double)(q - rem) / (double)q;
  }
  const double c = (rem == 0 && oct % 2 == 0) ? 1.0 : cos_series(phi);
  const double s = (rem == 0 && oct % 2 == 0) ? 0.0 : sin_series(phi);
  switch (base % 4) {
    case 0: return {c, s};
    case 1: return {-s, c};
    case 2: return {-c, -s};
    default: return {s, -c};
  }
}
}  // namespace ct

// x * exp(SIGN * 2 pi i E / N), with the trivial angles special-cased
template <int N, int SIGN, int E, typename T>
__device__ __forceinline__ cx<T> twiddle(cx<T> x) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0) {
    return x;
  } else if constexpr ((4 * e) % N == 0) {
    constexpr int quarter = (4 * e) / N;  // 1, 2, 3
    if constexpr (quarter == 2) return {-x.re, -x.im};
    else if constexpr (quarter == 1) return mul_si<SIGN>(x);
    else return mul_si<-SIGN>(x);
  } else if constexpr ((8 * e) % N == 0) {
    constexpr ct::CS w = ct::cis(e, N);
    constexpr T h = (T)0.70710678118654752440084436210484904;
    constexpr T cr = w.c > 0 ? h : -h;
    constexpr T si = (SIGN > 0 ? 1 : -1) * (w.s > 0 ? 1 : -1) * (double)h;
    return {cr * x.re - si * x.im, cr * x.im + si * x.re};
  } else {
    constexpr ct::CS w = ct::cis(e, N);
    constexpr T c = (T)w.c;
    constexpr T s = (T)((SIGN > 0 ? 1.0 : -1.0) * w.s);
    return {c * x.re - s * x.im, c * x.im + s * x.re};
  }
}

// A twiddled value x * w, w = exp(SIGN * 2 pi i E / N), as m * u: m is a
// compile-time real factor (the larger of |Re w|, |Im w|, with its sign; 1
// for the trivial angles) and u = x * (w / m) costs at most two fused
// multiply-adds, since one component of w / m is exactly 1. The butterflies
// below fold m into their own multiply-adds (after Linzer and Feig's
// FMA-oriented radix-2 and radix-4 FFTs), so a twiddle costs two
// instructions instead of four.
template <int N, int SIGN, int E>
struct tw_split {
  static constexpr int e = ((E % N) + N) % N;
  static constexpr bool trivial = (4 * e) % N == 0;
  static constexpr bool eighth = !trivial && (8 * e) % N == 0;
  static constexpr ct::CS w = ct::cis(e, N);
  static constexpr double c = w.c;
  static constexpr double s = SIGN > 0 ? w.s : -w.s;
  static constexpr bool cos_major = (c < 0 ? -c : c) >= (s < 0 ? -s : s);
  static constexpr double m = trivial ? 1.0 : (cos_major ? c : s);
};
template <int N, int SIGN, int E, typename T>
__device__ __forceinline__ cx<T> tw_unit(cx<T> x) {
  using S = tw_split<N, SIGN, E>;
  if constexpr (S::trivial) {
    return twiddle<N, SIGN, E>(x);
  } else if constexpr (S::eighth) {
    // w / m = 1 + i sigma with sigma = +-1 exactly
    if constexpr ((S::c > 0) == (S::s > 0)) return {x.re - x.im, x.im + x.re};
    else return {x.re + x.im, x.im - x.re};
  } else if constexpr (S::cos_major) {
    constexpr T t = (T)(S::s / S::c);  // w / m = 1 + i t
    return {x.re - t * x.im, x.im + t * x.re};
  } else {
    constexpr T t = (T)(S::c / S::s);  // w / m = t + i
    return {t * x.re - x.im, t * x.im + x.re};
  }
}

// --------------------------------------------------------------- base DFTs
template <int R, int SIGN, typename T>
__device__ __forceinline__ void dft_base(cx<T> (&x)[R]) {
  static_assert(R == 2 || R == 3 || R == 4 || R == 5, "base radix");
  if constexpr (R == 2) {
    const cx<T> a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  } else if constexpr (R == 3) {
    constexpr T h = (T)0.5;
    constexpr T s3 = (T)(SIGN * 0.86602540378443864676372317075293618);
    const cx<T> t1 = x[1] + x[2];
    const cx<T> t2 = {x[0].re - h * t1.re, x[0].im - h * t1.im};
    const cx<T> d = x[1] - x[2];
    const cx<T> t3 = {-s3 * d.im, s3 * d.re};  // i * s3 * d
    x[0] = x[0] + t1;
    x[1] = t2 + t3;
    x[2] = t2 - t3;
  } else if constexpr (R == 4) {
    const cx<T> a = x[0] + x[2], b = x[0] - x[2];
    const cx<T> c = x[1] + x[3], d = mul_si<SIGN>(x[1] - x[3]);
    x[0] = a + c;
    x[2] = a - c;
    x[1] = b + d;
    x[3] = b - d;
  } else {
    constexpr T c1 = (T)0.30901699437494742410229341718281906;   // cos(2pi/5)
    constexpr T c2 = (T)-0.80901699437494742410229341718281906;  // cos(4pi/5)
    constexpr T s1 = (T)(SIGN * 0.95105651629515357211643933337938214);  // sin(2pi/5)
    constexpr T s2 = (T)(SIGN * 0.58778525229247312916870595463907277);  // sin(4pi/5)
    const cx<T> a1 = x[1] + x[4], b1 = x[1] - x[4];
    const cx<T> a2 = x[2] + x[3], b2 = x[2] - x[3];
    const cx<T> x0 = x[0];
    const cx<T> r1 = {x0.re + c1 * a1.re + c2 * a2.re, x0.im + c1 * a1.im + c2 * a2.im};
    const cx<T> r2 = {x0.re + c2 * a1.re + c1 * a2.re, x0.im + c2 * a1.im + c1 * a2.im};
    // i * (s1 b1 + s2 b2) and i * (s2 b1 - s1 b2)
    const cx<T> i1 = {-(s1 * b1.im + s2 * b2.im), s1 * b1.re + s2 * b2.re};
    const cx<T> i2 = {-(s2 * b1.im - s1 * b2.im), s2 * b1.re - s1 * b2.re};
    x[0] = x0 + a1 + a2;
    x[1] = r1 + i1;
    x[4] = r1 - i1;
    x[2] = r2 + i2;
    x[3] = r2 - i2;
  }
}

// N = A * B with A the largest power of two dividing N: when both parts
// exceed 1 they are coprime, and the prime-factor (Good-Thomas) mapping
// applies: n = (B n1 + A n2) mod N on input, k = CRT(k mod A, k mod B) on
// output, with no twiddle factors between the A- and B-point transforms.
template <int N>
constexpr int pow2_part() {
  int a = 1;
  while ((N / a) % 2 == 0) a *= 2;
  return a;
}
template <int A, int B>
constexpr int crt_index(int k1, int k2) {
  for (int k = 0; k < A * B; ++k)
    if (k % A == k1 && k % B == k2) return k;
  return -1;
}

template <int N>
constexpr int first_radix() {
  if constexpr (N % 4 == 0) return 4;
  else if constexpr (N % 2 == 0) return 2;
  else if constexpr (N % 3 == 0) return 3;
  else return 5;
}

// Whether a transform of length N folds its twiddle factors into the radix-2
// and radix-4 butterflies (tw_split). The 32-point transform keeps plain
// twiddle multiplies throughout: the 32^3 pair kernel has fewer instructions
// with folding but ran slower in its paced persistent form.
template <int N>
constexpr bool fold_default() { return N != 32; }

// Decimation in time: N = R * M. The M-point transforms of the R
// subsequences x[R m + r] are combined by R-point transforms after twiddling.
template <int N, int SIGN, bool FOLD = fold_default<N>(), typename T>
__device__ __forceinline__ void fft(cx<T> (&x)[N]) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N == 2 || N == 3 || N == 4 || N == 5) {
    dft_base<N, SIGN>(x);
  } else if constexpr (pow2_part<N>() > 1 && pow2_part<N>() < N) {
    // prime-factor algorithm: B-point transforms of the A interleaved
    // subsequences, then A-point transforms across them
    constexpr int A = pow2_part<N>();
    constexpr int B = N / A;
    cx<T> z[A][B];
    static_for<A>([&](auto n1) {
      constexpr int a1 = decltype(n1)::value;
      static_for<B>([&](auto n2) {
        constexpr int b2 = decltype(n2)::value;
        z[a1][b2] = x[(a1 * B + b2 * A) % N];
      });
      fft<B, SIGN, FOLD>(z[a1]);
    });
    static_for<B>([&](auto k2) {
      constexpr int kb = decltype(k2)::value;
      cx<T> w[A];
      static_for<A>([&](auto n1) { w[decltype(n1)::value] = z[decltype(n1)::value][kb]; });
      fft<A, SIGN, FOLD>(w);
      static_for<A>([&](auto k1) {
        constexpr int ka = decltype(k1)::value;
        x[crt_index<A, B>(ka, kb)] = w[ka];
      });
    });
  } else {
    constexpr int R = first_radix<N>();
    constexpr int M = N / R;
    static_assert(R * M == N, "lengths are products of 2, 3, 5");
    cx<T> y[R][M];
    static_for<R>([&](auto r) {
      constexpr int rr = decltype(r)::value;
      static_for<M>([&](auto m) {
        constexpr int mm = decltype(m)::value;
        y[rr][mm] = x[mm * R + rr];
      });
      fft<M, SIGN, FOLD>(y[rr]);
    });
    static_for<M>([&](auto k1) {
      constexpr int kk = decltype(k1)::value;
      if constexpr (R == 2 && FOLD) {
        constexpr T m1 = (T)tw_split<N, SIGN, kk>::m;
        const cx<T> y0 = y[0][kk];
        const cx<T> u1 = tw_unit<N, SIGN, kk>(y[1][kk]);
        x[kk] = {y0.re + m1 * u1.re, y0.im + m1 * u1.im};
        x[kk + M] = {y0.re - m1 * u1.re, y0.im - m1 * u1.im};
      } else if constexpr (R == 4 && FOLD) {
        // z_r = m_r u_r; z1 + z3 and z1 - z3 are m1 (u1 +- (m3/m1) u3)
        constexpr double m1d = tw_split<N, SIGN, kk>::m;
        constexpr T m1 = (T)m1d;
        constexpr T m2 = (T)tw_split<N, SIGN, 2 * kk>::m;
        constexpr T rho = (T)(tw_split<N, SIGN, 3 * kk>::m / m1d);
        const cx<T> y0 = y[0][kk];
        const cx<T> u1 = tw_unit<N, SIGN, kk>(y[1][kk]);
        const cx<T> u2 = tw_unit<N, SIGN, 2 * kk>(y[2][kk]);
        const cx<T> u3 = tw_unit<N, SIGN, 3 * kk>(y[3][kk]);
        const cx<T> a = {y0.re + m2 * u2.re, y0.im + m2 * u2.im};
        const cx<T> b = {y0.re - m2 * u2.re, y0.im - m2 * u2.im};
        const cx<T> c = {u1.re + rho * u3.re, u1.im + rho * u3.im};
        const cx<T> d = mul_si<SIGN>(cx<T>{u1.re - rho * u3.re, u1.im - rho * u3.im});
        x[kk] = {a.re + m1 * c.re, a.im + m1 * c.im};
        x[kk + 2 * M] = {a.re - m1 * c.re, a.im - m1 * c.im};
        x[kk + M] = {b.re + m1 * d.re, b.im + m1 * d.im};
        x[kk + 3 * M] = {b.re - m1 * d.re, b.im - m1 * d.im};
      } else {
        cx<T> z[R];
        static_for<R>([&](auto r) {
          constexpr int rr = decltype(r)::value;
          z[rr] = twiddle<N, SIGN, rr * kk>(y[rr][kk]);
        });
        dft_base<R, SIGN>(z);
        static_for<R>([&](auto k2) {
          constexpr int k2v = decltype(k2)::value;
          x[kk + M * k2v] = z[k2v];
        });
      }
    });
  }
}

}  // namespace fockmi
