// Host build of the register FFTs (fft_reg.hpp with FOCKMI_FFT_HOST_CHECK):
// every length the kernels use, and a few more, both signs, with and without
// twiddle folding, in double and float, against a direct DFT summed in long
// double. Prints one line per case: N SIGN FOLD TYPE ERR, where ERR is the
// largest error over the outputs divided by the input's 2-norm (double) or the
// relative 2-norm error over many random inputs (float).
#include <cmath>
#include <complex>
#include <cstdio>

#include "fft_reg.hpp"

using namespace fockmi;
using cld = std::complex<long double>;

static unsigned lcg(unsigned& s) { return s = s * 1103515245u + 12345u; }
static double uni(unsigned& s) { return (lcg(s) >> 8) / 16777216.0 - 0.5; }

template <int N, int SIGN>
static void dft(const cld* in, cld* out) {
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int k = 0; k < N; ++k) {
    out[k] = 0;
    for (int m = 0; m < N; ++m) {
      const long double ang = SIGN * 2 * pi * (long double)((long)k * m % N) / N;
      out[k] += in[m] * cld(cosl(ang), sinl(ang));
    }
  }
}

template <int N, int SIGN, bool FOLD>
static double err_double() {
  unsigned s = 1000u + 7u * N + (SIGN > 0);
  double worst = 0;
  for (int trial = 0; trial < 64; ++trial) {
    cx<double> x[N];
    cld in[N], ref[N];
    long double nrm = 0;
    for (int i = 0; i < N; ++i) {
      x[i] = {uni(s), uni(s)};
      in[i] = cld(x[i].re, x[i].im);
      nrm += std::norm(in[i]);
    }
    dft<N, SIGN>(in, ref);
    fft<N, SIGN, FOLD>(x);
    for (int k = 0; k < N; ++k)
      worst = std::fmax(worst, (double)(std::abs(cld(x[k].re, x[k].im) - ref[k]) / sqrtl(nrm)));
  }
  return worst;
}

template <int N, int SIGN, bool FOLD>
static double err_float() {
  unsigned s = 2000u + 7u * N + (SIGN > 0);
  long double num = 0, den = 0;
  for (int trial = 0; trial < 500; ++trial) {
    cx<float> x[N];
    cld in[N], ref[N];
    for (int i = 0; i < N; ++i) {
      x[i] = {(float)uni(s), (float)uni(s)};
      in[i] = cld(x[i].re, x[i].im);
    }
    dft<N, SIGN>(in, ref);
    fft<N, SIGN, FOLD>(x);
    for (int k = 0; k < N; ++k) {
      num += std::norm(cld(x[k].re, x[k].im) - ref[k]);
      den += std::norm(ref[k]);
    }
  }
  return (double)sqrtl(num / den);
}

template <int N, int SIGN, bool FOLD>
static void one() {
  std::printf("%d %d %d f64 %.6e\n", N, SIGN, (int)FOLD, err_double<N, SIGN, FOLD>());
  std::printf("%d %d %d f32 %.6e\n", N, SIGN, (int)FOLD, err_float<N, SIGN, FOLD>());
}

template <int N>
static void all() {
  one<N, -1, false>();
  one<N, +1, false>();
  one<N, -1, true>();
  one<N, +1, true>();
}

int main() {
  all<2>();
  all<3>();
  all<4>();
  all<5>();
  all<6>();
  all<8>();
  all<10>();
  all<12>();
  all<16>();
  all<20>();
  all<24>();
  all<32>();
  all<40>();
  all<48>();
  return 0;
}
