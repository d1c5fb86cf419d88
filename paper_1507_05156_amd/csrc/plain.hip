// Plain path: the steps of Eq. (15) one kernel at a time, through HBM.
//
//   pair product  rho = conj(u_jk') * phi_ik      (launch_pair_product)
//   forward DFT   along n1, n2, n3               (launch_fft3_plain, sign -1)
//   kernel        rho_hat *= K_{k-k'} / N_r       (launch_kernel_mul)
//   inverse DFT   along n3, n2, n1               (launch_fft3_plain, sign +1)
//   accumulate    out_ik += scale * sum u_jk' W   (launch_mac)
//
// The pair batch holds complex128 values (the FP64 path) or complex64 values
// (the FP32 form on grids that are not cubic: the inputs are rounded to FP32
// as the pair product reads them, the product and both transforms run in FP32,
// and the multiply-accumulate widens W to FP64 and sums in FP64).
//
// Each FFT pass gives one thread one grid line, transformed in registers.
// Lines along n1 and n2 are strided, so neighbouring lanes take neighbouring
// lines and every load is coalesced; lines along n3 are contiguous and are
// staged through LDS so that the global loads stay coalesced.
#include "kernels.hpp"

namespace fockmi {

namespace {

// pair p = ((tb * nkb + kb) * nb + j) * nx + s of the batch: target k-point kt0 + tb,
// source k-point ks0 + kb, band j, target field s
template <typename T>
__global__ void pair_product_kernel(cx<T>* __restrict__ batch, const c128* __restrict__ X, const c128* __restrict__ P,
                                    int kt0, int ks0, int nkb, int nb, int nx, int nr, long npairs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  for (long p = blockIdx.y; p < npairs; p += gridDim.y) {
    const int s = (int)(p % nx);
    const long q = p / nx;  // (tb * nkb + kb) * nb + j
    const int j = (int)(q % nb);
    const long tk = q / nb;  // tb * nkb + kb
    const int kb = (int)(tk % nkb), tb = (int)(tk / nkb);
    const c128 x = X[((long)(kt0 + tb) * nx + s) * nr + r];
    const c128 u = P[((long)(ks0 + kb) * nb + j) * nr + r];
    batch[p * nr + r] = cmulc(cx<T>{(T)u.re, (T)u.im}, cx<T>{(T)x.re, (T)x.im});
  }
}

// one thread per line of length N with element stride `inner`; lines are
// enumerated (outer, inner) with base = outer * N * inner + inner_index
template <int N, int SIGN, typename T>
__global__ void __launch_bounds__(64) fft_strided_kernel(cx<T>* __restrict__ data, long nlines, int inner, long field_lines,
                                   long field_elems) {
  const long L = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= nlines) return;
  const long f = L / field_lines;
  const long li = L % field_lines;
  const long base = f * field_elems + (li / inner) * (long)N * inner + (li % inner);
  cx<T> v[N];
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = data[base + (long)i * inner];
  fft<N, SIGN>(v);
#pragma unroll
  for (int i = 0; i < N; ++i) data[base + (long)i * inner] = v[i];
}

constexpr int kContigLines = 64;

template <int N, int SIGN, typename T>
__global__ void __launch_bounds__(kContigLines) fft_contig_kernel(cx<T>* __restrict__ data, long nlines) {
  __shared__ cx<T> tile[kContigLines * (N + 1)];
  const long line0 = (long)blockIdx.x * kContigLines;
  const int tid = threadIdx.x;
  const long avail = nlines - line0;
  const int nl = avail < kContigLines ? (int)avail : kContigLines;
  cx<T>* gbase = data + line0 * N;
  for (int idx = tid; idx < nl * N; idx += kContigLines) {
    const int ln = idx / N, pos = idx % N;
    tile[ln * (N + 1) + pos] = gbase[idx];
  }
  __syncthreads();
  if (tid < nl) {
    cx<T> v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = tile[tid * (N + 1) + i];
    fft<N, SIGN>(v);
#pragma unroll
    for (int i = 0; i < N; ++i) tile[tid * (N + 1) + i] = v[i];
  }
  __syncthreads();
  for (int idx = tid; idx < nl * N; idx += kContigLines) {
    const int ln = idx / N, pos = idx % N;
    gbase[idx] = tile[ln * (N + 1) + pos];
  }
}

template <int N, int SIGN, typename T>
hipError_t strided_pass(cx<T>* data, int nfields, int inner, long field_lines, long field_elems, hipStream_t st) {
  const long nlines = (long)nfields * field_lines;
  const int bs = 64;
  hipLaunchKernelGGL((fft_strided_kernel<N, SIGN, T>), dim3((unsigned)((nlines + bs - 1) / bs)), dim3(bs), 0, st,
                     data, nlines, inner, field_lines, field_elems);
  return hipGetLastError();
}

template <int SIGN, typename T>
hipError_t strided_dispatch(int n, cx<T>* data, int nfields, int inner, long field_lines, long field_elems,
                            hipStream_t st) {
  switch (n) {
    case 16: return strided_pass<16, SIGN, T>(data, nfields, inner, field_lines, field_elems, st);
    case 20: return strided_pass<20, SIGN, T>(data, nfields, inner, field_lines, field_elems, st);
    case 24: return strided_pass<24, SIGN, T>(data, nfields, inner, field_lines, field_elems, st);
    case 32: return strided_pass<32, SIGN, T>(data, nfields, inner, field_lines, field_elems, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int SIGN, typename T>
hipError_t contig_pass(cx<T>* data, long nlines, hipStream_t st) {
  hipLaunchKernelGGL((fft_contig_kernel<N, SIGN, T>), dim3((unsigned)((nlines + kContigLines - 1) / kContigLines)),
                     dim3(kContigLines), 0, st, data, nlines);
  return hipGetLastError();
}

template <int SIGN, typename T>
hipError_t contig_dispatch(int n, cx<T>* data, long nlines, hipStream_t st) {
  switch (n) {
    case 16: return contig_pass<16, SIGN, T>(data, nlines, st);
    case 20: return contig_pass<20, SIGN, T>(data, nlines, st);
    case 24: return contig_pass<24, SIGN, T>(data, nlines, st);
    case 32: return contig_pass<32, SIGN, T>(data, nlines, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
__global__ void kernel_mul_kernel(cx<T>* __restrict__ batch, const double* __restrict__ K,
                                  const int* __restrict__ qidx, int kt0, int nk, int ks0, int nkb, int per_kb, int nr,
                                  long npairs) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nr) return;
  for (long p = blockIdx.y; p < npairs; p += gridDim.y) {
    const long tk = p / per_kb;  // tb * nkb + kb
    const int kb = (int)(tk % nkb), tb = (int)(tk / nkb);
    const T kv = (T)K[(long)qidx[(long)(kt0 + tb) * nk + ks0 + kb] * nr + l];
    cx<T> v = batch[p * nr + l];
    v.re *= kv;
    v.im *= kv;
    batch[p * nr + l] = v;
  }
}

// out[kt0 + tb][s] = (accumulate ? out : 0) + scale * sum_{kb, j} M[ks0 + kb][j] W[tb][kb][j][s], in FP64
template <typename T>
__global__ void mac_kernel(c128* __restrict__ out, const cx<T>* __restrict__ batch, const c128* __restrict__ M,
                           int kt0, int ntb, int ks0, int nkb, int nb, int nx, int nr, double scale, int accumulate) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  for (int ts = blockIdx.y; ts < ntb * nx; ts += gridDim.y) {
    const int tb = ts / nx, s = ts % nx;
    double are = 0.0, aim = 0.0;
    for (int kb = 0; kb < nkb; ++kb) {
      for (int j = 0; j < nb; ++j) {
        const c128 m = M[((long)(ks0 + kb) * nb + j) * nr + r];
        const cx<T> w0 = batch[((((long)tb * nkb + kb) * nb + j) * nx + s) * nr + r];
        const c128 w{(double)w0.re, (double)w0.im};
        are += m.re * w.re - m.im * w.im;
        aim += m.re * w.im + m.im * w.re;
      }
    }
    c128* o = out + ((long)(kt0 + tb) * nx + s) * nr + r;
    c128 v = accumulate ? *o : c128{0.0, 0.0};
    v.re += scale * are;
    v.im += scale * aim;
    *o = v;
  }
}

unsigned grid_y(long n) { return (unsigned)(n < 65535 ? n : 65535); }

}  // namespace

template <typename T>
hipError_t launch_pair_product(cx<T>* batch, const c128* X, const c128* P, int kt0, int ntb, int ks0, int nkb, int nb,
                               int nx, int nr, hipStream_t st) {
  const long np = (long)ntb * nkb * nb * nx;
  dim3 grid((unsigned)((nr + 255) / 256), grid_y(np));
  hipLaunchKernelGGL(pair_product_kernel<T>, grid, dim3(256), 0, st, batch, X, P, kt0, ks0, nkb, nb, nx, nr, np);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft3_plain(cx<T>* data, int nfields, const Geom& g, int sign, hipStream_t st) {
  const long fe = (long)g.n1 * g.n2 * g.n3;
  hipError_t e = hipSuccess;
  // axis 1 (stride n2*n3): lines (m2, m3); axis 2 (stride n3): lines (m1, m3); axis 3 contiguous
  auto ax1 = [&](int s) {
    return s < 0 ? strided_dispatch<-1, T>(g.n1, data, nfields, g.n2 * g.n3, (long)g.n2 * g.n3, fe, st)
                 : strided_dispatch<+1, T>(g.n1, data, nfields, g.n2 * g.n3, (long)g.n2 * g.n3, fe, st);
  };
  auto ax2 = [&](int s) {
    return s < 0 ? strided_dispatch<-1, T>(g.n2, data, nfields, g.n3, (long)g.n1 * g.n3, fe, st)
                 : strided_dispatch<+1, T>(g.n2, data, nfields, g.n3, (long)g.n1 * g.n3, fe, st);
  };
  auto ax3 = [&](int s) {
    const long nl = (long)nfields * g.n1 * g.n2;
    return s < 0 ? contig_dispatch<-1, T>(g.n3, data, nl, st) : contig_dispatch<+1, T>(g.n3, data, nl, st);
  };
  if (sign < 0) {
    if ((e = ax1(-1)) != hipSuccess) return e;
    if ((e = ax2(-1)) != hipSuccess) return e;
    return ax3(-1);
  }
  if ((e = ax3(+1)) != hipSuccess) return e;
  if ((e = ax2(+1)) != hipSuccess) return e;
  return ax1(+1);
}

template <typename T>
hipError_t launch_kernel_mul(cx<T>* batch, const double* K, const int* qidx, int kt0, int ntb, int nk, int ks0,
                             int nkb, int per_kb, int nr, hipStream_t st) {
  const long np = (long)ntb * nkb * per_kb;
  dim3 grid((unsigned)((nr + 255) / 256), grid_y(np));
  hipLaunchKernelGGL(kernel_mul_kernel<T>, grid, dim3(256), 0, st, batch, K, qidx, kt0, nk, ks0, nkb, per_kb, nr, np);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mac(c128* out, const cx<T>* batch, const c128* M, int kt0, int ntb, int ks0, int nkb, int nb, int nx,
                      int nr, double scale, int accumulate, hipStream_t st) {
  dim3 grid((unsigned)((nr + 255) / 256), grid_y((long)ntb * nx));
  hipLaunchKernelGGL(mac_kernel<T>, grid, dim3(256), 0, st, out, batch, M, kt0, ntb, ks0, nkb, nb, nx, nr, scale,
                     accumulate);
  return hipGetLastError();
}

#define FOCKMI_PLAIN_INSTANTIATE(T)                                                                              \
  template hipError_t launch_pair_product<T>(cx<T>*, const c128*, const c128*, int, int, int, int, int, int, int,    \
                                             hipStream_t);                                                         \
  template hipError_t launch_fft3_plain<T>(cx<T>*, int, const Geom&, int, hipStream_t);                            \
  template hipError_t launch_kernel_mul<T>(cx<T>*, const double*, const int*, int, int, int, int, int, int, int,     \
                                           hipStream_t);                                                           \
  template hipError_t launch_mac<T>(c128*, const cx<T>*, const c128*, int, int, int, int, int, int, int, double, int, \
                                    hipStream_t);
FOCKMI_PLAIN_INSTANTIATE(double)
FOCKMI_PLAIN_INSTANTIATE(float)
#undef FOCKMI_PLAIN_INSTANTIATE

}  // namespace fockmi
