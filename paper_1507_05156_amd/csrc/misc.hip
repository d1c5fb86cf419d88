// Small FP64 helpers: complex64 shadows, a deterministic double-double inner product, axpy.
#include "kernels.hpp"

namespace fockmi {

namespace {

__global__ void to_c64_kernel(c64* __restrict__ dst, const c128* __restrict__ src, long count) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    const c128 v = src[i];
    dst[i] = c64{(float)v.re, (float)v.im};
  }
}

constexpr int kDotThreads = 256;

// Double-double accumulation (hi + lo, |lo| <= ulp(hi)/2): x is added to hi with an
// error-free two-sum whose rounding error goes into lo. Products enter with their
// exact rounding error from an FMA, so the sums are accurate to a few units of
// 2^-104 relative: a difference of two nearby energies keeps its digits.
struct dd {
  double hi, lo;
};
__device__ __forceinline__ void dd_add(dd& a, double x) {
#pragma clang fp contract(off)
  const double s = a.hi + x;
  const double bb = s - a.hi;
  const double err = (a.hi - (s - bb)) + (x - bb);
  a.hi = s;
  a.lo += err;
}
__device__ __forceinline__ void dd_add(dd& a, dd b) {
#pragma clang fp contract(off)
  dd_add(a, b.hi);
  a.lo += b.lo;
}
// a += x * y, exactly up to the final rounding of the two parts
__device__ __forceinline__ void dd_add_prod(dd& a, double x, double y) {
#pragma clang fp contract(off)
  const double p = x * y;
  const double e = fma(x, y, -p);
  dd_add(a, p);
  a.lo += e;
}

// partial[4 b .. 4 b + 3] = (re.hi, re.lo, im.hi, im.lo) of sum conj(a) b over a fixed
// grid-stride slice, tree-reduced in a fixed order
__global__ void __launch_bounds__(kDotThreads) dot_partial_kernel(double* __restrict__ partial,
                                                                  const c128* __restrict__ a,
                                                                  const c128* __restrict__ b, long count) {
  __shared__ dd sre[kDotThreads], sim[kDotThreads];
  dd re{0.0, 0.0}, im{0.0, 0.0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    const c128 x = a[i], y = b[i];
    dd_add_prod(re, x.re, y.re);
    dd_add_prod(re, x.im, y.im);
    dd_add_prod(im, x.re, y.im);
    dd_add_prod(im, -x.im, y.re);
  }
  sre[threadIdx.x] = re;
  sim[threadIdx.x] = im;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      dd_add(sre[threadIdx.x], sre[threadIdx.x + w]);
      dd_add(sim[threadIdx.x], sim[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[4 * blockIdx.x + 0] = sre[0].hi;
    partial[4 * blockIdx.x + 1] = sre[0].lo;
    partial[4 * blockIdx.x + 2] = sim[0].hi;
    partial[4 * blockIdx.x + 3] = sim[0].lo;
  }
}

__global__ void __launch_bounds__(kDotThreads) dot_final_kernel(double* __restrict__ dst,
                                                                const double* __restrict__ partial, int nblk) {
  __shared__ dd sre[kDotThreads], sim[kDotThreads];
  dd re{0.0, 0.0}, im{0.0, 0.0};
  for (int i = threadIdx.x; i < nblk; i += kDotThreads) {
    dd_add(re, dd{partial[4 * i + 0], partial[4 * i + 1]});
    dd_add(im, dd{partial[4 * i + 2], partial[4 * i + 3]});
  }
  sre[threadIdx.x] = re;
  sim[threadIdx.x] = im;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      dd_add(sre[threadIdx.x], sre[threadIdx.x + w]);
      dd_add(sim[threadIdx.x], sim[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    dst[0] = sre[0].hi;
    dst[1] = sre[0].lo;
    dst[2] = sim[0].hi;
    dst[3] = sim[0].lo;
  }
}

__global__ void zero_kernel(c128* __restrict__ y, long count) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
    y[i] = c128{0.0, 0.0};
}

__global__ void scale_add_kernel(c128* __restrict__ y, const c128* __restrict__ x, double sre, double sim,
                                 long count) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    const c128 v = x[i];
    c128 o = y[i];
    o.re += sre * v.re - sim * v.im;
    o.im += sre * v.im + sim * v.re;
    y[i] = o;
  }
}

unsigned grid_for(long count, int bs) {
  long g = (count + bs - 1) / bs;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_to_c64(c64* dst, const c128* src, long count, hipStream_t st) {
  hipLaunchKernelGGL(to_c64_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, dst, src, count);
  return hipGetLastError();
}

hipError_t launch_dot(double* dst, double* partial, int nblk, const c128* a, const c128* b, long count,
                      hipStream_t st) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nblk), dim3(kDotThreads), 0, st, partial, a, b, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kDotThreads), 0, st, dst, partial, nblk);
  return hipGetLastError();
}

hipError_t launch_zero(c128* y, long count, hipStream_t st) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, y, count);
  return hipGetLastError();
}

hipError_t launch_scale_add(c128* y, const c128* x, double sre, double sim, long count, hipStream_t st) {
  hipLaunchKernelGGL(scale_add_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, y, x, sre, sim, count);
  return hipGetLastError();
}

}  // namespace fockmi
