// Device kernels of the propagator and orthonormalisation (FP64).
//
// Kinetic operator of the velocity-gauge Hamiltonian (Eq. (2)) on the periodic
// parts: T[a] u = IDFT( |k + G_l + a|^2 / 2 * DFT u ) / N_r with G_l in FFT
// order (l = -n/2 on the Nyquist slot) and a = A/c.
#include "kernels.hpp"
#include "prop.hpp"

namespace fockmi {

namespace {

__device__ __forceinline__ void gvec(const Geom& g, long l, double kx, double ky, double kz, double a0, double a1,
                                     double a2, double p[3]) {
  const int j3 = (int)(l % g.n3);
  const int j2 = (int)((l / g.n3) % g.n2);
  const int j1 = (int)(l / ((long)g.n2 * g.n3));
  const double l1 = j1 < (g.n1 + 1) / 2 ? j1 : j1 - g.n1;
  const double l2 = j2 < (g.n2 + 1) / 2 ? j2 : j2 - g.n2;
  const double l3 = j3 < (g.n3 + 1) / 2 ? j3 : j3 - g.n3;
  p[0] = kx + a0 + l1 * g.B[0][0] + l2 * g.B[1][0] + l3 * g.B[2][0];
  p[1] = ky + a1 + l1 * g.B[0][1] + l2 * g.B[1][1] + l3 * g.B[2][1];
  p[2] = kz + a2 + l1 * g.B[0][2] + l2 * g.B[1][2] + l3 * g.B[2][2];
}

// F[k][f][l] *= scale * |k + G_l + a|^2 / 2
__global__ void kinetic_mul_kernel(c128* __restrict__ F, const double* __restrict__ kpts, int nf, Geom g,
                                   double a0, double a1, double a2, double scale) {
  const long nr = (long)g.n1 * g.n2 * g.n3;
  const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int field = blockIdx.y;  // k * nf + f
  if (l >= nr) return;
  const int k = field / nf;
  double p[3];
  gvec(g, l, kpts[3 * k], kpts[3 * k + 1], kpts[3 * k + 2], a0, a1, a2, p);
  const double e = scale * 0.5 * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  c128 v = F[(long)field * nr + l];
  v.re *= e;
  v.im *= e;
  F[(long)field * nr + l] = v;
}

// F[k][f][l] *= scale / (1 + |k + G_l + a|^2 / (2 e0)): the kinetic preconditioner
// of the block eigensolver, damping the plane waves far above the energy e0
__global__ void precond_mul_kernel(c128* __restrict__ F, const double* __restrict__ kpts, int nf, Geom g, double a0,
                                   double a1, double a2, double e0, double scale) {
  const long nr = (long)g.n1 * g.n2 * g.n3;
  const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int field = blockIdx.y;
  if (l >= nr) return;
  const int k = field / nf;
  double p[3];
  gvec(g, l, kpts[3 * k], kpts[3 * k + 1], kpts[3 * k + 2], a0, a1, a2, p);
  const double f = scale / (1.0 + 0.5 * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) / e0);
  c128 v = F[(long)field * nr + l];
  v.re *= f;
  v.im *= f;
  F[(long)field * nr + l] = v;
}

// out = (base ? base : 0) + c * (kin + vloc .* x + alpha * vx)
__global__ void hcombine_kernel(c128* __restrict__ out, const c128* __restrict__ base, const c128* __restrict__ kin,
                                const c128* __restrict__ x, const c128* __restrict__ vx,
                                const double* __restrict__ vloc, double alpha, double cre, double cim, long count,
                                int nr) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    c128 h = kin[i];
    if (vloc) {
      const double v = vloc[i % nr];
      const c128 xi = x[i];
      h.re += v * xi.re;
      h.im += v * xi.im;
    }
    if (vx) {
      const c128 w = vx[i];
      h.re += alpha * w.re;
      h.im += alpha * w.im;
    }
    c128 o = base ? base[i] : c128{0.0, 0.0};
    o.re += cre * h.re - cim * h.im;
    o.im += cre * h.im + cim * h.re;
    out[i] = o;
  }
}

constexpr int kRedThreads = 256;

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh) {
  for (int q = 0; q < NV; ++q) sh[q * kRedThreads + threadIdx.x] = v[q];
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < NV; ++q) sh[q * kRedThreads + threadIdx.x] += sh[q * kRedThreads + threadIdx.x + w];
    __syncthreads();
  }
  for (int q = 0; q < NV; ++q) v[q] = sh[q * kRedThreads];
}

// out[f] = sum_r |psi[f][r]|^2, one block per field, fixed order
__global__ void __launch_bounds__(kRedThreads) norms_kernel(double* __restrict__ out, const c128* __restrict__ psi,
                                                            int nr) {
  __shared__ double sh[kRedThreads];
  const c128* p = psi + (long)blockIdx.x * nr;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < nr; i += kRedThreads) v[0] += p[i].re * p[i].re + p[i].im * p[i].im;
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

// partial[b][0..5] = sum over a grid-stride slice of conj(L) * (k+G+a)_d * F for d = 0, 1, 2 (re, im)
__global__ void __launch_bounds__(kRedThreads) agrad_partial_kernel(double* __restrict__ partial,
                                                                    const c128* __restrict__ L,
                                                                    const c128* __restrict__ F,
                                                                    const double* __restrict__ kpts, int nf,
                                                                    Geom g, double a0, double a1, double a2,
                                                                    long count) {
  __shared__ double sh[6 * kRedThreads];
  const long nr = (long)g.n1 * g.n2 * g.n3;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    const long field = i / nr;
    const long l = i % nr;
    const int k = (int)(field / nf);
    double p[3];
    gvec(g, l, kpts[3 * k], kpts[3 * k + 1], kpts[3 * k + 2], a0, a1, a2, p);
    const c128 x = L[i], y = F[i];
    const double re = x.re * y.re + x.im * y.im;  // conj(x) * y
    const double im = x.re * y.im - x.im * y.re;
    for (int d = 0; d < 3; ++d) {
      v[2 * d] += p[d] * re;
      v[2 * d + 1] += p[d] * im;
    }
  }
  block_sum<6>(v, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < 6; ++q) partial[6 * blockIdx.x + q] = v[q];
}

__global__ void __launch_bounds__(kRedThreads) sum_rows_kernel(double* __restrict__ out,
                                                               const double* __restrict__ partial, int nrows,
                                                               int width) {
  __shared__ double sh[kRedThreads];
  for (int q = 0; q < width; ++q) {
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < nrows; i += kRedThreads) v[0] += partial[(long)i * width + q];
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) out[q] = v[0];
    __syncthreads();
  }
}

// Modified Gram-Schmidt of the nb fields of one k-point (one workgroup per k), cell inner
// product w * sum conj(a) b
constexpr int kMgsThreads = 1024;
__global__ void __launch_bounds__(kMgsThreads) mgs_kernel(c128* __restrict__ psi, int nb, int nr, double w) {
  __shared__ double sh[2 * kMgsThreads];
  c128* base = psi + (long)blockIdx.x * nb * nr;
  const int t = threadIdx.x;
  for (int b = 0; b < nb; ++b) {
    c128* vb = base + (long)b * nr;
    for (int c = 0; c < b; ++c) {
      const c128* vc = base + (long)c * nr;
      double re = 0.0, im = 0.0;
      for (int i = t; i < nr; i += kMgsThreads) {
        const c128 x = vc[i], y = vb[i];
        re += x.re * y.re + x.im * y.im;
        im += x.re * y.im - x.im * y.re;
      }
      sh[t] = re;
      sh[kMgsThreads + t] = im;
      __syncthreads();
      for (int s = kMgsThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
          sh[t] += sh[t + s];
          sh[kMgsThreads + t] += sh[kMgsThreads + t + s];
        }
        __syncthreads();
      }
      const double pr = w * sh[0], pi = w * sh[kMgsThreads];
      __syncthreads();
      for (int i = t; i < nr; i += kMgsThreads) {
        const c128 x = vc[i];
        c128 y = vb[i];
        y.re -= pr * x.re - pi * x.im;
        y.im -= pr * x.im + pi * x.re;
        vb[i] = y;
      }
      __syncthreads();
    }
    double s2 = 0.0;
    for (int i = t; i < nr; i += kMgsThreads) s2 += vb[i].re * vb[i].re + vb[i].im * vb[i].im;
    sh[t] = s2;
    __syncthreads();
    for (int s = kMgsThreads / 2; s > 0; s >>= 1) {
      if (t < s) sh[t] += sh[t + s];
      __syncthreads();
    }
    const double inv = 1.0 / sqrt(w * sh[0]);
    __syncthreads();
    for (int i = t; i < nr; i += kMgsThreads) {
      c128 y = vb[i];
      y.re *= inv;
      y.im *= inv;
      vb[i] = y;
    }
    __syncthreads();
  }
}

unsigned grid_for(long count, int bs) {
  long g = (count + bs - 1) / bs;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_kinetic_mul(c128* F, const double* kpts, int nk, int nf, const Geom& g, const double a[3],
                              double scale, hipStream_t st) {
  const long nr = (long)g.n1 * g.n2 * g.n3;
  dim3 grid((unsigned)((nr + 255) / 256), (unsigned)(nk * nf));
  hipLaunchKernelGGL(kinetic_mul_kernel, grid, dim3(256), 0, st, F, kpts, nf, g, a[0], a[1], a[2], scale);
  return hipGetLastError();
}

hipError_t launch_precond_mul(c128* F, const double* kpts, int nk, int nf, const Geom& g, const double a[3],
                              double e0, double scale, hipStream_t st) {
  const long nr = (long)g.n1 * g.n2 * g.n3;
  dim3 grid((unsigned)((nr + 255) / 256), (unsigned)(nk * nf));
  hipLaunchKernelGGL(precond_mul_kernel, grid, dim3(256), 0, st, F, kpts, nf, g, a[0], a[1], a[2], e0, scale);
  return hipGetLastError();
}

hipError_t launch_hcombine(c128* out, const c128* base, const c128* kin, const c128* x, const c128* vx,
                           const double* vloc, double alpha, double cre, double cim, long count, int nr,
                           hipStream_t st) {
  hipLaunchKernelGGL(hcombine_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, out, base, kin, x, vx, vloc,
                     alpha, cre, cim, count, nr);
  return hipGetLastError();
}

hipError_t launch_norms(double* out, const c128* psi, int nfields, int nr, hipStream_t st) {
  hipLaunchKernelGGL(norms_kernel, dim3(nfields), dim3(kRedThreads), 0, st, out, psi, nr);
  return hipGetLastError();
}

hipError_t launch_agrad(double* out6, double* partial, int nblk, const c128* L, const c128* F, const double* kpts,
                        int nf, const Geom& g, const double a[3], long count, hipStream_t st) {
  hipLaunchKernelGGL(agrad_partial_kernel, dim3(nblk), dim3(kRedThreads), 0, st, partial, L, F, kpts, nf, g, a[0],
                     a[1], a[2], count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_rows_kernel, dim3(1), dim3(kRedThreads), 0, st, out6, partial, nblk, 6);
  return hipGetLastError();
}

hipError_t launch_mgs(c128* psi, int nk, int nb, int nr, double w, hipStream_t st) {
  hipLaunchKernelGGL(mgs_kernel, dim3(nk), dim3(kMgsThreads), 0, st, psi, nb, nr, w);
  return hipGetLastError();
}

}  // namespace fockmi
