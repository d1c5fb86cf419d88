// Screened-kernel tables K_q[l] (Eq. (15) with the HSE erfc interaction, Eq. (8)).
//
// v(p) = 4 pi/|p|^2 * (1 - exp(-|p|^2 / 4 w^2)), computed as -expm1 so that
// small |p| keeps its digits; v(0) = pi / w^2, the finite limit, used for the
// q = 0, l = 0 slot (q = 0 is an integer flag set by the host when the two
// k-points are the same entry of the mesh) and wherever q + G is exactly zero
// (two k-points that differ by a reciprocal-lattice vector of the grid). Nyquist
// slots (l_d = -n_d/2 for even n_d) take the average of v over l_d = +-n_d/2,
// over all such axes.
#include "kernels.hpp"

namespace fockmi {

namespace {

__device__ __forceinline__ double v_screened(double p2, double omega) {
  return 4.0 * M_PI / p2 * (-expm1(-p2 / (4.0 * omega * omega)));
}

__global__ void build_table_f64_kernel(double* __restrict__ K, const double* __restrict__ qvec,
                                       const int* __restrict__ qzero, int nq, Geom g, double omega,
                                       double scale) {
  const long nr = (long)g.n1 * g.n2 * g.n3;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (idx >= nr || q >= nq) return;
  const int j3 = (int)(idx % g.n3);
  const int j2 = (int)((idx / g.n3) % g.n2);
  const int j1 = (int)(idx / ((long)g.n2 * g.n3));
  const int n[3] = {g.n1, g.n2, g.n3};
  const int j[3] = {j1, j2, j3};
  int l[3];
  bool nyq[3];
  for (int d = 0; d < 3; ++d) {
    l[d] = j[d] < (n[d] + 1) / 2 ? j[d] : j[d] - n[d];
    nyq[d] = (n[d] % 2 == 0) && (j[d] == n[d] / 2);
  }
  const double qx = qvec[3 * q + 0], qy = qvec[3 * q + 1], qz = qvec[3 * q + 2];
  const bool g0 = qzero[q] && l[0] == 0 && l[1] == 0 && l[2] == 0;
  double sum = 0.0;
  int count = 0;
  for (int c = 0; c < 8; ++c) {
    bool skip = false;
    double lf[3];
    for (int d = 0; d < 3; ++d) {
      const bool flip = (c >> d) & 1;
      if (flip && !nyq[d]) skip = true;
      lf[d] = flip ? (double)(n[d] / 2) : (double)l[d];
    }
    if (skip) continue;
    const double px = qx + lf[0] * g.B[0][0] + lf[1] * g.B[1][0] + lf[2] * g.B[2][0];
    const double py = qy + lf[0] * g.B[0][1] + lf[1] * g.B[1][1] + lf[2] * g.B[2][1];
    const double pz = qz + lf[0] * g.B[0][2] + lf[1] * g.B[1][2] + lf[2] * g.B[2][2];
    const double p2 = px * px + py * py + pz * pz;
    sum += (g0 || p2 == 0.0) ? M_PI / (omega * omega) : v_screened(p2, omega);
    ++count;
  }
  K[(long)q * nr + idx] = scale * (sum / count);
}

// Fused layout: value index l3 of thread t in the z phase of the fused kernel,
// with the same (l1, l2) <- t map as that kernel (see fused.hip).
template <typename T>
__global__ void build_table_fused_kernel(T* __restrict__ Kt, const double* __restrict__ K, int nq, int n,
                                         int nph) {
  const int nt = n * n;
  const long nr = (long)nt * n;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;  // = l3 * nt + t
  const int q = blockIdx.y;
  if (idx >= nr || q >= nq) return;
  const int l3 = (int)(idx / nt);
  const int t = (int)(idx % nt);
  const int h = n / nph, tpg = nt / nph;
  const int grp = t / tpg, tl = t % tpg;
  const int l2 = tl % h + h * grp;
  const int l1 = tl / h;
  Kt[(long)q * nr + idx] = (T)K[(long)q * nr + ((long)l1 * n + l2) * n + l3];
}

}  // namespace

hipError_t launch_build_table_f64(double* K, const double* qvec, const int* qzero, int nq, const Geom& g,
                                  double omega, double scale, hipStream_t st) {
  const long nr = (long)g.n1 * g.n2 * g.n3;
  for (int q0 = 0; q0 < nq; q0 += 65535) {
    const int cnt = nq - q0 < 65535 ? nq - q0 : 65535;
    dim3 grid((unsigned)((nr + 255) / 256), (unsigned)cnt);
    hipLaunchKernelGGL(build_table_f64_kernel, grid, dim3(256), 0, st, K + (long)q0 * nr, qvec + 3L * q0,
                       qzero + q0, cnt, g, omega, scale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int fused_phases(int n);  // fused.hip

hipError_t launch_build_table_fused(float* Kt, const double* K, int nq, int n, hipStream_t st) {
  const long nr = (long)n * n * n;
  for (int q0 = 0; q0 < nq; q0 += 65535) {
    const int cnt = nq - q0 < 65535 ? nq - q0 : 65535;
    dim3 grid((unsigned)((nr + 255) / 256), (unsigned)cnt);
    hipLaunchKernelGGL(build_table_fused_kernel<float>, grid, dim3(256), 0, st, Kt + (long)q0 * nr,
                       K + (long)q0 * nr, cnt, n, fused_phases(n));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_build_table_fused64(double* Kt, const double* K, int nq, int n, int nph, hipStream_t st) {
  const long nr = (long)n * n * n;
  for (int q0 = 0; q0 < nq; q0 += 65535) {
    const int cnt = nq - q0 < 65535 ? nq - q0 : 65535;
    dim3 grid((unsigned)((nr + 255) / 256), (unsigned)cnt);
    hipLaunchKernelGGL(build_table_fused_kernel<double>, grid, dim3(256), 0, st, Kt + (long)q0 * nr,
                       K + (long)q0 * nr, cnt, n, nph);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace fockmi
