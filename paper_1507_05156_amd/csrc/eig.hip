// Device kernels of the block eigensolver for h(t_f) (Sec. IV B, Eq. (25)) and
// of the excited-electron density (Eq. (26)), all in FP64.
//
// Fields are [nk][m][N_r] complex128 blocks. A "column set" is up to three such
// blocks side by side (the current vectors, the preconditioned residuals and
// the previous search directions of LOBPCG), addressed without copying.
#include "eig.hpp"

namespace fockmi {

namespace {

__device__ __forceinline__ const c128* col_ptr(const ColSet& z, int k, int c, long nr) {
  for (int q = 0; q < z.nparts; ++q) {
    if (c < z.cnt[q]) return z.p[q] + ((long)k * z.cnt[q] + c) * nr;
    c -= z.cnt[q];
  }
  return nullptr;
}

__device__ __forceinline__ c128 cmul_(c128 a, c128 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ c128 cconj(c128 a) { return {a.re, -a.im}; }

// out[k][i][j] = w * sum_r conj(A_i(r)) B_j(r) for i < A.total(), j < B.total();
// one workgroup per (4 x 4 tile, k), fixed-order reduction
constexpr int kGT = 4;
constexpr int kGramThreads = 256;
__global__ void __launch_bounds__(kGramThreads) gram_kernel(c128* __restrict__ out, ColSet A, ColSet B, int ma, int mb,
                                                            long nr, double w) {
  __shared__ double sh[2 * kGT * kGT][kGramThreads];
  const int k = blockIdx.z, i0 = blockIdx.x * kGT, j0 = blockIdx.y * kGT, t = threadIdx.x;
  const c128* a[kGT];
  const c128* b[kGT];
#pragma unroll
  for (int q = 0; q < kGT; ++q) {
    a[q] = i0 + q < ma ? col_ptr(A, k, i0 + q, nr) : nullptr;
    b[q] = j0 + q < mb ? col_ptr(B, k, j0 + q, nr) : nullptr;
  }
  double re[kGT][kGT], im[kGT][kGT];
#pragma unroll
  for (int i = 0; i < kGT; ++i)
#pragma unroll
    for (int j = 0; j < kGT; ++j) re[i][j] = im[i][j] = 0.0;
  for (long r = t; r < nr; r += kGramThreads) {
    c128 av[kGT], bv[kGT];
#pragma unroll
    for (int q = 0; q < kGT; ++q) {
      av[q] = a[q] ? a[q][r] : c128{0.0, 0.0};
      bv[q] = b[q] ? b[q][r] : c128{0.0, 0.0};
    }
#pragma unroll
    for (int i = 0; i < kGT; ++i)
#pragma unroll
      for (int j = 0; j < kGT; ++j) {
        re[i][j] += av[i].re * bv[j].re + av[i].im * bv[j].im;
        im[i][j] += av[i].re * bv[j].im - av[i].im * bv[j].re;
      }
  }
#pragma unroll
  for (int i = 0; i < kGT; ++i)
#pragma unroll
    for (int j = 0; j < kGT; ++j) {
      sh[2 * (i * kGT + j)][t] = re[i][j];
      sh[2 * (i * kGT + j) + 1][t] = im[i][j];
    }
  __syncthreads();
  for (int s = kGramThreads / 2; s > 0; s >>= 1) {
    if (t < s)
      for (int v = 0; v < 2 * kGT * kGT; ++v) sh[v][t] += sh[v][t + s];
    __syncthreads();
  }
  if (t < kGT * kGT) {
    const int i = i0 + t / kGT, j = j0 + t % kGT;
    if (i < ma && j < mb) out[((long)k * ma + i) * mb + j] = c128{w * sh[2 * t][0], w * sh[2 * t + 1][0]};
  }
}

// Y[k][j][r] = sum_{i < Z.total()} Z_i(k, r) C[k][row0 + i][j] for j < ncol <= kRotMaxCols;
// C is [k][crows][ncol]
constexpr int kRotThreads = 256;
__global__ void __launch_bounds__(kRotThreads) rotate_kernel(c128* __restrict__ Y, ColSet Z, const c128* __restrict__ C,
                                                             int row0, int crows, int ncol, long nr) {
  __shared__ c128 cs[kEigMax * kRotMaxCols];
  const int k = blockIdx.y, t = threadIdx.x;
  const int nz = Z.total();
  for (int idx = t; idx < nz * ncol; idx += kRotThreads)
    cs[idx] = C[((long)k * crows + row0 + idx / ncol) * ncol + idx % ncol];
  __syncthreads();
  const long r = (long)blockIdx.x * kRotThreads + t;
  if (r >= nr) return;
  c128 acc[kRotMaxCols];
#pragma unroll
  for (int j = 0; j < kRotMaxCols; ++j) acc[j] = c128{0.0, 0.0};
  for (int i = 0; i < nz; ++i) {
    const c128 z = col_ptr(Z, k, i, nr)[r];
#pragma unroll
    for (int j = 0; j < kRotMaxCols; ++j)
      if (j < ncol) {
        const c128 c = cs[i * ncol + j];
        acc[j].re += z.re * c.re - z.im * c.im;
        acc[j].im += z.re * c.im + z.im * c.re;
      }
  }
#pragma unroll
  for (int j = 0; j < kRotMaxCols; ++j)
    if (j < ncol) Y[((long)k * ncol + j) * nr + r] = acc[j];
}

// R[k][b][r] = HX[k][b][r] - lam[k][b] X[k][b][r]
__global__ void resid_kernel(c128* __restrict__ R, const c128* __restrict__ HX, const c128* __restrict__ X,
                             const double* __restrict__ lam, long nr, long count) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    const double l = lam[i / nr];
    R[i] = c128{HX[i].re - l * X[i].re, HX[i].im - l * X[i].im};
  }
}

// Soft locking: fields f whose residual sqrt(w * norms[f]) is at most tol are
// set to zero (their columns then drop out of the next Rayleigh-Ritz basis)
__global__ void lock_kernel(c128* __restrict__ a, const double* __restrict__ norms, double w, double tol, long nr,
                            long count) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
    if (sqrt(w * norms[i / nr]) <= tol) a[i] = c128{0.0, 0.0};
}

// Rayleigh-Ritz on a basis of m <= kEigMax vectors for one k (one wavefront):
// given S = Z^H Z and A = Z^H h Z, the nsel lowest solutions of A c = lam S c.
//   1. D = diag(S)^(-1/2) (scales the basis to unit columns);
//   2. Cholesky D S D = L L^H; a column whose remaining pivot is below
//      kDropTol (its vector lies within ~1e-4 of the span of the earlier ones)
//      is dropped: its row and column of L become those of the identity and
//      its diagonal entry of the projected matrix is pushed far above the
//      spectrum, so that it decouples and is never selected;
//   3. M = L^-1 (D A D) L^-H, made exactly Hermitian;
//   4. parallel cyclic complex Jacobi on M (rotation J = diag(1, e^-i theta)
//      R(c, s) on each pair p < q, theta the phase of M_pq), eigenvectors in V;
//   5. the nsel smallest eigenvalues in ascending order, and C = D L^-H V_sel.
// status[k] = number of dropped columns among the first nkeep.
constexpr double kDropTol = 1e-8;
// twelve waves: one row index per lane and twelve pair slots, so that a Jacobi
// round of up to 24 disjoint pairs costs each wave at most two rotations (with
// four waves, six: 163 ms against 146 ms for a 16^3, 8 k, 16-band eigensolve,
// 138.5 ms once a round also lost a barrier)
constexpr int kEigThreads = 768;
static_assert(kEigMax <= 64, "one lane per row of the projected matrix");
__global__ void __launch_bounds__(kEigThreads) rayleigh_ritz_kernel(const c128* __restrict__ S_, const c128* __restrict__ A_,
                                                                    int m, int nsel, int nkeep, c128* __restrict__ C_,
                                                                    double* __restrict__ lam_, int* __restrict__ status) {
  // row stride ld odd: a column access then spreads over the LDS banks instead
  // of striking one bank per 16-byte element
  __shared__ c128 L[kEigMax * (kEigMax + 1)], M[kEigMax * (kEigMax + 1)], V[kEigMax * (kEigMax + 1)];
  __shared__ c128 xs[kEigMax * kRotMaxCols];  // back-substitution work
  __shared__ double d[kEigMax], ev[kEigMax], offs[64];
  __shared__ int drop[kEigMax], order[kEigMax];
  __shared__ double rcs[kEigMax / 2], rsn[kEigMax / 2], rer[kEigMax / 2], rei[kEigMax / 2], scale;
  __shared__ int rp[2][kEigMax / 2], rq[2][kEigMax / 2], rskip[2][kEigMax / 2], done;
  __shared__ int cidx[kEigMax], mc;  // the directions that were not dropped, ascending
  const int k = blockIdx.x, t = threadIdx.x;
  const int ld = m | 1;
  const c128* S = S_ + (long)k * m * m;
  const c128* A = A_ + (long)k * m * m;

  for (int i = t; i < m; i += kEigThreads) {
    const double sii = S[i * m + i].re;
    drop[i] = !(sii > 1e-300);
    d[i] = drop[i] ? 0.0 : 1.0 / sqrt(sii);
  }
  __syncthreads();
  for (int idx = t; idx < m * m; idx += kEigThreads) {
    const int i = idx / m, j = idx % m;
    const double f = d[i] * d[j];
    L[i * ld + j] = c128{f * S[idx].re, f * S[idx].im};
    M[i * ld + j] = c128{f * A[idx].re, f * A[idx].im};
    V[i * ld + j] = c128{i == j ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();

  // Cholesky, column by column
  for (int j = 0; j < m; ++j) {
    if (t == 0) {
      double s = L[j * ld + j].re;
      for (int p = 0; p < j; ++p) s -= L[j * ld + p].re * L[j * ld + p].re + L[j * ld + p].im * L[j * ld + p].im;
      if (drop[j] || !(s > kDropTol)) {
        drop[j] = 1;
        for (int p = 0; p < j; ++p) L[j * ld + p] = c128{0.0, 0.0};
        L[j * ld + j] = c128{1.0, 0.0};
      } else {
        L[j * ld + j] = c128{sqrt(s), 0.0};
      }
    }
    __syncthreads();
    for (int i = j + 1 + t; i < m; i += kEigThreads) {
      if (drop[j]) {
        L[i * ld + j] = c128{0.0, 0.0};
      } else {
        c128 s = L[i * ld + j];
        for (int p = 0; p < j; ++p) {
          const c128 x = cmul_(L[i * ld + p], cconj(L[j * ld + p]));
          s.re -= x.re;
          s.im -= x.im;
        }
        const double inv = 1.0 / L[j * ld + j].re;
        L[i * ld + j] = c128{s.re * inv, s.im * inv};
      }
    }
    __syncthreads();
  }
  // upper triangle of L is not used; dropped rows/columns of M decouple
  if (t == 0) {
    double big = 1.0;
    for (int i = 0; i < m; ++i)
      if (!drop[i]) big = fmax(big, fabs(M[i * ld + i].re));
    scale = big;
  }
  __syncthreads();
  for (int idx = t; idx < m * m; idx += kEigThreads) {
    const int i = idx / m, j = idx % m;
    if (drop[i] || drop[j]) M[i * ld + j] = c128{(i == j) ? 1e6 * scale + i : 0.0, 0.0};
  }
  __syncthreads();
  // M <- L^-1 M (forward substitution, one column per thread)
  for (int c = t; c < m; c += kEigThreads) {
    for (int i = 0; i < m; ++i) {
      c128 s = M[i * ld + c];
      for (int p = 0; p < i; ++p) {
        const c128 x = cmul_(L[i * ld + p], M[p * ld + c]);
        s.re -= x.re;
        s.im -= x.im;
      }
      const double inv = 1.0 / L[i * ld + i].re;
      M[i * ld + c] = c128{s.re * inv, s.im * inv};
    }
  }
  __syncthreads();
  // M <- M L^-H (one row per thread): Z L^H = Y
  for (int r = t; r < m; r += kEigThreads) {
    for (int j = 0; j < m; ++j) {
      c128 s = M[r * ld + j];
      for (int p = 0; p < j; ++p) {
        const c128 x = cmul_(M[r * ld + p], cconj(L[j * ld + p]));
        s.re -= x.re;
        s.im -= x.im;
      }
      const double inv = 1.0 / L[j * ld + j].re;
      M[r * ld + j] = c128{s.re * inv, s.im * inv};
    }
  }
  __syncthreads();
  // exact Hermitian symmetry
  for (int idx = t; idx < m * m; idx += kEigThreads) {
    const int i = idx / m, j = idx % m;
    if (i < j) {
      const c128 a = M[i * ld + j], b = M[j * ld + i];
      const c128 h{0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
      M[i * ld + j] = h;
      M[j * ld + i] = cconj(h);
    } else if (i == j) {
      M[i * ld + j].im = 0.0;
    }
  }
  __syncthreads();

  // parallel cyclic Jacobi over the directions that were not dropped (the
  // dropped ones are already decoupled): every round rotates mm/2 disjoint pairs
  // at once (the circle method over mm = mc rounded up to even; pairs with the
  // padding index are skipped). Rotations on disjoint pairs commute, so a round
  // equals its rotations applied one after another; a sweep of mm - 1 rounds
  // meets every pair. Locked bands drop their W and P columns, so late
  // iterations rotate fewer pairs.
  if (t == 0) {
    int n = 0;
    for (int i = 0; i < m; ++i)
      if (!drop[i]) cidx[n++] = i;
    mc = n;
  }
  __syncthreads();
  const int mm = mc + (mc & 1), npair = mm / 2;
  const int lane = t & 63, slot = t >> 6;  // row (or column) index, pair slot
  for (int sweep = 0; sweep < 40; ++sweep) {
    // largest off-diagonal modulus: per-lane maxima over rows, then one lane
    {
      double off = 0.0;
      if (slot == 0 && lane < m)
        for (int q = lane + 1; q < m; ++q) off = fmax(off, fabs(M[lane * ld + q].re) + fabs(M[lane * ld + q].im));
      if (slot == 0) offs[lane] = off;  // lanes >= m hold 0
      __syncthreads();
      if (t == 0) {
        double o = 0.0;
        for (int i = 0; i < 64; ++i) o = fmax(o, offs[i]);
        done = o <= 1e-16 * scale;
      }
      __syncthreads();
    }
    if (done) break;
    for (int r = 0; r < mm - 1; ++r) {
      const int cb = r & 1, pb = cb ^ 1;  // this round's and the previous round's pair tables
      // wave 0: this round's pairs and their rotations, from M before the round;
      // wave 1: the previous round's rotated entries set to their exact values
      // (their rows and columns are not read until after the next barrier)
      if (t < npair) {
        const int i = t;
        const int a = i == 0 ? mm - 1 : (r + i) % (mm - 1);
        const int b = i == 0 ? r : (r - i + mm - 1) % (mm - 1);
        const int lo = a < b ? a : b, hi = a < b ? b : a;  // compact indices
        int sk = hi >= mc;
        const int p = sk ? 0 : cidx[lo], q = sk ? 0 : cidx[hi];
        rp[cb][i] = p;
        rq[cb][i] = q;
        if (!sk) {
          const c128 apq = M[p * ld + q];
          const double r2 = apq.re * apq.re + apq.im * apq.im;
          sk = !(r2 > 1e-36 * scale * scale);
          if (!sk) {
            const double inv = rsqrt(r2);  // 1 / |a_pq|
            rer[i] = apq.re * inv;          // e^{i theta}
            rei[i] = apq.im * inv;
            const double tau = (M[q * ld + q].re - M[p * ld + p].re) * (0.5 * inv);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            rcs[i] = rsqrt(1.0 + tt * tt);
            rsn[i] = tt * rcs[i];
          }
        }
        rskip[cb][i] = sk;
      } else if (r > 0 && t >= 64 && t < 64 + npair) {
        const int i = t - 64;
        if (!rskip[pb][i]) {
          const int p = rp[pb][i], q = rq[pb][i];
          M[p * ld + q] = c128{0.0, 0.0};
          M[q * ld + p] = c128{0.0, 0.0};
          M[p * ld + p].im = 0.0;
          M[q * ld + q].im = 0.0;
        }
      }
      __syncthreads();
      // columns: M <- M J, V <- V J with J = [[c, s], [-s e^{-i th}, c e^{-i th}]] on (p, q)
      for (int i = slot; i < npair; i += kEigThreads / 64) {
        const int row = lane;
        if (row >= m || rskip[cb][i]) continue;
        const int p = rp[cb][i], q = rq[cb][i];
        const double c = rcs[i], s = rsn[i], er = rer[i], ei = rei[i];
        const c128 mp = M[row * ld + p], mq = M[row * ld + q];
        const c128 mqe{mq.re * er + mq.im * ei, mq.im * er - mq.re * ei};  // mq e^{-i th}
        M[row * ld + p] = c128{c * mp.re - s * mqe.re, c * mp.im - s * mqe.im};
        M[row * ld + q] = c128{s * mp.re + c * mqe.re, s * mp.im + c * mqe.im};
        const c128 vp = V[row * ld + p], vq = V[row * ld + q];
        const c128 vqe{vq.re * er + vq.im * ei, vq.im * er - vq.re * ei};
        V[row * ld + p] = c128{c * vp.re - s * vqe.re, c * vp.im - s * vqe.im};
        V[row * ld + q] = c128{s * vp.re + c * vqe.re, s * vp.im + c * vqe.im};
      }
      __syncthreads();
      // rows: M <- J^H M
      for (int i = slot; i < npair; i += kEigThreads / 64) {
        const int col = lane;
        if (col >= m || rskip[cb][i]) continue;
        const int p = rp[cb][i], q = rq[cb][i];
        const double c = rcs[i], s = rsn[i], er = rer[i], ei = rei[i];
        const c128 mp = M[p * ld + col], mq = M[q * ld + col];
        const c128 mqe{mq.re * er - mq.im * ei, mq.im * er + mq.re * ei};  // mq e^{+i th}
        M[p * ld + col] = c128{c * mp.re - s * mqe.re, c * mp.im - s * mqe.im};
        M[q * ld + col] = c128{s * mp.re + c * mqe.re, s * mp.im + c * mqe.im};
      }
      __syncthreads();
    }
    // the last round's rotated entries
    {
      const int lb = (mm - 2) & 1;
      for (int i = t; i < npair; i += kEigThreads) {
        if (rskip[lb][i]) continue;
        const int p = rp[lb][i], q = rq[lb][i];
        M[p * ld + q] = c128{0.0, 0.0};
        M[q * ld + p] = c128{0.0, 0.0};
        M[p * ld + p].im = 0.0;
        M[q * ld + q].im = 0.0;
      }
      __syncthreads();
    }
  }
  if (t == 0) {
    for (int i = 0; i < m; ++i) {
      ev[i] = M[i * ld + i].re;
      order[i] = i;
    }
    for (int i = 0; i < nsel; ++i) {  // selection of the nsel smallest, ascending
      int b = i;
      for (int j = i + 1; j < m; ++j)
        if (ev[order[j]] < ev[order[b]]) b = j;
      const int tmp = order[i];
      order[i] = order[b];
      order[b] = tmp;
    }
    int nd = 0;
    for (int i = 0; i < nkeep && i < m; ++i) nd += drop[i];
    status[k] = nd;
  }
  __syncthreads();
  // C = D L^-H V_sel (back substitution with L^H, one selected vector per thread,
  // worked in LDS and written out once)
  for (int j = t; j < nsel; j += kEigThreads) {
    const int col = order[j];
    for (int i = m - 1; i >= 0; --i) {
      c128 s = V[i * ld + col];
      for (int p = i + 1; p < m; ++p) {
        const c128 x = cmul_(cconj(L[p * ld + i]), xs[p * kRotMaxCols + j]);
        s.re -= x.re;
        s.im -= x.im;
      }
      const double inv = 1.0 / L[i * ld + i].re;
      xs[i * kRotMaxCols + j] = c128{s.re * inv, s.im * inv};
    }
    c128* Ck = C_ + (long)k * m * nsel;
    for (int i = 0; i < m; ++i) {
      const c128 x = xs[i * kRotMaxCols + j];
      Ck[i * nsel + j] = c128{d[i] * x.re, d[i] * x.im};
    }
    lam_[(long)k * nsel + j] = ev[col];
  }
}

// out[0] = sum |S|^2 over count entries, fixed order (one workgroup)
constexpr int kSumThreads = 256;
__global__ void __launch_bounds__(kSumThreads) sum_abs2_kernel(double* __restrict__ out, const c128* __restrict__ S,
                                                               long count) {
  __shared__ double sh[kSumThreads];
  double s = 0.0;
  for (long i = threadIdx.x; i < count; i += kSumThreads) s += S[i].re * S[i].re + S[i].im * S[i].im;
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kSumThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

}  // namespace

hipError_t launch_gram(c128* out, const ColSet& A, const ColSet& B, int nk, long nr, double w, hipStream_t st) {
  const int ma = A.total(), mb = B.total();
  if (ma <= 0 || mb <= 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)((ma + kGT - 1) / kGT), (unsigned)((mb + kGT - 1) / kGT), (unsigned)nk);
  hipLaunchKernelGGL(gram_kernel, grid, dim3(kGramThreads), 0, st, out, A, B, ma, mb, nr, w);
  return hipGetLastError();
}

hipError_t launch_rotate(c128* Y, const ColSet& Z, const c128* C, int row0, int crows, int ncol, int nk, long nr,
                         hipStream_t st) {
  if (ncol <= 0 || ncol > kRotMaxCols || Z.total() > kEigMax || row0 + Z.total() > crows) return hipErrorInvalidValue;
  dim3 grid((unsigned)((nr + kRotThreads - 1) / kRotThreads), (unsigned)nk);
  hipLaunchKernelGGL(rotate_kernel, grid, dim3(kRotThreads), 0, st, Y, Z, C, row0, crows, ncol, nr);
  return hipGetLastError();
}

hipError_t launch_resid(c128* R, const c128* HX, const c128* X, const double* lam, long nr, long count,
                        hipStream_t st) {
  long g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(resid_kernel, dim3((unsigned)g), dim3(256), 0, st, R, HX, X, lam, nr, count);
  return hipGetLastError();
}

hipError_t launch_lock(c128* a, const double* norms, double w, double tol, long nr, long count, hipStream_t st) {
  long g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(lock_kernel, dim3((unsigned)g), dim3(256), 0, st, a, norms, w, tol, nr, count);
  return hipGetLastError();
}

hipError_t launch_rayleigh_ritz(const c128* S, const c128* A, int m, int nsel, int nkeep, c128* C, double* lam,
                                int* status, int nk, hipStream_t st) {
  if (m <= 0 || m > kEigMax || nsel <= 0 || nsel > m || nsel > kRotMaxCols) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rayleigh_ritz_kernel, dim3((unsigned)nk), dim3(kEigThreads), 0, st, S, A, m, nsel, nkeep, C, lam,
                     status);
  return hipGetLastError();
}

hipError_t launch_sum_abs2(double* out, const c128* S, long count, hipStream_t st) {
  hipLaunchKernelGGL(sum_abs2_kernel, dim3(1), dim3(kSumThreads), 0, st, out, S, count);
  return hipGetLastError();
}

}  // namespace fockmi
