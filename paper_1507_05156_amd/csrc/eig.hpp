// Launchers of the block-eigensolver kernels (eig.hip). FP64 throughout.
#pragma once

#include "kernels.hpp"

namespace fockmi {

constexpr int kEigMax = 48;      // largest Rayleigh-Ritz basis per k
constexpr int kRotMaxCols = 16;  // largest block of vectors formed by one rotation

// Up to three [nk][cnt][N_r] blocks read as one set of cnt[0] + cnt[1] + cnt[2] columns.
struct ColSet {
  const c128* p[3];
  int cnt[3];
  int nparts;
  __host__ __device__ int total() const {
    int s = 0;
    for (int q = 0; q < nparts; ++q) s += cnt[q];
    return s;
  }
};

// out[k][i][j] = w sum_r conj(A_i) B_j  (A.total() x B.total() per k), fixed order
hipError_t launch_gram(c128* out, const ColSet& A, const ColSet& B, int nk, long nr, double w, hipStream_t st);
// Y[k][j] = sum_i Z_i C[k][row0 + i][j], j < ncol (C is [nk][crows][ncol]); Y distinct from Z
hipError_t launch_rotate(c128* Y, const ColSet& Z, const c128* C, int row0, int crows, int ncol, int nk, long nr,
                         hipStream_t st);
// R = HX - lam X, lam per field
hipError_t launch_resid(c128* R, const c128* HX, const c128* X, const double* lam, long nr, long count,
                        hipStream_t st);
// a[f][r] = 0 for the fields f with sqrt(w norms[f]) <= tol (norms: sum_r |residual|^2 per field)
hipError_t launch_lock(c128* a, const double* norms, double w, double tol, long nr, long count, hipStream_t st);
// per k: the nsel lowest solutions of A c = lam S c on an m-vector basis (m <= kEigMax,
// nsel <= kRotMaxCols);
// C [nk][m][nsel], lam [nk][nsel], status[k] = dropped basis vectors among the first nkeep
hipError_t launch_rayleigh_ritz(const c128* S, const c128* A, int m, int nsel, int nkeep, c128* C, double* lam,
                                int* status, int nk, hipStream_t st);
// out[0] = sum |S_i|^2, i < count (fixed order)
hipError_t launch_sum_abs2(double* out, const c128* S, long count, hipStream_t st);

}  // namespace fockmi
