// FP64 dense kernels on the small n x n complex128 matrix of the ACE
// construction (row-major, interleaved re/im):
//
//   hermitize : M <- (M + M^H)/2
//   cholesky  : -M = L L^H, L lower triangular with real positive diagonal
//               (the unique factor); on breakdown the 1-based column goes to
//               the status word and the factor is left incomplete
//   inverse   : U = L^{-H} (upper triangular), the right factor of xi = W U
//
// These steps stay in FP64 in both precision forms.
#include "px_internal.hpp"

namespace px {

__global__ void hermitize_k(double* M, int n) {
  const size_t total = size_t(n) * n;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += size_t(gridDim.x) * blockDim.x) {
    const int i = int(e / n), j = int(e % n);
    if (j < i) continue;
    double* a = M + (size_t(i) * n + j) * 2;
    double* b = M + (size_t(j) * n + i) * 2;
    const double re = 0.5 * (a[0] + b[0]);
    const double im = 0.5 * (a[1] - b[1]);
    a[0] = re;
    a[1] = im;
    b[0] = re;
    b[1] = -im;
  }
}

hipError_t launch_hermitize(double* M, int n, hipStream_t s) {
  const size_t total = size_t(n) * n;
  const int blocks = int((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  hipLaunchKernelGGL(hermitize_k, dim3(blocks), dim3(256), 0, s, M, n);
  return hipGetLastError();
}

// Left-looking (Crout) Cholesky of A = -M in one workgroup.  Column k:
//   L[k][k] = sqrt(A[k][k] - sum_{p<k} |L[k][p]|^2)
//   L[i][k] = (A[i][k] - sum_{p<k} L[i][p] conj(L[k][p])) / L[k][k],  i > k
// Rows of L are contiguous, so each dot product streams two rows.
__global__ __launch_bounds__(1024) void cholesky_k(const double* M, int n, double* L,
                                                   int32_t* status) {
  __shared__ double diag;
  __shared__ int failed;
  if (threadIdx.x == 0) failed = 0;
  // zero the strict upper triangle, copy -M's lower triangle
  for (size_t e = threadIdx.x; e < size_t(n) * n; e += blockDim.x) {
    const int i = int(e / n), j = int(e % n);
    if (j > i) {
      L[e * 2] = 0.0;
      L[e * 2 + 1] = 0.0;
    } else {
      L[e * 2] = -M[e * 2];
      L[e * 2 + 1] = -M[e * 2 + 1];
    }
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      const double* lk = L + size_t(k) * n * 2;
      double d = lk[2 * k];
      for (int p = 0; p < k; ++p) d -= lk[2 * p] * lk[2 * p] + lk[2 * p + 1] * lk[2 * p + 1];
      if (!(d > 0.0)) {
        failed = k + 1;
        d = 1.0;
      }
      diag = sqrt(d);
    }
    __syncthreads();
    if (failed) break;
    const double lkk = diag;
    const double* lk = L + size_t(k) * n * 2;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) {
      double* li = L + size_t(i) * n * 2;
      double re = li[2 * k], im = li[2 * k + 1];
      for (int p = 0; p < k; ++p) {
        // L[i][p] * conj(L[k][p])
        const double ar = li[2 * p], ai = li[2 * p + 1], br = lk[2 * p], bi = lk[2 * p + 1];
        re -= ar * br + ai * bi;
        im -= ai * br - ar * bi;
      }
      li[2 * k] = re / lkk;
      li[2 * k + 1] = im / lkk;
    }
    if (threadIdx.x == 0) {
      double* lkw = L + size_t(k) * n * 2;
      lkw[2 * k] = lkk;
      lkw[2 * k + 1] = 0.0;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) status[0] = failed;
}

// U = L^{-H}: thread c solves L x = e_c by forward substitution and writes
// row c of U as conj(x) (U[c][i] = conj(Linv[i][c]), zero for i < c).
__global__ __launch_bounds__(64) void tri_inv_k(const double* L, int n, double* U,
                                                const int32_t* status) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double* urow = U + size_t(c) * n * 2;
  if (status[0] != 0) {
    for (int i = 0; i < n; ++i) urow[2 * i] = urow[2 * i + 1] = 0.0;
    return;
  }
  for (int i = 0; i < c; ++i) urow[2 * i] = urow[2 * i + 1] = 0.0;
  // x_c = 1/L[c][c]; x_i = -(sum_{p=c}^{i-1} L[i][p] x_p)/L[i][i]; x kept in urow (conjugated at the end)
  urow[2 * c] = 1.0 / L[(size_t(c) * n + c) * 2];
  urow[2 * c + 1] = 0.0;
  for (int i = c + 1; i < n; ++i) {
    const double* li = L + size_t(i) * n * 2;
    double re = 0.0, im = 0.0;
    for (int p = c; p < i; ++p) {
      const double ar = li[2 * p], ai = li[2 * p + 1], xr = urow[2 * p], xi = urow[2 * p + 1];
      re += ar * xr - ai * xi;
      im += ar * xi + ai * xr;
    }
    const double inv = 1.0 / li[2 * i];
    urow[2 * i] = -re * inv;
    urow[2 * i + 1] = -im * inv;
  }
  for (int i = c; i < n; ++i) urow[2 * i + 1] = -urow[2 * i + 1];
}

hipError_t launch_chol_inv(const double* M, int n, double* L, double* U, int32_t* status,
                           hipStream_t s) {
  hipLaunchKernelGGL(cholesky_k, dim3(1), dim3(1024), 0, s, M, n, L, status);
  hipLaunchKernelGGL(tri_inv_k, dim3((n + 63) / 64), dim3(64), 0, s, L, n, U, status);
  return hipGetLastError();
}

}  // namespace px
