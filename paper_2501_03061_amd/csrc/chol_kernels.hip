// FP64 dense kernels on the small n x n complex128 matrix of the ACE
// construction (row-major, interleaved re/im):
//
//   hermitize : M <- (M + M^H)/2
//   cholesky  : -M = L L^H, L lower triangular with real positive diagonal
//               (the unique factor), blocked in 32-column panels; on
//               breakdown the 1-based column goes to the status word
//   inverse   : U = L^{-H} (upper triangular), the right factor of xi = W U
//
// These steps stay in FP64 in both precision forms.
#include "px_internal.hpp"

namespace px {

// The factorisation of a launch: the argument, or entry blockIdx.z of a job
// table in device memory (a group shares one launch per step).
__device__ __forceinline__ CholJob chol_job(const CholJob& j0, const CholJob* jobs) {
  return jobs ? jobs[blockIdx.z] : j0;
}

__global__ void hermitize_k(CholJob j0, const CholJob* jobs) {
  const CholJob j = chol_job(j0, jobs);
  double* const M = j.M;
  const int n = j.n;
  const size_t total = size_t(n) * n;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += size_t(gridDim.x) * blockDim.x) {
    const int i = int(e / n), c = int(e % n);
    if (c < i) continue;
    double* a = M + (size_t(i) * n + c) * 2;
    double* b = M + (size_t(c) * n + i) * 2;
    const double re = 0.5 * (a[0] + b[0]);
    const double im = 0.5 * (a[1] - b[1]);
    a[0] = re;
    a[1] = im;
    b[0] = re;
    b[1] = -im;
  }
}

namespace {
int elementwise_blocks(int n) {
  const size_t total = size_t(n) * n;
  return int((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
}
}  // namespace

hipError_t launch_hermitize(double* M, int n, hipStream_t s) {
  CholJob j{};
  j.M = M;
  j.n = n;
  hipLaunchKernelGGL(hermitize_k, dim3(elementwise_blocks(n)), dim3(256), 0, s, j,
                     static_cast<const CholJob*>(nullptr));
  return hipGetLastError();
}

// Blocked right-looking Cholesky of A = -M, block width KB = 32:
//   for each diagonal block k: factor A_kk = L_kk L_kk^H in LDS (one
//   workgroup) and keep inv(L_kk); panel L_ik = A_ik L_kk^{-H} (one thread per
//   row); trailing update A_ij -= L_ik L_jk^H for i >= j (32 x 32 tiles).
// The working matrix L starts as -M and ends as the lower factor with a
// zeroed strict upper triangle.  A non-positive pivot stops the factorisation:
// status = 1-based global column, and every later kernel returns at once.
// In a group every job runs the steps of the largest n; a step past a job's
// own size returns at once.
constexpr int KB = 32;

__global__ void chol_init_k(CholJob j0, const CholJob* jobs) {
  const CholJob j = chol_job(j0, jobs);
  const size_t total = size_t(j.n) * j.n;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += size_t(gridDim.x) * blockDim.x) {
    j.L[2 * e] = -j.M[2 * e];
    j.L[2 * e + 1] = -j.M[2 * e + 1];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) j.status[0] = 0;
}

// Factor the diagonal block at k0 (size kb <= KB) in LDS; write L_kk back and
// inv(L_kk) into the job's dinv (KB x KB per block, row-major complex).
__global__ __launch_bounds__(256) void chol_diag_k(CholJob j0, const CholJob* jobs, int k0) {
  __shared__ double a[KB][KB][2];
  __shared__ double x[KB][KB][2];
  __shared__ int bad;
  const CholJob j = chol_job(j0, jobs);
  const int n = j.n;
  if (k0 >= n || j.status[0] != 0) return;
  double* const L = j.L;
  double* const Dinv = j.dinv + size_t(k0 / KB) * KB * KB * 2;
  const int kb = (n - k0) < KB ? (n - k0) : KB;
  const int t = threadIdx.x;
  for (int e = t; e < KB * KB; e += 256) {
    const int r = e / KB, c = e % KB;
    const bool in = r < kb && c < kb;
    a[r][c][0] = in ? L[(size_t(k0 + r) * n + k0 + c) * 2] : 0.0;
    a[r][c][1] = in ? L[(size_t(k0 + r) * n + k0 + c) * 2 + 1] : 0.0;
  }
  if (t == 0) bad = 0;
  __syncthreads();
  // unblocked right-looking factorisation of the lower triangle
  for (int k = 0; k < kb; ++k) {
    if (t == 0) {
      const double d = a[k][k][0];
      if (!(d > 0.0)) bad = k0 + k + 1;
      a[k][k][0] = d > 0.0 ? sqrt(d) : 1.0;
      a[k][k][1] = 0.0;
    }
    __syncthreads();
    if (bad) break;
    const double dk = a[k][k][0];
    for (int r = k + 1 + t; r < kb; r += 256) {
      a[r][k][0] /= dk;
      a[r][k][1] /= dk;
    }
    __syncthreads();
    for (int e = t; e < KB * KB; e += 256) {
      const int r = e / KB, c = e % KB;
      if (r > k && c > k && c <= r && r < kb) {
        // a[r][c] -= a[r][k] * conj(a[c][k])
        const double ar = a[r][k][0], ai = a[r][k][1], br = a[c][k][0], bi = a[c][k][1];
        a[r][c][0] -= ar * br + ai * bi;
        a[r][c][1] -= ai * br - ar * bi;
      }
    }
    __syncthreads();
  }
  if (bad) {
    if (t == 0) j.status[0] = bad;
    return;
  }
  // inverse of the lower factor: column c by forward substitution (thread c)
  if (t < KB) {
    const int c = t;
    for (int r = 0; r < KB; ++r) x[r][c][0] = x[r][c][1] = 0.0;
    if (c < kb) {
      x[c][c][0] = 1.0 / a[c][c][0];
      for (int r = c + 1; r < kb; ++r) {
        double sr = 0.0, si = 0.0;
        for (int p = c; p < r; ++p) {
          sr += a[r][p][0] * x[p][c][0] - a[r][p][1] * x[p][c][1];
          si += a[r][p][0] * x[p][c][1] + a[r][p][1] * x[p][c][0];
        }
        x[r][c][0] = -sr / a[r][r][0];
        x[r][c][1] = -si / a[r][r][0];
      }
    }
  }
  __syncthreads();
  for (int e = t; e < KB * KB; e += 256) {
    const int r = e / KB, c = e % KB;
    Dinv[2 * e] = x[r][c][0];
    Dinv[2 * e + 1] = x[r][c][1];
    if (r < kb && c < kb) {
      const bool low = c <= r;
      L[(size_t(k0 + r) * n + k0 + c) * 2] = low ? a[r][c][0] : 0.0;
      L[(size_t(k0 + r) * n + k0 + c) * 2 + 1] = low ? a[r][c][1] : 0.0;
    }
  }
}

// Panel: for rows i >= k0 + kb, L[i][k0:k0+kb] = A[i][k0:k0+kb] * inv(L_kk)^H,
// and zero the block above the diagonal (L[k0..][i] for the same columns).
// inv(L_kk) is staged in LDS (every lane then reads the same entry).
__global__ __launch_bounds__(64) void chol_panel_k(CholJob j0, const CholJob* jobs, int k0) {
  __shared__ double dl[KB * KB * 2];
  const CholJob j = chol_job(j0, jobs);
  const int n = j.n;
  if (k0 >= n || j.status[0] != 0) return;
  const int kb = (n - k0) < KB ? (n - k0) : KB;
  if (k0 + kb + int(blockIdx.x) * 64 >= n) return;  // no row of this job in the workgroup
  const double* const Dinv = j.dinv + size_t(k0 / KB) * KB * KB * 2;
  for (int e = threadIdx.x; e < KB * KB * 2; e += 64) dl[e] = Dinv[e];
  __syncthreads();
  double* const L = j.L;
  const int i = k0 + kb + blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  double ar[KB], ai[KB];
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    ar[c] = c < kb ? L[(size_t(i) * n + k0 + c) * 2] : 0.0;
    ai[c] = c < kb ? L[(size_t(i) * n + k0 + c) * 2 + 1] : 0.0;
  }
  // out[c] = sum_p a[p] * conj(Dinv[c][p])
  for (int c = 0; c < kb; ++c) {
    double sr = 0.0, si = 0.0;
    for (int p = 0; p <= c; ++p) {
      const double dr = dl[(c * KB + p) * 2], di = dl[(c * KB + p) * 2 + 1];
      sr += ar[p] * dr + ai[p] * di;
      si += ai[p] * dr - ar[p] * di;
    }
    L[(size_t(i) * n + k0 + c) * 2] = sr;
    L[(size_t(i) * n + k0 + c) * 2 + 1] = si;
    // strict upper triangle of the final factor: zero L[k0 + c][i]
    L[(size_t(k0 + c) * n + i) * 2] = 0.0;
    L[(size_t(k0 + c) * n + i) * 2 + 1] = 0.0;
  }
}

// Trailing update of the lower triangle: tile (bi, bj) of 32 x 32 with
// bi >= bj over rows/columns >= k0 + kb.
__global__ __launch_bounds__(256) void chol_update_k(CholJob j0, const CholJob* jobs, int k0) {
  __shared__ double pi_[KB][KB + 1][2];
  __shared__ double pj_[KB][KB + 1][2];
  const CholJob j = chol_job(j0, jobs);
  const int n = j.n;
  if (k0 >= n || j.status[0] != 0) return;
  const int kb = (n - k0) < KB ? (n - k0) : KB;
  const int base = k0 + kb;
  const int bi = blockIdx.x, bj = blockIdx.y;
  if (bj > bi) return;
  const int r0 = base + bi * KB, c0 = base + bj * KB;
  if (r0 >= n) return;
  double* const L = j.L;
  const int t = threadIdx.x;
  for (int e = t; e < KB * KB; e += 256) {
    const int r = e / KB, p = e % KB;
    const bool vi = r0 + r < n && p < kb, vj = c0 + r < n && p < kb;
    pi_[r][p][0] = vi ? L[(size_t(r0 + r) * n + k0 + p) * 2] : 0.0;
    pi_[r][p][1] = vi ? L[(size_t(r0 + r) * n + k0 + p) * 2 + 1] : 0.0;
    pj_[r][p][0] = vj ? L[(size_t(c0 + r) * n + k0 + p) * 2] : 0.0;
    pj_[r][p][1] = vj ? L[(size_t(c0 + r) * n + k0 + p) * 2 + 1] : 0.0;
  }
  __syncthreads();
  for (int e = t; e < KB * KB; e += 256) {
    const int r = e / KB, c = e % KB;
    const int gi = r0 + r, gj = c0 + c;
    if (gi >= n || gj >= n || gj > gi) continue;
    double sr = 0.0, si = 0.0;
#pragma unroll 8
    for (int p = 0; p < KB; ++p) {
      const double ar = pi_[r][p][0], ai = pi_[r][p][1], br = pj_[c][p][0], bi2 = pj_[c][p][1];
      sr += ar * br + ai * bi2;
      si += ai * br - ar * bi2;
    }
    L[(size_t(gi) * n + gj) * 2] -= sr;
    L[(size_t(gi) * n + gj) * 2 + 1] -= si;
  }
}

// U = L^{-H} from the blocked inverse X = L^{-1}, by block wavefronts.  The
// factorisation leaves inv(L_kk) of every diagonal block in dinv
// (nb x KB x KB).  Wavefront d = 0 sets X_cc = inv(L_cc); wavefront d >= 1
// computes, for every block column c with r = c + d < nb,
//   X_rc = -inv(L_rr) * sum_{p=c}^{r-1} L_rp X_pc,
// one workgroup per block.  X is never stored itself: block (r, c) of X goes
// to U as U[c0 + j][r0 + i] = conj(X_rc[i][j]), and later wavefronts read X_pc
// back from there (a launch boundary orders the store before the load).
// The strict lower triangle of U is zeroed first; after a breakdown U stays 0.
__global__ void tri_zero_k(CholJob j0, const CholJob* jobs) {
  const CholJob j = chol_job(j0, jobs);
  const size_t total = size_t(j.n) * j.n * 2;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += size_t(gridDim.x) * blockDim.x)
    j.U[e] = 0.0;
}

__global__ __launch_bounds__(256) void tri_wave_k(CholJob j0, const CholJob* jobs, int d) {
  __shared__ double ls[KB][KB + 1][2];
  __shared__ double xs[KB][KB + 1][2];
  const CholJob jb = chol_job(j0, jobs);
  if (jb.status[0] != 0) return;
  const int n = jb.n;
  const double* const L = jb.L;
  const double* const Dinv = jb.dinv;
  double* const U = jb.U;
  const int nb = (n + KB - 1) / KB;
  const int c = blockIdx.x, r = c + d;
  if (r >= nb) return;
  const int c0 = c * KB, r0 = r * KB;
  const int rb = (n - r0) < KB ? (n - r0) : KB;   // only the last block row can be short
  const int t = threadIdx.x;
  const int row = t / 8, col = t % 8;              // outputs (row, col + 8k), k < 4
  double ar[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
  const double* dr = Dinv + size_t(r) * KB * KB * 2;
  if (d == 0) {
    for (int k = 0; k < 4; ++k) {
      ar[k] = dr[(row * KB + col + 8 * k) * 2];
      ai[k] = dr[(row * KB + col + 8 * k) * 2 + 1];
    }
  } else {
    // T = sum_p L_rp X_pc
    for (int p = c; p < r; ++p) {
      const int p0 = p * KB;
      const double* dp = Dinv + size_t(p) * KB * KB * 2;
      for (int e = t; e < KB * KB; e += 256) {
        const int i = e / KB, q = e % KB;
        const bool in = i < rb;
        ls[i][q][0] = in ? L[(size_t(r0 + i) * n + p0 + q) * 2] : 0.0;
        ls[i][q][1] = in ? L[(size_t(r0 + i) * n + p0 + q) * 2 + 1] : 0.0;
        // X_pc[q][j] with j = e / KB, q = e % KB (contiguous reads of U row c0 + j)
        const int jj = e / KB, qq = e % KB;
        if (p == c) {
          xs[qq][jj][0] = dp[(qq * KB + jj) * 2];
          xs[qq][jj][1] = dp[(qq * KB + jj) * 2 + 1];
        } else {
          xs[qq][jj][0] = U[(size_t(c0 + jj) * n + p0 + qq) * 2];
          xs[qq][jj][1] = -U[(size_t(c0 + jj) * n + p0 + qq) * 2 + 1];
        }
      }
      __syncthreads();
#pragma unroll 4
      for (int q = 0; q < KB; ++q) {
        const double lr = ls[row][q][0], li = ls[row][q][1];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double xr = xs[q][col + 8 * k][0], xi = xs[q][col + 8 * k][1];
          ar[k] += lr * xr - li * xi;
          ai[k] += lr * xi + li * xr;
        }
      }
      __syncthreads();
    }
    // X_rc = -inv(L_rr) T
    for (int k = 0; k < 4; ++k) {
      xs[row][col + 8 * k][0] = ar[k];
      xs[row][col + 8 * k][1] = ai[k];
    }
    for (int e = t; e < KB * KB; e += 256) {
      const int i = e / KB, q = e % KB;
      ls[i][q][0] = dr[e * 2];
      ls[i][q][1] = dr[e * 2 + 1];
    }
    __syncthreads();
    for (int k = 0; k < 4; ++k) ar[k] = ai[k] = 0.0;
#pragma unroll 4
    for (int q = 0; q < KB; ++q) {
      const double lr = ls[row][q][0], li = ls[row][q][1];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double xr = xs[q][col + 8 * k][0], xi = xs[q][col + 8 * k][1];
        ar[k] -= lr * xr - li * xi;
        ai[k] -= lr * xi + li * xr;
      }
    }
  }
  if (row < rb) {
    for (int k = 0; k < 4; ++k) {
      const int jc = col + 8 * k;
      if (c0 + jc >= n) continue;
      U[(size_t(c0 + jc) * n + r0 + row) * 2] = ar[k];
      U[(size_t(c0 + jc) * n + r0 + row) * 2 + 1] = -ai[k];
    }
  }
}

namespace {
// Every step of the factorisation and the inverse for one job (jobs ==
// nullptr) or a table of njobs (steps and grids of the largest size n).
hipError_t chol_steps(const CholJob& j0, const CholJob* jobs, int njobs, int n, hipStream_t s) {
  const int blocks = elementwise_blocks(n);
  hipLaunchKernelGGL(chol_init_k, dim3(blocks, 1, njobs), dim3(256), 0, s, j0, jobs);
  for (int k0 = 0; k0 < n; k0 += KB) {
    hipLaunchKernelGGL(chol_diag_k, dim3(1, 1, njobs), dim3(256), 0, s, j0, jobs, k0);
    const int kb = (n - k0) < KB ? (n - k0) : KB;
    const int rest = n - k0 - kb;
    if (rest > 0) {
      hipLaunchKernelGGL(chol_panel_k, dim3((rest + 63) / 64, 1, njobs), dim3(64), 0, s, j0, jobs,
                         k0);
      const int nt = (rest + KB - 1) / KB;
      hipLaunchKernelGGL(chol_update_k, dim3(nt, nt, njobs), dim3(256), 0, s, j0, jobs, k0);
    }
  }
  hipLaunchKernelGGL(tri_zero_k, dim3(blocks, 1, njobs), dim3(256), 0, s, j0, jobs);
  const int nb = (n + KB - 1) / KB;
  for (int d = 0; d < nb; ++d)
    hipLaunchKernelGGL(tri_wave_k, dim3(nb - d, 1, njobs), dim3(256), 0, s, j0, jobs, d);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_chol_inv(const double* M, int n, double* L, double* U, int32_t* status,
                           double* dinv, hipStream_t s) {
  CholJob j{};
  j.M = const_cast<double*>(M);  // read only by these kernels
  j.L = L;
  j.U = U;
  j.dinv = dinv;
  j.status = status;
  j.n = n;
  return chol_steps(j, nullptr, 1, n, s);
}

hipError_t launch_chol_inv_group(const CholJob* jobs, int njobs, int max_n, hipStream_t s) {
  const CholJob none{};
  hipLaunchKernelGGL(hermitize_k, dim3(elementwise_blocks(max_n), 1, njobs), dim3(256), 0, s, none,
                     jobs);
  return chol_steps(none, jobs, njobs, max_n, s);
}

size_t chol_dinv_bytes(int n) { return size_t((n + KB - 1) / KB) * KB * KB * 16; }


}  // namespace px

// ---------------------------------------------------------------- small FP64 products
namespace px {

// C = alpha op(A) B for complex128 row-major matrices: op(A) is m x k (A
// itself, or A^H with A stored k x m), B is k x n, C is m x n, with leading
// dimensions lda, ldb, ldc in elements.  16 x 16 tiles of C per workgroup,
// 16 x 16 tiles of op(A) and B staged in LDS, one entry of C per thread.
// Used for the small matrix algebra of the PT-IM step (N_phi x N_phi, and
// N_phi x N_phi products over the rank of xi), where the FP64 vector rate is
// ample.
template <bool AH>
__global__ __launch_bounds__(256) void zgemm_k(int m, int n, int kd, const double* A, int lda,
                                               const double* B, int ldb, double* C, int ldc,
                                               double alpha) {
  __shared__ double2 sa[16][17], sb[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
  double cr = 0.0, ci = 0.0;
  for (int k0 = 0; k0 < kd; k0 += 16) {
    // op(A)[row][k0 + tx]: A[row][k] or conj(A[k][row])
    {
      const int k = k0 + tx;
      double2 v = make_double2(0.0, 0.0);
      if (row < m && k < kd) {
        if (AH) {
          const double* p = A + (size_t(k) * lda + row) * 2;
          v = make_double2(p[0], -p[1]);
        } else {
          const double* p = A + (size_t(row) * lda + k) * 2;
          v = make_double2(p[0], p[1]);
        }
      }
      sa[ty][tx] = v;
    }
    {
      const int k = k0 + ty;
      double2 v = make_double2(0.0, 0.0);
      if (k < kd && col < n) {
        const double* p = B + (size_t(k) * ldb + col) * 2;
        v = make_double2(p[0], p[1]);
      }
      sb[ty][tx] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double2 a = sa[ty][k], b = sb[k][tx];
      cr += a.x * b.x - a.y * b.y;
      ci += a.x * b.y + a.y * b.x;
    }
    __syncthreads();
  }
  if (row < m && col < n) {
    C[(size_t(row) * ldc + col) * 2] = alpha * cr;
    C[(size_t(row) * ldc + col) * 2 + 1] = alpha * ci;
  }
}

hipError_t launch_zgemm_gen(bool ah, int m, int n, int k, const double* A, int lda, const double* B,
                            int ldb, double* C, int ldc, double alpha, hipStream_t s) {
  if (m <= 0 || n <= 0 || k <= 0) return hipErrorInvalidValue;
  const dim3 g((n + 15) / 16, (m + 15) / 16);
  if (ah)
    hipLaunchKernelGGL(zgemm_k<true>, g, dim3(256), 0, s, m, n, k, A, lda, B, ldb, C, ldc, alpha);
  else
    hipLaunchKernelGGL(zgemm_k<false>, g, dim3(256), 0, s, m, n, k, A, lda, B, ldb, C, ldc, alpha);
  return hipGetLastError();
}

hipError_t launch_zgemm(bool ah, int n, const double* A, const double* B, double* C, hipStream_t s) {
  return launch_zgemm_gen(ah, n, n, n, A, n, B, n, C, n, 1.0, s);
}

// dst = alpha * src over n real values
__global__ void scale_k(size_t n, const double* src, double alpha, double* dst) {
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
       e += size_t(gridDim.x) * blockDim.x)
    dst[e] = alpha * src[e];
}

hipError_t launch_scale(size_t n, const double* src, double alpha, double* dst, hipStream_t s) {
  const int blocks = int((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(scale_k, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, n, src, alpha, dst);
  return hipGetLastError();
}

// sigma_nxt = sigma_n - i c (A1 - A2) over n x n complex values, and
// res = ||sigma_nxt - sigma_cur||_F / ||sigma_nxt||_F (one workgroup, fixed
// summation order).
__global__ __launch_bounds__(1024) void sigma_update_k(size_t nel, const double* sigma_n,
                                                       const double* A1, const double* A2,
                                                       const double* cur, double* nxt, double c,
                                                       double* res) {
  __shared__ double rd[1024], rn[1024];
  double dd = 0.0, nn = 0.0;
  for (size_t e = threadIdx.x; e < nel; e += blockDim.x) {
    const double gr = A1[2 * e] - A2[2 * e], gi = A1[2 * e + 1] - A2[2 * e + 1];
    // -i c (gr + i gi) = c gi - i c gr
    const double xr = sigma_n[2 * e] + c * gi, xi = sigma_n[2 * e + 1] - c * gr;
    nxt[2 * e] = xr;
    nxt[2 * e + 1] = xi;
    const double dr = xr - cur[2 * e], di = xi - cur[2 * e + 1];
    dd += dr * dr + di * di;
    nn += xr * xr + xi * xi;
  }
  rd[threadIdx.x] = dd;
  rn[threadIdx.x] = nn;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      rd[threadIdx.x] += rd[threadIdx.x + w];
      rn[threadIdx.x] += rn[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *res = rn[0] > 0.0 ? sqrt(rd[0] / rn[0]) : 0.0;
}

hipError_t launch_sigma_update(int n, const double* sigma_n, const double* A1, const double* A2,
                               const double* cur, double* nxt, double c, double* res, hipStream_t s) {
  hipLaunchKernelGGL(sigma_update_k, dim3(1), dim3(1024), 0, s, size_t(n) * n, sigma_n, A1, A2, cur,
                     nxt, c, res);
  return hipGetLastError();
}

// out[0] = the first non-zero of st[0 .. k), else 0
__global__ void status_first_k(const int32_t* st, int k, int32_t* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t v = 0;
  for (int i = 0; i < k && v == 0; ++i) v = st[i];
  out[0] = v;
}

hipError_t launch_status_first(const int32_t* st, int k, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(status_first_k, dim3(1), dim3(64), 0, s, st, k, out);
  return hipGetLastError();
}

}  // namespace px
