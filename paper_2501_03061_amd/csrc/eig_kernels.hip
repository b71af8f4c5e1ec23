// FP64 Hermitian eigendecomposition of the occupation matrix, sigma = Q D Q^H
// (Sec. IV-A-1, Eq. 11), by the cyclic Jacobi method in a blocked parallel
// ordering.
//
// The indices are cut into blocks of BJ = 16 (nb blocks, rounded up to even;
// indices past n are absent).  A sweep visits every pair of blocks once, in
// nb - 1 rounds of nb/2 disjoint block pairs (the circle method: block nb - 1
// stays put, the others rotate).  In a round, one workgroup per block pair
// takes the 32 x 32 Hermitian submatrix of its 32 indices into LDS and runs
// one sweep of scalar cyclic Jacobi on it (31 rounds of 16 disjoint index
// pairs in the same circle ordering; each pair gets the unitary G = P J that
// zeroes its off-diagonal entry: with A_pq = |A_pq| e^{i theta},
// P = diag(1, e^{-i theta}) makes the 2 x 2 block real symmetric and J is its
// real Jacobi rotation, tangent t = sgn(tau)/(|tau| + sqrt(1 + tau^2)),
// tau = (A_qq - A_pp)/(2 |A_pq|), the smaller angle), accumulating the 32 x 32
// unitary U of the pair.  The U of a round act on disjoint index sets, so
// A <- G^H A G splits into 32 x 32 tiles A_PS <- U_P^H A_PS U_S and V <- V G
// into 32-row tiles V_rS <- V_rS U_S, one workgroup per tile.  Compared with
// rotating single index pairs, a sweep reads and writes A and V nb - 1 times
// instead of n - 1 times, which is what bounds the method at these sizes.
// After each sweep the off-diagonal Frobenius norm is formed (partial sums,
// then a fixed-order total); below
// 64 eps sqrt(n) ||A||_F a device flag makes the remaining launches return at
// once, so the host enqueues a fixed number of sweeps without waiting for the
// device.  Finally d = diag(A) in ascending order, Q the matching columns of V.
#include <float.h>

#include "px_internal.hpp"

namespace px {

namespace {

struct Rot {
  double c, s;    // real rotation
  double er, ei;  // e^{-i theta}
  int p, q;       // the pair; q = -1 when the partner is the padding index
  int id;         // 1: identity (padding pair or zero off-diagonal entry)
  int pad;
};

// Pair `slot` of round k (0 <= k < np - 1) of the circle ordering of np
// (even) indices; p < q.
__device__ __forceinline__ void round_pair(int np, int k, int slot, int& p, int& q) {
  const int m = np - 1;
  int a, b;
  if (slot == 0) {
    a = k % m;
    b = m;
  } else {
    a = (k + slot) % m;
    b = (k - slot + m) % m;
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj2(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Entries of G (2 x 2): g00 = c, g01 = s, g10 = -s e, g11 = c e, e = e^{-i theta}.
__device__ __forceinline__ void rot_matrix(const Rot& r, double2 g[2][2]) {
  if (r.id) {
    g[0][0] = make_double2(1.0, 0.0);
    g[0][1] = make_double2(0.0, 0.0);
    g[1][0] = make_double2(0.0, 0.0);
    g[1][1] = make_double2(1.0, 0.0);
    return;
  }
  g[0][0] = make_double2(r.c, 0.0);
  g[0][1] = make_double2(r.s, 0.0);
  g[1][0] = make_double2(-r.s * r.er, -r.s * r.ei);
  g[1][1] = make_double2(r.c * r.er, r.c * r.ei);
}

__device__ __forceinline__ double2 ld2(const double* A, int n, int r, int c) {
  return *reinterpret_cast<const double2*>(A + (size_t(r) * n + c) * 2);
}
__device__ __forceinline__ void st2(double* A, int n, int r, int c, double2 v) {
  *reinterpret_cast<double2*>(A + (size_t(r) * n + c) * 2) = v;
}

// A = (sigma + sigma^H)/2, V = I, flags cleared.
__global__ void eig_init_k(const double* sigma, int n, double* A, double* V, int* flags) {
  const size_t total = size_t(n) * n;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += size_t(gridDim.x) * blockDim.x) {
    const int i = int(e / n), j = int(e % n);
    const double2 a = ld2(sigma, n, i, j), b = ld2(sigma, n, j, i);
    st2(A, n, i, j, make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y)));
    st2(V, n, i, j, make_double2(i == j ? 1.0 : 0.0, 0.0));
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    flags[0] = 0;  // converged
    flags[1] = 0;  // sweeps completed
  }
}

constexpr int BJ = 16;        // indices per block
constexpr int BJ2 = 2 * BJ;   // size of a block pair's subproblem

// Index t (0 <= t < 32) of block pair `slot` in block round k: block I's 16
// indices, then block J's.
__device__ __forceinline__ int bj_index(int nb, int k, int slot, int t) {
  int I, J;
  round_pair(nb, k, slot, I, J);
  return t < BJ ? I * BJ + t : J * BJ + (t - BJ);
}

// Rotation of indices (p, q) of the 2 x 2 diagonal block (app, aqq real, apq).
__device__ __forceinline__ Rot make_rot(double app, double aqq, double2 apq, int p, int q) {
  Rot r;
  r.p = p;
  r.q = q;
  r.id = 1;
  r.pad = 0;
  r.c = 1.0;
  r.s = 0.0;
  r.er = 1.0;
  r.ei = 0.0;
  const double m = hypot(apq.x, apq.y);
  if (m > 0.0) {
    const double tau = (aqq - app) / (2.0 * m);
    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    r.c = 1.0 / sqrt(1.0 + t * t);
    r.s = t * r.c;
    r.er = apq.x / m;  // e^{-i theta} = conj(A_pq)/|A_pq|
    r.ei = -apq.y / m;
    r.id = 0;
  }
  return r;
}

// One inner sweep on the 32 x 32 subproblem of each block pair of round k
// (one workgroup per pair): U_P (32 x 32, row-major) into Ug[P].
__global__ __launch_bounds__(256) void bj_solve_k(const double* A, int n, int nb, int k, double* Ug,
                                                  const int* flags) {
  if (flags[0]) return;
  __shared__ double2 S[BJ2][BJ2 + 1];
  __shared__ double2 U[BJ2][BJ2 + 1];
  __shared__ Rot rot[BJ];
  __shared__ int gi[BJ2];
  const int P = blockIdx.x, tid = threadIdx.x;
  if (tid < BJ2) gi[tid] = bj_index(nb, k, P, tid);
  __syncthreads();
  for (int e = tid; e < BJ2 * BJ2; e += 256) {
    const int i = e / BJ2, j = e % BJ2;
    S[i][j] = (gi[i] < n && gi[j] < n) ? ld2(A, n, gi[i], gi[j]) : make_double2(0.0, 0.0);
    U[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int kk = 0; kk < BJ2 - 1; ++kk) {
    if (tid < BJ) {
      int p, q;
      round_pair(BJ2, kk, tid, p, q);
      rot[tid] = make_rot(S[p][p].x, S[q][q].x, S[p][q], p, q);
    }
    __syncthreads();
    {  // S <- G^H S G on the 2 x 2 blocks (pair x, pair y): 16 x 16 = 256 blocks
      const Rot rp = rot[tid / BJ], rs = rot[tid % BJ];
      if (!(rp.id && rs.id)) {
        double2 gp[2][2], gs[2][2], b[2][2], t[2][2];
        rot_matrix(rp, gp);
        rot_matrix(rs, gs);
        const int ip[2] = {rp.p, rp.q}, is[2] = {rs.p, rs.q};
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) b[x][y] = S[ip[x]][is[y]];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) t[x][y] = cadd2(cmul2(b[x][0], gs[0][y]), cmul2(b[x][1], gs[1][y]));
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            S[ip[x]][is[y]] = cadd2(cmul2(cconj2(gp[0][x]), t[0][y]), cmul2(cconj2(gp[1][x]), t[1][y]));
      }
    }
    for (int e = tid; e < BJ2 * BJ; e += 256) {  // U <- U G: (row, pair) pieces
      const int r = e / BJ;
      const Rot rs = rot[e % BJ];
      if (rs.id) continue;
      double2 g[2][2];
      rot_matrix(rs, g);
      const double2 v0 = U[r][rs.p], v1 = U[r][rs.q];
      U[r][rs.p] = cadd2(cmul2(v0, g[0][0]), cmul2(v1, g[1][0]));
      U[r][rs.q] = cadd2(cmul2(v0, g[0][1]), cmul2(v1, g[1][1]));
    }
    __syncthreads();
  }
  double2* out = reinterpret_cast<double2*>(Ug) + size_t(P) * BJ2 * BJ2;
  for (int e = tid; e < BJ2 * BJ2; e += 256) out[e] = U[e / BJ2][e % BJ2];
}

// The block rotations of round k: A_PS <- U_P^H A_PS U_S for every pair of
// block pairs (blockIdx.y = 0, blockIdx.x = P * m + S), V_rS <- V_rS U_S for
// every 32-row tile r and block pair S (blockIdx.y = 1, blockIdx.x = r * m + S).
// Each tile is read and written by its own workgroup only.
__global__ __launch_bounds__(256) void bj_apply_k(double* A, double* V, int n, int nb, int k,
                                                  const double* Ug, const int* flags) {
  if (flags[0]) return;
  const int m = nb / 2, tid = threadIdx.x;
  const int rows = (n + BJ2 - 1) / BJ2;
  const bool is_a = blockIdx.y == 0;
  if (blockIdx.x >= unsigned(is_a ? m * m : rows * m)) return;
  __shared__ double2 X[BJ2][BJ2 + 1];
  __shared__ double2 W[BJ2][BJ2 + 1];
  __shared__ int ri[BJ2], ci[BJ2];
  const int P = blockIdx.x / m, Sx = blockIdx.x % m;
  if (tid < BJ2) {
    ri[tid] = is_a ? bj_index(nb, k, P, tid) : P * BJ2 + tid;
    ci[tid] = bj_index(nb, k, Sx, tid);
  }
  __syncthreads();
  double* M = is_a ? A : V;
  const double2* us = reinterpret_cast<const double2*>(Ug) + size_t(Sx) * BJ2 * BJ2;
  for (int e = tid; e < BJ2 * BJ2; e += 256) {
    const int i = e / BJ2, j = e % BJ2;
    X[i][j] = (ri[i] < n && ci[j] < n) ? ld2(M, n, ri[i], ci[j]) : make_double2(0.0, 0.0);
    W[i][j] = us[e];
  }
  __syncthreads();
  // T = X U_S: four entries per thread, rows i0 + 8q of one column j (each
  // entry of U_S read once for the four)
  const int i0 = tid / BJ2, j = tid % BJ2;
  double2 t[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) t[q] = make_double2(0.0, 0.0);
#pragma unroll 8
  for (int l = 0; l < BJ2; ++l) {
    const double2 w = W[l][j];
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] = cadd2(t[q], cmul2(X[i0 + 8 * q][l], w));
  }
  if (is_a) {
    // out = U_P^H T
    __syncthreads();
    const double2* up = reinterpret_cast<const double2*>(Ug) + size_t(P) * BJ2 * BJ2;
#pragma unroll
    for (int q = 0; q < 4; ++q) X[i0 + 8 * q][j] = t[q];
    for (int e = tid; e < BJ2 * BJ2; e += 256) W[e / BJ2][e % BJ2] = up[e];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] = make_double2(0.0, 0.0);
#pragma unroll 8
    for (int l = 0; l < BJ2; ++l) {
      const double2 x = X[l][j];
#pragma unroll
      for (int q = 0; q < 4; ++q) t[q] = cadd2(t[q], cmul2(cconj2(W[l][i0 + 8 * q]), x));
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + 8 * q;
    if (ri[i] < n && ci[j] < n) st2(M, n, ri[i], ci[j], t[q]);
  }
}

// End of a sweep: off-diagonal and total squared Frobenius norms, first as
// partial sums of kConvBlocks workgroups (a strided share of the entries
// each), then summed in fixed order by one workgroup, which sets the
// convergence flag.
constexpr int kConvBlocks = 256;

__global__ __launch_bounds__(256) void eig_norm_part_k(const double* A, int n, double* part, const int* flags) {
  __shared__ double so[256], st[256];
  if (flags[0]) return;
  double off = 0.0, tot = 0.0;
  const size_t total = size_t(n) * n;
  for (size_t e = size_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += size_t(kConvBlocks) * 256) {
    const int i = int(e / n), j = int(e % n);
    const double2 a = ld2(A, n, i, j);
    const double m2 = a.x * a.x + a.y * a.y;
    tot += m2;
    if (i != j) off += m2;
  }
  so[threadIdx.x] = off;
  st[threadIdx.x] = tot;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      st[threadIdx.x] += st[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = so[0];
    part[2 * blockIdx.x + 1] = st[0];
  }
}

__global__ __launch_bounds__(kConvBlocks) void eig_conv_k(const double* part, int n, int* flags) {
  __shared__ double so[kConvBlocks], st[kConvBlocks];
  if (flags[0]) return;
  so[threadIdx.x] = part[2 * threadIdx.x];
  st[threadIdx.x] = part[2 * threadIdx.x + 1];
  __syncthreads();
  for (int w = kConvBlocks / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      st[threadIdx.x] += st[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double tol = 64.0 * DBL_EPSILON * sqrt(double(n > 1 ? n : 1));
    flags[1] += 1;
    if (so[0] <= tol * tol * st[0]) flags[0] = 1;
  }
}

// Ascending order of the eigenvalues (ties by index): rank of each, d in
// order, and the status word (0 converged, else the sweeps made).
__global__ void eig_rank_k(const double* A, int n, int* rank, double* d, const int* flags,
                           int32_t* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) status[0] = flags[0] ? 0 : (flags[1] > 0 ? flags[1] : 1);
  if (i >= n) return;
  const double di = ld2(A, n, i, i).x;
  int r = 0;
  for (int j = 0; j < n; ++j) {
    const double dj = ld2(A, n, j, j).x;
    r += (dj < di || (dj == di && j < i)) ? 1 : 0;
  }
  rank[i] = r;
  d[r] = di;
}

// Q[:, rank[i]] = V[:, i]
__global__ void eig_permute_k(const double* V, int n, const int* rank, double* Q) {
  const size_t total = size_t(n) * n;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += size_t(gridDim.x) * blockDim.x) {
    const int r = int(e / n), i = int(e % n);
    st2(Q, n, r, rank[i], ld2(V, n, r, i));
  }
}

int grid_for(size_t total) {
  const size_t b = (total + 255) / 256;
  return int(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

int eig_blocks(int n) {
  const int nb = (n + BJ - 1) / BJ;
  return nb + (nb & 1) < 2 ? 2 : nb + (nb & 1);
}

size_t eig_work_bytes(int n) {
  const size_t mat = size_t(n) * n * 16;
  const size_t ug = size_t(eig_blocks(n) / 2) * BJ2 * BJ2 * 16;
  return 2 * mat + ug + size_t(2 * kConvBlocks) * sizeof(double) + size_t(n) * sizeof(int) + 4 * sizeof(int) +
         5 * 256;
}

hipError_t launch_eig_hermitian(const double* sigma, int n, double* Q, double* d, int32_t* status,
                                void* work, int max_sweeps, hipStream_t s) {
  const int nb = eig_blocks(n), m = nb / 2;
  char* w = static_cast<char*>(work);
  auto carve = [&w](size_t bytes) {
    char* p = w;
    w += (bytes + 255) / 256 * 256;
    return p;
  };
  double* A = reinterpret_cast<double*>(carve(size_t(n) * n * 16));
  double* V = reinterpret_cast<double*>(carve(size_t(n) * n * 16));
  double* Ug = reinterpret_cast<double*>(carve(size_t(m) * BJ2 * BJ2 * 16));
  double* part = reinterpret_cast<double*>(carve(size_t(2 * kConvBlocks) * sizeof(double)));
  int* rank = reinterpret_cast<int*>(carve(size_t(n) * sizeof(int)));
  int* flags = reinterpret_cast<int*>(carve(4 * sizeof(int)));
  const size_t total = size_t(n) * n;
  hipLaunchKernelGGL(eig_init_k, dim3(grid_for(total)), dim3(256), 0, s, sigma, n, A, V, flags);
  if (n > 1) {
    const int rows = (n + BJ2 - 1) / BJ2;
    const int tiles = m * m > rows * m ? m * m : rows * m;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
      for (int k = 0; k < nb - 1; ++k) {
        hipLaunchKernelGGL(bj_solve_k, dim3(m), dim3(256), 0, s, A, n, nb, k, Ug, flags);
        hipLaunchKernelGGL(bj_apply_k, dim3(tiles, 2), dim3(256), 0, s, A, V, n, nb, k, Ug, flags);
      }
      hipLaunchKernelGGL(eig_norm_part_k, dim3(kConvBlocks), dim3(256), 0, s, A, n, part, flags);
      hipLaunchKernelGGL(eig_conv_k, dim3(1), dim3(kConvBlocks), 0, s, part, n, flags);
    }
  } else {
    hipLaunchKernelGGL(eig_norm_part_k, dim3(kConvBlocks), dim3(256), 0, s, A, n, part, flags);
    hipLaunchKernelGGL(eig_conv_k, dim3(1), dim3(kConvBlocks), 0, s, part, n, flags);
  }
  hipLaunchKernelGGL(eig_rank_k, dim3((n + 255) / 256), dim3(256), 0, s, A, n, rank, d, flags, status);
  hipLaunchKernelGGL(eig_permute_k, dim3(grid_for(total)), dim3(256), 0, s, V, n, rank, Q);
  return hipGetLastError();
}

}  // namespace px
