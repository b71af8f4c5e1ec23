// FP64 Hermitian eigendecomposition of the occupation matrix, sigma = Q D Q^H
// (Sec. IV-A-1, Eq. 11), by the cyclic Jacobi method in a parallel ordering.
//
// A sweep visits every index pair (p, q) once, in n' - 1 rounds of n'/2
// disjoint pairs (n' = n rounded up to even; the circle method: index n' - 1
// stays put, the others rotate, and a pair with the padding index n is
// skipped).  In a round, each pair gets the unitary G = P J that zeroes its
// off-diagonal entry: with A_pq = |A_pq| e^{i theta}, P = diag(1, e^{-i theta})
// makes the 2 x 2 block real symmetric and J is the real Jacobi rotation of
// that block (tangent t = sgn(tau)/(|tau| + sqrt(1 + tau^2)),
// tau = (A_qq - A_pp)/(2 |A_pq|), the smaller of the two angles).  The
// rotations of a round are disjoint, so A <- G^H A G and V <- V G split into
// independent 2 x 2 blocks: one thread per block updates A in place (every
// rotation was formed from the diagonal blocks before any update) and one per
// (row, pair) updates V.  After each sweep one workgroup forms the off-diagonal
// Frobenius norm; below 64 eps sqrt(n) ||A||_F a device flag makes the
// remaining launches return at once, so the host enqueues a fixed number of
// sweeps without waiting for the device.  Finally d = diag(A) in ascending
// order, Q the matching columns of V.
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

// The rotations of round k, one thread per pair.
__global__ void eig_rot_k(const double* A, int n, int np, int k, Rot* rot, const int* flags) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= np / 2 || flags[0]) return;
  int p, q;
  round_pair(np, k, slot, p, q);
  Rot r;
  r.p = p;
  r.q = q < n ? q : -1;
  r.id = 1;
  r.pad = 0;
  r.c = 1.0;
  r.s = 0.0;
  r.er = 1.0;
  r.ei = 0.0;
  if (q < n) {
    const double app = ld2(A, n, p, p).x, aqq = ld2(A, n, q, q).x;
    const double2 apq = ld2(A, n, p, q);
    const double m = hypot(apq.x, apq.y);
    if (m > 0.0) {
      const double tau = (aqq - app) / (2.0 * m);
      const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      r.c = 1.0 / sqrt(1.0 + t * t);
      r.s = t * r.c;
      r.er = apq.x / m;   // e^{-i theta} = conj(A_pq)/|A_pq|
      r.ei = -apq.y / m;
      r.id = 0;
    }
  }
  rot[slot] = r;
}

// A <- G^H A G on the 2 x 2 blocks (pair P, pair S) (blockIdx.y = 0), and
// V <- V G on the (row, pair) pieces (blockIdx.y = 1).
__global__ void eig_apply_k(double* A, double* V, int n, int np, const Rot* rot, const int* flags) {
  if (flags[0]) return;
  const int half = np / 2;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (blockIdx.y == 0) {
    if (e >= size_t(half) * half) return;
    const int P = int(e / half), S = int(e % half);
    const Rot rp = rot[P], rs = rot[S];
    if (rp.id && rs.id) return;  // both identities: the block keeps its values
    double2 gp[2][2], gs[2][2];
    rot_matrix(rp, gp);
    rot_matrix(rs, gs);
    // rows of pair P, columns of pair S (-1: the padding index, left out;
    // the partner of an identity pair takes part with a unit rotation)
    const int ip[2] = {rp.p, rp.q}, is[2] = {rs.p, rs.q};
    double2 b[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        b[x][y] = (ip[x] >= 0 && is[y] >= 0) ? ld2(A, n, ip[x], is[y]) : make_double2(0.0, 0.0);
    // T = B G_S, A' = G_P^H T
    double2 t[2][2], o[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) t[x][y] = cadd2(cmul2(b[x][0], gs[0][y]), cmul2(b[x][1], gs[1][y]));
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        o[x][y] = cadd2(cmul2(cconj2(gp[0][x]), t[0][y]), cmul2(cconj2(gp[1][x]), t[1][y]));
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        if (ip[x] >= 0 && is[y] >= 0) st2(A, n, ip[x], is[y], o[x][y]);
  } else {
    if (e >= size_t(n) * half) return;
    const int r = int(e / half), S = int(e % half);
    const Rot rs = rot[S];
    if (rs.id) return;
    double2 g[2][2];
    rot_matrix(rs, g);
    const double2 v0 = ld2(V, n, r, rs.p), v1 = ld2(V, n, r, rs.q);
    st2(V, n, r, rs.p, cadd2(cmul2(v0, g[0][0]), cmul2(v1, g[1][0])));
    st2(V, n, r, rs.q, cadd2(cmul2(v0, g[0][1]), cmul2(v1, g[1][1])));
  }
}

// End of a sweep: off-diagonal and total Frobenius norms (one workgroup, fixed
// order); sets the convergence flag.
__global__ __launch_bounds__(1024) void eig_conv_k(const double* A, int n, int* flags) {
  __shared__ double so[1024], st[1024];
  if (flags[0]) return;
  double off = 0.0, tot = 0.0;
  const size_t total = size_t(n) * n;
  for (size_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = int(e / n), j = int(e % n);
    const double2 a = ld2(A, n, i, j);
    const double m2 = a.x * a.x + a.y * a.y;
    tot += m2;
    if (i != j) off += m2;
  }
  so[threadIdx.x] = off;
  st[threadIdx.x] = tot;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
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

size_t eig_work_bytes(int n) {
  const int np = n + (n & 1);
  const size_t mat = size_t(n) * n * 16;
  return 2 * mat + size_t(np / 2) * sizeof(Rot) + size_t(n) * sizeof(int) + 4 * sizeof(int) + 4 * 256;
}

hipError_t launch_eig_hermitian(const double* sigma, int n, double* Q, double* d, int32_t* status,
                                void* work, int max_sweeps, hipStream_t s) {
  const int np = n + (n & 1);
  char* w = static_cast<char*>(work);
  auto carve = [&w](size_t bytes) {
    char* p = w;
    w += (bytes + 255) / 256 * 256;
    return p;
  };
  double* A = reinterpret_cast<double*>(carve(size_t(n) * n * 16));
  double* V = reinterpret_cast<double*>(carve(size_t(n) * n * 16));
  Rot* rot = reinterpret_cast<Rot*>(carve(size_t(np / 2) * sizeof(Rot)));
  int* rank = reinterpret_cast<int*>(carve(size_t(n) * sizeof(int)));
  int* flags = reinterpret_cast<int*>(carve(4 * sizeof(int)));
  const size_t total = size_t(n) * n;
  hipLaunchKernelGGL(eig_init_k, dim3(grid_for(total)), dim3(256), 0, s, sigma, n, A, V, flags);
  if (n > 1) {
    const int half = np / 2;
    const size_t work_a = size_t(half) * half, work_v = size_t(n) * half;
    const size_t most = work_a > work_v ? work_a : work_v;
    const dim3 ga(unsigned((most + 255) / 256), 2);
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
      for (int k = 0; k < np - 1; ++k) {
        hipLaunchKernelGGL(eig_rot_k, dim3((half + 255) / 256), dim3(256), 0, s, A, n, np, k, rot,
                           flags);
        hipLaunchKernelGGL(eig_apply_k, ga, dim3(256), 0, s, A, V, n, np, rot, flags);
      }
      hipLaunchKernelGGL(eig_conv_k, dim3(1), dim3(1024), 0, s, A, n, flags);
    }
  } else {
    hipLaunchKernelGGL(eig_conv_k, dim3(1), dim3(1024), 0, s, A, n, flags);
  }
  hipLaunchKernelGGL(eig_rank_k, dim3((n + 255) / 256), dim3(256), 0, s, A, n, rank, d, flags, status);
  hipLaunchKernelGGL(eig_permute_k, dim3(grid_for(total)), dim3(256), 0, s, V, n, rank, Q);
  return hipGetLastError();
}

}  // namespace px
