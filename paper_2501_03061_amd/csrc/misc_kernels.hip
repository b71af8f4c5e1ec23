// Small kernels around the pair pipeline: the screened kernel table, FP64 ->
// FP32 staging, and the fixed-order FP64 reductions of the exchange energy.
#include "px_internal.hpp"

namespace px {

// K(G) of the HSE06 screened interaction (Fourier transform of erfc(mu r)/r):
// 4 pi (1 - exp(-G^2/(4 mu^2))) / G^2 for G != 0 via expm1, pi/mu^2 at G = 0.
// G = 2 pi m / L per axis, m the signed frequency of the FFT index.
__global__ void kernel_hse_k(int n0, int n1, int n2, double L0, double L1, double L2, double mu,
                             double* kern) {
  const size_t ng = size_t(n0) * n1 * n2;
  for (size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < ng;
       idx += size_t(gridDim.x) * blockDim.x) {
    const int x = int(idx % n0), y = int((idx / n0) % n1), z = int(idx / (size_t(n0) * n1));
    const int mx = (2 * x < n0) ? x : x - n0;
    const int my = (2 * y < n1) ? y : y - n1;
    const int mz = (2 * z < n2) ? z : z - n2;
    const double tp = 6.283185307179586476925286766559;
    const double gx = tp * mx / L0, gy = tp * my / L1, gz = tp * mz / L2;
    const double g2 = gx * gx + gy * gy + gz * gz;
    double k;
    if (g2 > 0.0) k = 4.0 * 3.14159265358979323846264338328 * (-expm1(-g2 / (4.0 * mu * mu))) / g2;
    else k = 3.14159265358979323846264338328 / (mu * mu);
    kern[idx] = k;
  }
}

hipError_t launch_kernel_hse(int n0, int n1, int n2, double L0, double L1, double L2, double mu,
                             double* kern, hipStream_t s) {
  const size_t ng = size_t(n0) * n1 * n2;
  const int blocks = int((ng + 255) / 256 < 65536 ? (ng + 255) / 256 : 65536);
  hipLaunchKernelGGL(kernel_hse_k, dim3(blocks), dim3(256), 0, s, n0, n1, n2, L0, L1, L2, mu, kern);
  return hipGetLastError();
}

typedef double vd4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// Plain device copy, 16 bytes per thread step: the reference kernel for HBM
// counter calibration and the copy-bandwidth ceiling.
__global__ __launch_bounds__(256) void stream_copy_k(size_t n16, const u4* src, u4* dst) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(size_t bytes, const void* src, void* dst, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  const size_t blocks = (n16 + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stream_copy_k, dim3(unsigned(blocks)), dim3(256), 0, s, n16,
                     static_cast<const u4*>(src), static_cast<u4*>(dst));
  return hipGetLastError();
}

typedef float vf4 __attribute__((ext_vector_type(4)));

// complex128 -> complex64, round to nearest even; two complex values per
// thread, one thread per pair (no grid-stride loop: streams at copy speed)
__global__ __launch_bounds__(256) void convert_k(size_t n, const double* src, float* dst) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n / 2) {
    vd4 v = __builtin_nontemporal_load(reinterpret_cast<const vd4*>(src) + i);
    vf4 o = {float(v.x), float(v.y), float(v.z), float(v.w)};
    reinterpret_cast<vf4*>(dst)[i] = o;
  } else if (i == n / 2 && (n & 1)) {
    dst[2 * (n - 1)] = float(src[2 * (n - 1)]);
    dst[2 * (n - 1) + 1] = float(src[2 * (n - 1) + 1]);
  }
}

hipError_t launch_convert_c128_c64(size_t n, const void* src, void* dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = (n / 2 + 1 + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(convert_k, dim3(unsigned(blocks)), dim3(256), 0, s, n,
                     static_cast<const double*>(src), static_cast<float*>(dst));
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void convert_real_k(size_t n, const double* src, float* dst) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = float(src[i]);
}

hipError_t launch_convert_f64_f32(size_t n, const double* src, float* dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(convert_real_k, dim3(unsigned(blocks)), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

// Pair energy S_ij = sum_G K |rho_ij(G)|^2 from the per-plane partials.
// FP32 form: S = K(0)|rho(0)|^2 + A * (N_g E_r - |rho(0)|^2) / B, where A and B
// are the FP32-transform sums of K|rho|^2 and |rho|^2 over G != 0, E_r the
// FP64 energy of the transform input and rho(0) its FP64 sum: the transform's
// systematic norm drift (about 1e-7 relative in FP32) cancels in A / B.
// One wave per pair: lane l adds the planes y = l, l + 64, ... (and the z
// slabs likewise), then the wave adds its lanes in a fixed butterfly order.
// (One thread per pair, as before, left a 1,024-pair chunk to four
// workgroups that walked 432 values each: 42 us per chunk at 72^3.)
__device__ __forceinline__ double lane_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double pair_energy(const double* expart, const G0Part* g0, int p, int n1,
                                              int n2, double ng, int lane) {
  if (g0 == nullptr) {
    double s = 0.0;
    for (int y = lane; y < n1; y += 64) s += expart[size_t(p) * n1 + y];
    return lane_sum(s);
  }
  double a = 0.0, b = 0.0, e0 = 0.0;
  for (int y = lane; y < n1; y += 64) {
    const double* e = expart + (size_t(p) * n1 + y) * 3;
    a += e[0];
    b += e[1];
    e0 += e[2];
  }
  double sr = 0.0, si = 0.0, er = 0.0;
  for (int z = lane; z < n2; z += 64) {
    sr += g0[size_t(p) * n2 + z].re;
    si += g0[size_t(p) * n2 + z].im;
    er += g0[size_t(p) * n2 + z].en;
  }
  a = lane_sum(a);
  b = lane_sum(b);
  e0 = lane_sum(e0);
  sr = lane_sum(sr);
  si = lane_sum(si);
  er = lane_sum(er);
  const double target = ng * er - (sr * sr + si * si);
  return e0 + (b > 0.0 && target > 0.0 ? a * (target / b) : a);
}

__global__ __launch_bounds__(256) void expart_reduce_k(const double* expart, const G0Part* g0,
                                                       int n1, int n2, double ng, int i0, int ic,
                                                       int j0, int jc, double* S, int lds,
                                                       int mirror, int tri) {
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (p >= ic * jc) return;  // wave-uniform
  const int ii = p / jc, jj = p % jc;
  if (tri && jj > ii) return;  // a triangular block solves jj <= ii only
  if (tri) mirror = jj < ii;
  const double s = pair_energy(expart, g0, p, n1, n2, ng, lane);
  if (lane == 0) {
    S[size_t(i0 + ii) * lds + (j0 + jj)] = s;
    if (mirror) S[size_t(j0 + jj) * lds + (i0 + ii)] = s;  // S_ji = S_ij for a real even kernel
  }
}

hipError_t launch_expart_reduce(const double* expart, const G0Part* g0, int n1, int n2, double ng,
                                int i0, int ic, int j0, int jc, double* S, int lds, bool mirror,
                                bool tri, hipStream_t s) {
  const int np = ic * jc;
  hipLaunchKernelGGL(expart_reduce_k, dim3((np + 3) / 4), dim3(256), 0, s, expart, g0, n1, n2,
                     ng, i0, ic, j0, jc, S, lds, int(mirror), int(tri));
  return hipGetLastError();
}

// The same reduction for every chunk of a task table (S, its stride and the
// mirror flag taken from each task).
__global__ __launch_bounds__(256) void expart_reduce_tasks_k(const ChunkArgs* tasks, int fp32,
                                                             int n1, int n2, double ng) {
  const ChunkArgs& a = tasks[blockIdx.y];
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (p >= a.ic * a.jc) return;  // wave-uniform
  const int ii = p / a.jc, jj = p % a.jc;
  if (a.tri && jj > ii) return;  // a triangular block solves jj <= ii only
  const double s = pair_energy(a.expart, fp32 ? a.g0 : nullptr, p, n1, n2, ng, lane);
  if (lane == 0) {
    a.S[size_t(a.i0 + ii) * a.s_ld + (a.j0 + jj)] = s;
    if (a.store_v && (!a.tri || jj < ii)) a.S[size_t(a.j0 + jj) * a.s_ld + (a.i0 + ii)] = s;
  }
}

hipError_t launch_expart_reduce_tasks(bool fp32, const ChunkArgs* tasks, int ntasks, int max_slots,
                                      int n1, int n2, double ng, hipStream_t s) {
  hipLaunchKernelGGL(expart_reduce_tasks_k, dim3((max_slots + 3) / 4, ntasks), dim3(256), 0, s,
                     tasks, int(fp32), n1, n2, ng);
  return hipGetLastError();
}

// e_x = scale * sum_i f_i sum_j f_j S[i][j]; one block, fixed summation order.
__global__ __launch_bounds__(256) void energy_k(const double* S, const double* occ, int n,
                                                double scale, double* e_x) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    double row = 0.0;
    for (int j = 0; j < n; ++j) row += occ[j] * S[size_t(i) * n + j];
    acc += occ[i] * row;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *e_x = scale * red[0];
}

hipError_t launch_energy(const double* S, const double* occ, int n, double scale, double* e_x,
                         hipStream_t s) {
  hipLaunchKernelGGL(energy_k, dim3(1), dim3(256), 0, s, S, occ, n, scale, e_x);
  return hipGetLastError();
}

}  // namespace px

// ---------------------------------------------------------------- PT-IM-style loop
namespace px {

template <typename T> struct V2;
template <> struct V2<double> { typedef double t __attribute__((ext_vector_type(2))); };
template <> struct V2<float> { typedef float t __attribute__((ext_vector_type(2))); };

// mid = (a + b)/2 over n complex values
template <typename T>
__global__ void midpoint_k(size_t n, const T* a, const T* b, T* mid) {
  using V = typename V2<T>::t;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    V x = reinterpret_cast<const V*>(a)[i], y = reinterpret_cast<const V*>(b)[i];
    V m = {T(0.5) * (x.x + y.x), T(0.5) * (x.y + y.y)};
    reinterpret_cast<V*>(mid)[i] = m;
  }
}

// nxt = phi_n - i*c*(y + y2) (y2 nullable); per-block FP64 partials of
// |nxt - cur|^2 and |nxt|^2
template <typename T>
__global__ __launch_bounds__(256) void ptim_update_k(size_t n, const T* phi_n, const T* y,
                                                     const T* y2, const T* cur, T* nxt, double c,
                                                     double* partial) {
  using V = typename V2<T>::t;
  __shared__ double red[2][256];
  double dd = 0.0, nn = 0.0;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    V p = reinterpret_cast<const V*>(phi_n)[i], v = reinterpret_cast<const V*>(y)[i];
    double vr = double(v.x), vi = double(v.y);
    if (y2) {  // the two terms are added in FP64
      const V w = reinterpret_cast<const V*>(y2)[i];
      vr += double(w.x);
      vi += double(w.y);
    }
    V q = reinterpret_cast<const V*>(cur)[i];
    // -i c (vr + i vi) = c vi - i c vr
    const double nr = double(p.x) + c * vi, ni = double(p.y) - c * vr;
    V o = {T(nr), T(ni)};
    reinterpret_cast<V*>(nxt)[i] = o;
    const double dr = double(o.x) - double(q.x), di = double(o.y) - double(q.y);
    dd += dr * dr + di * di;
    nn += double(o.x) * double(o.x) + double(o.y) * double(o.y);
  }
  red[0][threadIdx.x] = dd;
  red[1][threadIdx.x] = nn;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = red[0][0];
    partial[2 * blockIdx.x + 1] = red[1][0];
  }
}

// res = sqrt(sum dd / sum nn) over nblocks partials, fixed order
__global__ void residual_k(const double* partial, int nblocks, double* res) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nblocks; ++k) {
    a += partial[2 * k];
    b += partial[2 * k + 1];
  }
  *res = sqrt(a / b);
}

constexpr int kUpdateBlocks = 1024;

int ptim_update_blocks() { return kUpdateBlocks; }

hipError_t launch_midpoint(bool fp32, size_t n, const void* a, const void* b, void* mid,
                           hipStream_t s) {
  const int blocks = int((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
  if (fp32)
    hipLaunchKernelGGL(midpoint_k<float>, dim3(blocks), dim3(256), 0, s, n,
                       static_cast<const float*>(a), static_cast<const float*>(b),
                       static_cast<float*>(mid));
  else
    hipLaunchKernelGGL(midpoint_k<double>, dim3(blocks), dim3(256), 0, s, n,
                       static_cast<const double*>(a), static_cast<const double*>(b),
                       static_cast<double*>(mid));
  return hipGetLastError();
}

hipError_t launch_ptim_update(bool fp32, size_t n, const void* phi_n, const void* y,
                              const void* y2, const void* cur, void* nxt, double c, double* partial,
                              double* res, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(ptim_update_k<float>, dim3(kUpdateBlocks), dim3(256), 0, s, n,
                       static_cast<const float*>(phi_n), static_cast<const float*>(y),
                       static_cast<const float*>(y2), static_cast<const float*>(cur),
                       static_cast<float*>(nxt), c, partial);
  else
    hipLaunchKernelGGL(ptim_update_k<double>, dim3(kUpdateBlocks), dim3(256), 0, s, n,
                       static_cast<const double*>(phi_n), static_cast<const double*>(y),
                       static_cast<const double*>(y2), static_cast<const double*>(cur),
                       static_cast<double*>(nxt), c, partial);
  hipLaunchKernelGGL(residual_k, dim3(1), dim3(64), 0, s, partial, kUpdateBlocks, res);
  return hipGetLastError();
}

}  // namespace px

// ---------------------------------------------------------------- density
namespace px {

// rho(r) = sum_i w_i |phi_i(r)|^2 with the occupation-matrix eigenvalues w_i
// (Eq. 12 with sigma diagonalised: N products instead of N^2), accumulated in
// FP64 from the orbital values.  Two consecutive grid points per thread: one
// 16-byte load per orbital in the FP32 form (N_g even), two in FP64; the
// orbital loop is unrolled so that several loads are in flight.
template <typename T>
__global__ __launch_bounds__(256) void density_k(size_t ng, int n, const T* phi, const double* w,
                                                 double* rho) {
  using V = typename V2<T>::t;
  const size_t r = (size_t(blockIdx.x) * blockDim.x + threadIdx.x) * 2;
  if (r >= ng) return;
  const bool two = r + 1 < ng;
  double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
  for (int i = 0; i < n; ++i) {
    const V* p = reinterpret_cast<const V*>(phi) + size_t(i) * ng + r;
    const V x = p[0];
    const V y = two ? p[1] : V{T(0), T(0)};
    const double wi = w[i];
    a0 += wi * (double(x.x) * double(x.x) + double(x.y) * double(x.y));
    a1 += wi * (double(y.x) * double(y.x) + double(y.y) * double(y.y));
  }
  rho[r] = a0;
  if (two) rho[r + 1] = a1;
}

hipError_t launch_density(bool fp32, size_t ng, int n, const void* phi, const double* w,
                          double* rho, hipStream_t s) {
  const size_t threads = (ng + 1) / 2;
  const unsigned blocks = unsigned((threads + 255) / 256);
  if (fp32)
    hipLaunchKernelGGL(density_k<float>, dim3(blocks), dim3(256), 0, s, ng, n,
                       static_cast<const float*>(phi), w, rho);
  else
    hipLaunchKernelGGL(density_k<double>, dim3(blocks), dim3(256), 0, s, ng, n,
                       static_cast<const double*>(phi), w, rho);
  return hipGetLastError();
}

}  // namespace px
