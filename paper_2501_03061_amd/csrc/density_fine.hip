// The density on the charge-density grid (Sec. VI: twice as fine per axis as
// the wavefunction grid) for orbitals with occupations, rho_f = sum_i occ_i
// |phi_i^f|^2 (Eq. 12's diagonal form), phi_i^f the trigonometric
// interpolation of phi_i: its spectrum zero-padded, the Nyquist coefficient of
// each (even) axis split evenly between +n/2 and -n/2.
//
// The interpolation is separable and, per axis of length n, a real circular
// convolution: the even fine points are the samples, out[2j] = in[j], and the
// odd ones out[2j+1] = sum_k h[(j - k) mod n] in[k] with
//   h[t] = (1 + 2 sum_{g=1}^{n/2-1} cos(pi g (2t+1)/n)) / n
// (the Nyquist term cos(pi n u / L) vanishes halfway between samples).  Per
// chunk of orbitals: x, then y (each pass doubles one axis; lines staged in
// LDS, each thread computing JB consecutive odd points of one line with a
// sliding window of h in registers), then z, the largest pass, on the matrix
// cores: the odd z planes of a chunk are O = H^T Y with Y its y-refined data
// laid out [n2][orbital][4 n0 n1] and H[k][j] = h[(j - k) mod n2] (one xc
// contraction), the even ones are Y itself; finally the weighted squares of
// both summed into rho_f in FP64.  The interpolation runs in the form's
// precision.
#include "density_fine.hpp"

#include "fft_core.hpp"
#include "px_internal.hpp"

namespace px {

namespace {

template <typename T> using C = cpx<T>;

template <typename T> __device__ __forceinline__ C<T> cfma(T a, C<T> x, C<T> acc) {
  return C<T>{acc.x + a * x.x, acc.y + a * x.y};
}

// h[t] for the three axes: tables at h + a * hstride, computed in FP64.
template <typename T>
__global__ void interp_table_k(int n0, int n1, int n2, int hstride, T* h) {
  const int a = blockIdx.y;
  const int n = a == 0 ? n0 : a == 1 ? n1 : n2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double s = 1.0;
  for (int g = 1; g < n / 2; ++g) s += 2.0 * cos(3.14159265358979323846 * g * (2.0 * t + 1.0) / n);
  h[a * hstride + t] = T(s / n);
}

// Odd points j0 .. j0 + JB - 1 of one line of length n held at stride `st`
// in LDS: out_j = sum_k h[(j - k) mod n] line[k], with the JB values of h a
// thread needs for one k kept in registers and shifted by one per k.
constexpr int JB = 8;
template <typename T>
__device__ __forceinline__ void odd_block(const C<T>* line, int st, int n, const T* hs, int j0, C<T> acc[JB]) {
  T hw[JB];
#pragma unroll
  for (int q = 0; q < JB; ++q) {
    acc[q] = C<T>{T(0), T(0)};
    hw[q] = hs[(j0 + q) % n];  // k = 0
  }
  for (int k = 0; k < n; ++k) {
    const C<T> x = line[k * st];
#pragma unroll
    for (int q = 0; q < JB; ++q) acc[q] = cfma(hw[q], x, acc[q]);
    // next k: hw[q] = h[(j0 + q - k - 1) mod n] = the current hw[q - 1]
#pragma unroll
    for (int q = JB - 1; q > 0; --q) hw[q] = hw[q - 1];
    int t = j0 - k - 1;
    t += t < 0 ? n : 0;
    hw[0] = hs[t];
  }
}

// x: rows of n0 contiguous values -> rows of 2 n0; RB rows per workgroup.
constexpr int RB = 8;
template <typename T>
__global__ __launch_bounds__(256) void interp_x_k(size_t rows, int n0, const C<T>* in, C<T>* out,
                                                  const T* h) {
  extern __shared__ unsigned char smem[];
  C<T>* line = reinterpret_cast<C<T>*>(smem);  // RB x n0
  T* hs = reinterpret_cast<T*>(line + RB * n0);
  const size_t r0 = size_t(blockIdx.x) * RB;
  const int nr = rows - r0 < size_t(RB) ? int(rows - r0) : RB;
  for (int e = threadIdx.x; e < nr * n0; e += 256) line[e] = in[r0 * n0 + e];
  for (int e = threadIdx.x; e < n0; e += 256) hs[e] = h[e];
  __syncthreads();
  const int w = 2 * n0;
  for (int e = threadIdx.x; e < nr * n0; e += 256) {  // even points: the samples
    const int r = e / n0, j = e % n0;
    out[(r0 + r) * w + 2 * j] = line[r * n0 + j];
  }
  const int nb = (n0 + JB - 1) / JB;  // odd blocks per row
  for (int e = threadIdx.x; e < nr * nb; e += 256) {
    const int r = e / nb, j0 = (e % nb) * JB;
    C<T> acc[JB];
    odd_block(line + r * n0, 1, n0, hs, j0, acc);
#pragma unroll
    for (int q = 0; q < JB; ++q)
      if (j0 + q < n0) out[(r0 + r) * w + 2 * (j0 + q) + 1] = acc[q];
  }
}

// A strided axis: in [outer][na][inner] -> out [outer'][2 na][inner]; a
// workgroup takes one outer index and IB consecutive inner positions.  With
// zdim > 0 the outer index o = b zdim + z is written at position z bdim + b
// (orbital-major in, plane-major out).
constexpr int IB = 32;
template <typename T>
__global__ __launch_bounds__(256) void interp_strided_k(int na, size_t inner, const C<T>* in, C<T>* out,
                                                        const T* h, int zdim, int bdim) {
  extern __shared__ unsigned char smem[];
  C<T>* tile = reinterpret_cast<C<T>*>(smem);  // na x IB
  T* hs = reinterpret_cast<T*>(tile + na * IB);
  const size_t o = blockIdx.y;
  const size_t i0 = size_t(blockIdx.x) * IB;
  const int ni = inner - i0 < size_t(IB) ? int(inner - i0) : IB;
  const C<T>* src = in + o * na * inner + i0;
  for (int e = threadIdx.x; e < na * IB; e += 256) {
    const int k = e / IB, i = e % IB;
    if (i < ni) tile[e] = src[size_t(k) * inner + i];
  }
  for (int e = threadIdx.x; e < na; e += 256) hs[e] = h[e];
  __syncthreads();
  const size_t oo = zdim > 0 ? (o % zdim) * bdim + o / zdim : o;
  C<T>* dst = out + oo * 2 * na * inner + i0;
  for (int e = threadIdx.x; e < na * IB; e += 256) {  // even points
    const int j = e / IB, i = e % IB;
    if (i < ni) dst[size_t(2 * j) * inner + i] = tile[e];
  }
  const int nb = (na + JB - 1) / JB;
  for (int e = threadIdx.x; e < nb * IB; e += 256) {  // odd points, JB per thread
    const int j0 = (e / IB) * JB, i = e % IB;
    if (i >= ni) continue;
    C<T> acc[JB];
    odd_block(tile + i, IB, na, hs, j0, acc);
#pragma unroll
    for (int q = 0; q < JB; ++q)
      if (j0 + q < na) dst[size_t(2 * (j0 + q) + 1) * inner + i] = acc[q];
  }
}

// The z interpolation matrix for the xc contraction: H[k][j] = h[(j - k) mod n]
// as complex values with zero imaginary part (the form's precision).
template <typename T>
__global__ void interp_matrix_k(int n, const T* h, C<T>* H) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int k = e / n, j = e % n;
  int t = j - k;
  t += t < 0 ? n : 0;
  H[e] = C<T>{h[t], T(0)};
}

// rho[z_f][r] (+)= sum_i w_i |v_i|^2 in FP64 over the fine grid, v_i from the
// even z planes (Y, the y-refined data [n2][nb][plane]) or the odd ones (O,
// the same layout); two points per thread (plane is even).
template <typename T>
__global__ __launch_bounds__(256) void density_acc_k(int n2, size_t plane, int nb, const C<T>* Y, const C<T>* O,
                                                     const double* w, double* rho, int accumulate) {
  const size_t p = (size_t(blockIdx.x) * blockDim.x + threadIdx.x) * 2;  // fine index
  const size_t total = size_t(2) * n2 * plane;
  if (p >= total) return;
  const size_t zf = p / plane, r = p % plane;   // p and p + 1 share zf
  const C<T>* src = (zf & 1) ? O : Y;
  const size_t off = (zf >> 1) * nb * plane + r;
  const size_t per = plane;
  double a0 = accumulate ? rho[p] : 0.0, a1 = accumulate ? rho[p + 1] : 0.0;
  for (int i = 0; i < nb; ++i) {
    const C<T> x = src[size_t(i) * per + off], y = src[size_t(i) * per + off + 1];
    const double wi = w[i];
    a0 += wi * (double(x.x) * double(x.x) + double(x.y) * double(x.y));
    a1 += wi * (double(y.x) * double(y.x) + double(y.y) * double(y.y));
  }
  rho[p] = a0;
  rho[p + 1] = a1;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

template <typename T>
hipError_t run_fine(const int* n, int norb, const void* phi_v, const double* occ, double* rho, void* work,
                    hipStream_t s) {
  const int n0 = n[0], n1 = n[1], n2 = n[2];
  const size_t ng = size_t(n0) * n1 * n2;
  const int hstride = (n0 > n1 ? (n0 > n2 ? n0 : n2) : (n1 > n2 ? n1 : n2));
  char* w = static_cast<char*>(work);
  T* h = reinterpret_cast<T*>(w);
  w += align256(size_t(3) * hstride * sizeof(T));
  C<T>* H = reinterpret_cast<C<T>*>(w);  // n2 x n2
  w += align256(size_t(n2) * n2 * sizeof(C<T>));
  C<T>* P = reinterpret_cast<C<T>*>(w);  // x-refined, 2 N_g per orbital of a chunk
  w += align256(size_t(2) * ng * kFineChunk * sizeof(C<T>));
  C<T>* Y = reinterpret_cast<C<T>*>(w);  // y-refined (the even z planes), 4 N_g per orbital
  w += align256(size_t(4) * ng * kFineChunk * sizeof(C<T>));
  C<T>* O = reinterpret_cast<C<T>*>(w);  // the odd z planes, 4 N_g per orbital
  hipLaunchKernelGGL(interp_table_k<T>, dim3((hstride + 127) / 128, 3), dim3(128), 0, s, n0, n1, n2, hstride, h);
  hipLaunchKernelGGL(interp_matrix_k<T>, dim3((n2 * n2 + 255) / 256), dim3(256), 0, s, n2, h + 2 * hstride, H);
  const C<T>* phi = static_cast<const C<T>*>(phi_v);
  const size_t plane = size_t(4) * n0 * n1;  // one z plane of the y-refined data
  hipError_t e = hipSuccess;
  for (int c0 = 0; c0 < norb && e == hipSuccess; c0 += kFineChunk) {
    const int b = norb - c0 < kFineChunk ? norb - c0 : kFineChunk;
    // x: [b n2 n1][n0] -> P [b n2 n1][2 n0]
    const size_t rows = size_t(b) * n2 * n1;
    hipLaunchKernelGGL(interp_x_k<T>, dim3(unsigned((rows + RB - 1) / RB)), dim3(256),
                       RB * n0 * sizeof(C<T>) + n0 * sizeof(T), s, rows, n0, phi + size_t(c0) * ng, P, h);
    // y: P [b n2][n1][2 n0] -> Y [n2][b][2 n1][2 n0] (plane-major, for one z contraction)
    const size_t inner = size_t(2) * n0;
    hipLaunchKernelGGL(interp_strided_k<T>, dim3(unsigned((inner + IB - 1) / IB), unsigned(b * n2)), dim3(256),
                       n1 * IB * sizeof(C<T>) + n1 * sizeof(T), s, n1, inner, P, Y, h + hstride, n2, b);
    // z, odd planes: O = H^T Y, one contraction over the n2 planes for the whole
    // chunk (each plane row holds the b orbitals' planes side by side; matrix cores)
    e = launch_gemm_xc(sizeof(T) == 4, n2, n2, size_t(b) * plane, Y, H, n2, 1.0, O, false, s);
    if (e != hipSuccess) break;
    const size_t half = (size_t(2) * n2 * plane) / 2;
    hipLaunchKernelGGL(density_acc_k<T>, dim3(unsigned((half + 255) / 256)), dim3(256), 0, s, n2, plane, b, Y, O,
                       occ + c0, rho, c0 > 0 ? 1 : 0);
    e = hipGetLastError();
  }
  return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace

size_t density_fine_work_bytes(bool fp32, const int* n, int /*norb*/) {
  const size_t ng = size_t(n[0]) * n[1] * n[2];
  const size_t el = fp32 ? 8 : 16;
  const int hm = n[0] > n[1] ? (n[0] > n[2] ? n[0] : n[2]) : (n[1] > n[2] ? n[1] : n[2]);
  return align256(size_t(3) * hm * (fp32 ? 4 : 8)) + align256(size_t(n[2]) * n[2] * el) +
         align256(2 * ng * kFineChunk * el) + 2 * align256(4 * ng * kFineChunk * el);
}

hipError_t launch_density_fine(bool fp32, const int* n, int norb, const void* phi, const double* occ,
                               double* rho_fine, void* work, hipStream_t s) {
  if (norb <= 0 || n[0] % 2 || n[1] % 2 || n[2] % 2) return hipErrorInvalidValue;
  return fp32 ? run_fine<float>(n, norb, phi, occ, rho_fine, work, s)
              : run_fine<double>(n, norb, phi, occ, rho_fine, work, s);
}

}  // namespace px
