// Pass 4 of the symmetric pair pipeline (orbitals and density orbitals are
// the same block, so v_ji = conj(v_ij) for a real even kernel): for an
// off-diagonal chunk, pass 3 has left the real-space pair potentials
// N_g * v_ij in the pair buffer, and this pass adds the transposed
// contributions
//     (Vx psi_j)(r) -= sum_i f_i / N_g * psi_i(r) * conj(N_g v_ij(r))
// for every j of the chunk, summing over the chunk's i in a fixed order (no
// atomics).  Pure streaming: no transform, one read of each pair slab.
#include "fft_core.hpp"
#include "px_internal.hpp"

namespace px {

// EV consecutive complex values of one thread as one 16-byte vector: two
// complex64 (FP32 form) or one complex128.  Address-space-1 accesses: global
// instructions rather than flat ones (the pointers come from a struct, so the
// compiler cannot infer it).
#define PX_GLOBAL __attribute__((address_space(1)))
template <typename T> struct Lane;
template <> struct Lane<float> {
  static constexpr int EV = 2;
  typedef float v __attribute__((ext_vector_type(4)));
};
template <> struct Lane<double> {
  static constexpr int EV = 1;
  typedef double v __attribute__((ext_vector_type(2)));
};
template <typename T> __device__ __forceinline__ typename Lane<T>::v ldv(const T* p) {
  return *(const PX_GLOBAL typename Lane<T>::v*)p;
}
template <typename T> __device__ __forceinline__ typename Lane<T>::v ldvnt(const T* p) {
  return __builtin_nontemporal_load((const PX_GLOBAL typename Lane<T>::v*)p);
}

// grid (ceil(N_g / (256 EV)), ceil(jc / JB)): a thread owns EV consecutive
// grid points (16-byte accesses: -4 % pass time in the FP32 form at 72^3 over
// one point per thread) and JB output orbitals j, so each psi_i value is
// loaded once for the JB of them.  N_g is even for every supported grid.
constexpr int JB = 16;

template <typename T>
__global__ __launch_bounds__(256) void pass4_transpose_acc(ChunkArgs a0, const ChunkArgs* tasks,
                                                           size_t ng) {
  using V = typename Lane<T>::v;
  constexpr int EV = Lane<T>::EV;
  const ChunkArgs a = chunk_args(a0, tasks);
  const size_t e = (size_t(blockIdx.x) * 256 + threadIdx.x) * EV;
  const int j0 = blockIdx.y * JB;
  if (!a.store_v || j0 >= a.jc || e >= ng) return;
  const int nj = (a.jc - j0) < JB ? (a.jc - j0) : JB;
  // interleaved (re, im) scalars: element e of orbital or slab q is at 2 (q ng + e)
  const T* psi = reinterpret_cast<const T*>(a.psi);
  const T* t = reinterpret_cast<const T*>(a.t);
  V acc[JB];
#pragma unroll
  for (int u = 0; u < JB; ++u) acc[u] = V{};
  // a triangular diagonal block (tri) holds v_ij for jj <= ii; its transposed
  // contributions are the pairs jj < ii, so rows start past the first j
  const int ibeg = a.tri ? j0 + 1 : 0;
  for (int ii = ibeg; ii < a.ic; ++ii) {
    const V ps = ldv(psi + 2 * (size_t(a.i0 + ii) * ng + e));
    const T w = T(*(const PX_GLOBAL double*)(a.occ + a.i0 + ii) * a.inv_ng);
    const T* row = t + 2 * (size_t(ii * a.jc + j0) * ng + e);
    V v[JB];
    // slabs past the chunk's last j re-read its first (never stored); in a
    // triangular block the slots jj >= ii re-read the first too, and add zero
#pragma unroll
    for (int u = 0; u < JB; ++u) {
      const bool live = u < nj && (!a.tri || j0 + u < ii);
      const V x = ldvnt(row + 2 * size_t(live ? u : 0) * ng);
      v[u] = live || !a.tri ? x : V{};
    }
#pragma unroll
    for (int u = 0; u < JB; ++u) {
#pragma unroll
      for (int q = 0; q < EV; ++q) {
        // f_i/N_g psi_i * conj(v)
        const T px_ = w * ps[2 * q], py_ = w * ps[2 * q + 1];
        acc[u][2 * q] += px_ * v[u][2 * q] + py_ * v[u][2 * q + 1];
        acc[u][2 * q + 1] += py_ * v[u][2 * q] - px_ * v[u][2 * q + 1];
      }
    }
  }
  // all output loads in flight before the first store
  T* const o = reinterpret_cast<T*>(a.out) + 2 * (size_t(a.j0 + j0) * ng + e);
  V prev[JB];
#pragma unroll
  for (int u = 0; u < JB; ++u) prev[u] = ldv(o + 2 * size_t(u < nj ? u : 0) * ng);
#pragma unroll
  for (int u = 0; u < JB; ++u)
    if (u < nj) *(PX_GLOBAL V*)(o + 2 * size_t(u) * ng) = prev[u] - acc[u];
}

template <typename T> dim3 pass4_grid(size_t ng, int jc, int ntasks) {
  const size_t per = 256 * size_t(Lane<T>::EV);
  return dim3(unsigned((ng + per - 1) / per), (jc + JB - 1) / JB, ntasks);
}

hipError_t launch_pass4(bool fp32, const ChunkArgs& a, size_t ng, hipStream_t s) {
  const ChunkArgs* none = nullptr;
  if (ng % 2) return hipErrorInvalidValue;
  if (fp32) hipLaunchKernelGGL(pass4_transpose_acc<float>, pass4_grid<float>(ng, a.jc, 1), dim3(256), 0, s, a, none, ng);
  else hipLaunchKernelGGL(pass4_transpose_acc<double>, pass4_grid<double>(ng, a.jc, 1), dim3(256), 0, s, a, none, ng);
  return hipGetLastError();
}

hipError_t launch_pass4_tasks(bool fp32, const ChunkArgs* tasks, int ntasks, int max_jc, size_t ng,
                              hipStream_t s) {
  ChunkArgs dummy{};
  if (ng % 2) return hipErrorInvalidValue;
  if (fp32) hipLaunchKernelGGL(pass4_transpose_acc<float>, pass4_grid<float>(ng, max_jc, ntasks), dim3(256), 0, s, dummy, tasks, ng);
  else hipLaunchKernelGGL(pass4_transpose_acc<double>, pass4_grid<double>(ng, max_jc, ntasks), dim3(256), 0, s, dummy, tasks, ng);
  return hipGetLastError();
}

}  // namespace px
