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

template <typename T> struct V2t;
template <> struct V2t<double> { typedef double t __attribute__((ext_vector_type(2))); };
template <> struct V2t<float> { typedef float t __attribute__((ext_vector_type(2))); };

// Address-space-1 accesses: global instructions rather than flat ones (the
// pointers come from a struct, so the compiler cannot infer it).
#define PX_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ cpx<T> ld2(const cpx<T>* p) {
  typename V2t<T>::t v = *(const PX_GLOBAL typename V2t<T>::t*)p;
  return {v.x, v.y};
}
template <typename T> __device__ __forceinline__ cpx<T> ld2nt(const cpx<T>* p) {
  typename V2t<T>::t v = __builtin_nontemporal_load((const PX_GLOBAL typename V2t<T>::t*)p);
  return {v.x, v.y};
}

// grid (ceil(N_g / 256), ceil(jc / JB)): a thread owns one grid point and JB
// output orbitals j, so each psi_i value is loaded once for the JB of them.
constexpr int JB = 16;

template <typename T>
__global__ __launch_bounds__(256) void pass4_transpose_acc(ChunkArgs a0, const ChunkArgs* tasks,
                                                           size_t ng) {
  const ChunkArgs a = chunk_args(a0, tasks);
  const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
  const int j0 = blockIdx.y * JB;
  if (!a.store_v || j0 >= a.jc || e >= ng) return;
  const int nj = (a.jc - j0) < JB ? (a.jc - j0) : JB;
  const cpx<T>* psi = reinterpret_cast<const cpx<T>*>(a.psi);
  const cpx<T>* t = reinterpret_cast<const cpx<T>*>(a.t);
  T ax[JB], ay[JB];
#pragma unroll
  for (int u = 0; u < JB; ++u) ax[u] = ay[u] = T(0);
  for (int ii = 0; ii < a.ic; ++ii) {
    const cpx<T> ps = ld2(psi + size_t(a.i0 + ii) * ng + e);
    const T w = T(*(const PX_GLOBAL double*)(a.occ + a.i0 + ii) * a.inv_ng);
    const T px_ = w * ps.x, py_ = w * ps.y;
    const cpx<T>* row = t + size_t(ii * a.jc + j0) * ng + e;
    cpx<T> v[JB];
#pragma unroll
    for (int u = 0; u < JB; ++u) v[u] = u < nj ? ld2nt(row + size_t(u) * ng) : cpx<T>{T(0), T(0)};
#pragma unroll
    for (int u = 0; u < JB; ++u) {
      // f_i/N_g psi_i * conj(v)
      ax[u] += px_ * v[u].x + py_ * v[u].y;
      ay[u] += py_ * v[u].x - px_ * v[u].y;
    }
  }
  // all output loads in flight before the first store
  cpx<T>* const o = reinterpret_cast<cpx<T>*>(a.out) + size_t(a.j0 + j0) * ng + e;
  cpx<T> prev[JB];
#pragma unroll
  for (int u = 0; u < JB; ++u) prev[u] = u < nj ? ld2(o + size_t(u) * ng) : cpx<T>{T(0), T(0)};
#pragma unroll
  for (int u = 0; u < JB; ++u) {
    if (u < nj) {
      typename V2t<T>::t r;
      r.x = prev[u].x - ax[u];
      r.y = prev[u].y - ay[u];
      *(PX_GLOBAL typename V2t<T>::t*)(o + size_t(u) * ng) = r;
    }
  }
}

hipError_t launch_pass4(bool fp32, const ChunkArgs& a, size_t ng, hipStream_t s) {
  dim3 grid(unsigned((ng + 255) / 256), (a.jc + JB - 1) / JB);
  const ChunkArgs* none = nullptr;
  if (fp32) hipLaunchKernelGGL(pass4_transpose_acc<float>, grid, dim3(256), 0, s, a, none, ng);
  else hipLaunchKernelGGL(pass4_transpose_acc<double>, grid, dim3(256), 0, s, a, none, ng);
  return hipGetLastError();
}

hipError_t launch_pass4_tasks(bool fp32, const ChunkArgs* tasks, int ntasks, int max_jc, size_t ng,
                              hipStream_t s) {
  dim3 grid(unsigned((ng + 255) / 256), (max_jc + JB - 1) / JB, ntasks);
  ChunkArgs dummy{};
  if (fp32) hipLaunchKernelGGL(pass4_transpose_acc<float>, grid, dim3(256), 0, s, dummy, tasks, ng);
  else hipLaunchKernelGGL(pass4_transpose_acc<double>, grid, dim3(256), 0, s, dummy, tasks, ng);
  return hipGetLastError();
}

}  // namespace px
