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

template <typename T> __device__ __forceinline__ cpx<T> ld2(const cpx<T>* p) {
  typename V2t<T>::t v = *reinterpret_cast<const typename V2t<T>::t*>(p);
  return {v.x, v.y};
}
template <typename T> __device__ __forceinline__ cpx<T> ld2nt(const cpx<T>* p) {
  typename V2t<T>::t v = __builtin_nontemporal_load(reinterpret_cast<const typename V2t<T>::t*>(p));
  return {v.x, v.y};
}

// grid (ceil(N_g / 256), jc): thread = one grid point of one output orbital j.
template <typename T>
__global__ __launch_bounds__(256) void pass4_transpose_acc(ChunkArgs a, size_t ng) {
  const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
  const int jj = blockIdx.y;
  if (e >= ng) return;
  const cpx<T>* psi = reinterpret_cast<const cpx<T>*>(a.psi);
  const cpx<T>* t = reinterpret_cast<const cpx<T>*>(a.t);
  T accx = T(0), accy = T(0);
  int ii = 0;
  for (; ii + 4 <= a.ic; ii += 4) {
    cpx<T> ps[4], v[4];
    T w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ps[u] = ld2(psi + size_t(a.i0 + ii + u) * ng + e);
      v[u] = ld2nt(t + size_t((ii + u) * a.jc + jj) * ng + e);
      w[u] = T(a.occ[a.i0 + ii + u] * a.inv_ng);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // psi_i * conj(v)
      const T rx = ps[u].x * v[u].x + ps[u].y * v[u].y;
      const T ry = ps[u].y * v[u].x - ps[u].x * v[u].y;
      accx += w[u] * rx;
      accy += w[u] * ry;
    }
  }
  for (; ii < a.ic; ++ii) {
    const cpx<T> ps = ld2(psi + size_t(a.i0 + ii) * ng + e);
    const cpx<T> v = ld2nt(t + size_t(ii * a.jc + jj) * ng + e);
    const T w = T(a.occ[a.i0 + ii] * a.inv_ng);
    accx += w * (ps.x * v.x + ps.y * v.y);
    accy += w * (ps.y * v.x - ps.x * v.y);
  }
  cpx<T>* o = reinterpret_cast<cpx<T>*>(a.out) + size_t(a.j0 + jj) * ng + e;
  const cpx<T> prev = ld2(o);
  typename V2t<T>::t r;
  r.x = prev.x - accx;
  r.y = prev.y - accy;
  *reinterpret_cast<typename V2t<T>::t*>(o) = r;
}

hipError_t launch_pass4(bool fp32, const ChunkArgs& a, size_t ng, hipStream_t s) {
  dim3 grid(unsigned((ng + 255) / 256), a.jc);
  if (fp32) hipLaunchKernelGGL(pass4_transpose_acc<float>, grid, dim3(256), 0, s, a, ng);
  else hipLaunchKernelGGL(pass4_transpose_acc<double>, grid, dim3(256), 0, s, a, ng);
  return hipGetLastError();
}

}  // namespace px
