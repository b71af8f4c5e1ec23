// The fused pair pipeline of the exchange operator (Eq. 13 with occupations f_j):
//
//   (Vx phi_i)(r) = -sum_j f_j psi_j(r) * IFFT[ K(G) * FFT(conj(psi_j) * phi_i) ](r)
//
// split into three passes over a chunk of orbital pairs (i, j), each pass a
// kernel that keeps one 2D section of the grid in LDS:
//
//   pass 1  (z-slab, i) : pair product conj(psi_j)*phi_i, forward x and y
//                         transforms, slab written to the pair buffer T.
//   pass 2  (y-plane, pair): forward z transform, multiply by K(G) (and, in
//                         FP32 form, the G = 0 coefficient taken from FP64
//                         slab sums), FP64 partial of sum_G K |rho(G)|^2 for
//                         the exchange energy, inverse z transform; in place.
//   pass 3  (z-slab, i) : inverse x and y transforms, then the weighted sum
//                         over the chunk's j of f_j/N_g * psi_j * v_ij kept in
//                         registers and subtracted from the output slab once.
//
// Layout of every grid array: [n2][n1][n0] with x = n0 fastest; orbital blocks
// are orbital-major.  T is float (complex64 data) or double (complex128).
#pragma once
#include <type_traits>
#include "fft_core.hpp"
#include "px_internal.hpp"

namespace px {

typedef double vd2 __attribute__((ext_vector_type(2)));
typedef float vf2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec;
template <> struct Vec<double> { using t = vd2; };
template <> struct Vec<float> { using t = vf2; };

// Global-memory access through address-space-1 pointers.  The chunk
// arguments arrive in a struct (or a task table), so the compiler cannot
// prove that their pointers are global and would otherwise emit flat
// instructions, which count against the LDS wait counter as well: every
// wait for an LDS access would then also wait for the prefetched slabs.
#define PX_GLOBAL __attribute__((address_space(1)))
template <typename V> __device__ __forceinline__ V gld(const V* p) {
  return *(const PX_GLOBAL V*)p;
}
template <typename V> __device__ __forceinline__ void gst(V* p, V v) {
  *(PX_GLOBAL V*)p = v;
}

template <typename T> __device__ __forceinline__ cpx<T> ldg(const cpx<T>* p) {  // streaming load
  using V = typename Vec<T>::t;
  V v = __builtin_nontemporal_load((const PX_GLOBAL V*)p);
  return {v.x, v.y};
}
template <typename T> __device__ __forceinline__ cpx<T> ldc(const cpx<T>* p) {  // cached load
  using V = typename Vec<T>::t;
  V v = gld(reinterpret_cast<const V*>(p));
  return {v.x, v.y};
}
template <typename T> __device__ __forceinline__ void stg(cpx<T>* p, cpx<T> a) {
  using V = typename Vec<T>::t;
  V v;
  v.x = a.x;
  v.y = a.y;
  gst(reinterpret_cast<V*>(p), v);
}
// Streaming store for the pair buffer: the slab is read back only by the
// next pass, so it should not displace the orbital slabs that the current
// pass re-reads from the caches.
template <typename T> __device__ __forceinline__ void stn(cpx<T>* p, cpx<T> a) {
  using V = typename Vec<T>::t;
  V v;
  v.x = a.x;
  v.y = a.y;
  __builtin_nontemporal_store(v, (PX_GLOBAL V*)p);
}

// Pair-slab loads of pass 2: each element is read once, so they take the
// streaming (non-temporal) policy (pass 2 -4.5 % at 96^3 and -5 % at 72^3 in
// the FP32 form against cached loads; a build may set PX_P2_NT=0 to time
// those).
#ifndef PX_P2_NT
#define PX_P2_NT 1
#endif
template <typename T> __device__ __forceinline__ cpx<T> ld_pair2(const cpx<T>* p) {
  if constexpr (PX_P2_NT != 0) return ldg(p);
  else return ldc(p);
}

// Twiddle table: tw[m] = exp(-2 pi i m / N) from the compile-time roots
// (FP64, about one ulp) rounded to T; copied into LDS by each workgroup.
template <typename T, int N, int NT> __device__ __forceinline__ void fill_twiddles(cpx<T>* tw) {
  constexpr const RootTable<N>& tab = kRoots<N>;
  for (int m = threadIdx.x; m < N; m += NT) tw[m] = {T(tab.c[m]), T(-tab.s[m])};
}

// One DPP step on an FP64 value (both 32-bit halves moved with the same
// control).  With ROW_MASK = 0xF every lane is written; otherwise lanes of the
// rows outside the mask receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  int lo, hi;
  if constexpr (ROW_MASK == 0xF) {
    lo = __builtin_amdgcn_mov_dpp(int(unsigned(u)), CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(int(unsigned(u >> 32)), CTRL, 0xF, 0xF, false);
  } else {
    lo = __builtin_amdgcn_update_dpp(0, int(unsigned(u)), CTRL, ROW_MASK, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, int(unsigned(u >> 32)), CTRL, ROW_MASK, 0xF, false);
  }
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(unsigned(hi)) << 32) | unsigned(lo));
}

// FP64 sum over the 64 lanes of a wave, returned wave-uniform.  Data-parallel
// moves only: pair and quad swaps, half-row and row mirrors (every lane of a
// 16-lane row then holds the row sum), then the GFX9 row broadcasts of lanes
// 15 and 31, after which lane 63 holds the total.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_f64<0x140, 0xF>(v);  // row_mirror
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane(int(unsigned(u)), 63);
  const unsigned hi = __builtin_amdgcn_readlane(int(unsigned(u >> 32)), 63);
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

// Waves per SIMD that a CU could hold given the LDS of one workgroup (and at
// most `cap`): used as the kernel's occupancy target, so that the register
// allocation does not become the tighter limit.  Pass 2 in the FP32 form at
// 40^3 and 64^3 gains from it (-22 %, -7 %; cap 6 keeps it free of spills);
// elsewhere it did not help (32^3 got slower) and the cap is 1 (no target).
template <typename T, int N> constexpr int pass2_wave_cap() {
#if defined(PX_SH_CAP2)
  if (N == 90 || N == 120) return PX_SH_CAP2;
#endif
  // 90 and 120 occur as z lengths of the non-cubic grids only: FP32 pass 2 at
  // 60 x 90 x 120 with two 768-thread workgroups per CU instead of one,
  // 3.42 -> 2.88 ms per 1,024-pair launch
  return sizeof(T) == 4 && (N == 40 || N == 64 || N == 90 || N == 120) ? 6 : 1;
}
constexpr int lds_waves_per_simd(int lds_bytes, int nt, int cap) {
  const int waves = (nt + 63) / 64;
  int wgs = (160 * 1024) / lds_bytes;
  if (wgs * waves > 32) wgs = 32 / waves;
  const int w = (wgs * waves + 3) / 4;
  return w < 1 ? 1 : (w > cap ? cap : w);
}

// Whether two slab buffers (ping-pong) fit in LDS next to the small tables.
template <typename T, int N0, int N1> constexpr bool pingpong_fits() {
  return 2 * N1 * (N0 + 1) * int(sizeof(cpx<T>)) <= 150 * 1024;
}

// Workgroups of nt threads and lds bytes that a CU can hold (LDS and waves).
constexpr int wgs_per_cu(int lds_bytes, int nt) {
  const int cap = 32 / ((nt + 63) / 64);
  const int w = (160 * 1024) / lds_bytes;
  return w < cap ? w : cap;
}
// Whether a workgroup's LDS can grow from `base` to `with` bytes without
// lowering the number of workgroups that a CU can hold.  Used for the
// per-thread partial sums that a few waves add up after a barrier (one wave
// per sum instead of a wave reduction in every wave).
constexpr bool lds_growth_free(int base, int with, int nt) {
  return with <= 160 * 1024 && wgs_per_cu(with, nt) >= wgs_per_cu(base, nt);
}
template <typename T, int N0, int N1, int NT> constexpr bool g0_lds_fits() {
  constexpr int nw = (NT + 63) / 64;
  constexpr int sl = N1 * (N0 + 1) * int(sizeof(cpx<T>));
  constexpr int base = (pingpong_fits<T, N0, N1>() ? 2 : 1) * sl + (N0 + N1) * int(sizeof(cpx<T>)) + 3 * nw * 8;
  return lds_growth_free(base, base - 3 * nw * 8 + 3 * NT * int(sizeof(T)), NT);
}
template <typename T, int N0, int N2, int NT, bool G0> constexpr bool ex_lds_fits() {
  constexpr int nw = (NT + 63) / 64;
  constexpr int base = (N2 * (N0 + 1) + N2) * int(sizeof(cpx<T>)) + 2 * nw * 8;
  return lds_growth_free(base, base - 2 * nw * 8 + (G0 ? 2 : 1) * NT * 8, NT);
}

// Branch-free gather of the R inputs of every butterfly slot of a stage whose
// reads are x[j + r*N/R] along the lines of geometry G: slot indices past the
// last butterfly are clamped to it (loaded, never stored), so all loads of a
// slab issue back to back and stay in flight across the LDS stages that follow.
template <typename T, class G, int R, int NT, int BPT, class F>
__device__ __forceinline__ void gather(cpx<T> (&v)[BPT][R], F&& load) {
  constexpr int NB = G::nl * (G::n / R);
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    int b = threadIdx.x + k * NT;
    if (NB % NT != 0) b = b < NB ? b : NB - 1;
    int line, j;
    decode<G, R>(b, line, j);
#pragma unroll
    for (int r = 0; r < R; ++r) v[k][r] = load(line, j + r * (G::n / R));
  }
}

// The same for kernels without prefetch: a wave whose slots all lie past the
// last butterfly issues no loads at all (the address unit is the bottleneck
// of such kernels; their slots are never used).
template <typename T, class G, int R, int NT, int BPT, class F>
__device__ __forceinline__ void gather_live(cpx<T> (&v)[BPT][R], F&& load) {
  constexpr int NB = G::nl * (G::n / R);
  const int wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63);
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    if (NB % NT != 0 && wave0 + k * NT >= NB) continue;
    int b = threadIdx.x + k * NT;
    if (NB % NT != 0) b = b < NB ? b : NB - 1;
    int line, j;
    decode<G, R>(b, line, j);
#pragma unroll
    for (int r = 0; r < R; ++r) v[k][r] = load(line, j + r * (G::n / R));
  }
}

// ============================================================== pass 1
// PF: prefetch the next density orbital's slab while the current one is
// transformed.  With two slab buffers in LDS (ping-pong, PP) every stage is
// out of place and the buffers swap roles each pair, so a slab costs three
// barriers; otherwise the middle stages run in place (two barriers each).
template <typename T, int N0, int N1, int NT, bool G0, bool PF, bool PP>
__global__ __launch_bounds__(NT) void pass1_fwd_xy(ChunkArgs a0, const ChunkArgs* tasks) {
  static_assert(!PP || pingpong_fits<T, N0, N1>(), "two slabs do not fit in LDS");
  const ChunkArgs a = chunk_args(a0, tasks);
  if (int(blockIdx.y) >= a.ic) return;
  constexpr int P0 = N0 + 1;  // odd row pitch: no bank conflicts on stride-R writes
  constexpr int SL = N1 * P0;
  __shared__ cpx<T> lds[PP ? 2 * SL : SL];
  __shared__ cpx<T> tw0[N0];
  __shared__ cpx<T> tw1[N1];
  using GX = Lines<N0, N1, P0, 1, false>;  // rows: contiguous lines
  using GY = Lines<N1, N0, 1, P0, true>;   // columns: strided lines
  constexpr int NSX = Plan<N0>::nst, NSY = Plan<N1>::nst;
  static_assert(!PP || (NSX == 2 && NSY == 2), "ping-pong path assumes two-stage plans");
  // x stages in the reversed radix order: the first stage writes LDS at a
  // stride of its radix along a line, and the plans' later radices are the
  // ones that spread such writes over the banks (9 before 8 at 72^3)
  using X0 = StageOf<N0, 0, true>;
  using X1 = StageOf<N0, 1, true>;
  using Y0 = StageOf<N1, 0, false>;
  using YL = StageOf<N1, NSY - 1, false>;
  constexpr int NB0 = N1 * (N0 / X0::R), BPT0 = (NB0 + NT - 1) / NT;
  constexpr int NBL = N0 * (N1 / YL::R), BPTL = (NBL + NT - 1) / NT;
  // G = 0 sums: with GL every thread leaves its FP32 partials in LDS and a
  // few waves add them in FP64 after the barrier that follows the first
  // stage (one wave per sum instead of a wave reduction in every wave: -6 %
  // pass time at 72^3); otherwise each wave reduces its own partials
  constexpr int NW = NT / 64;
  constexpr bool GL = G0 && BPT0 == 1 && NT % 64 == 0 && g0_lds_fits<T, N0, N1, NT>();
  __shared__ T gpart[GL ? 3 * NT : 1];
  __shared__ double red[GL || !G0 ? 1 : 3][NW];

  fill_twiddles<T, N0, NT>(tw0);
  fill_twiddles<T, N1, NT>(tw1);
  const int z = blockIdx.x, ii = blockIdx.y;
  const int jend = a.tri ? ii + 1 : a.jc;  // pairs jj < jend of row ii
  const size_t slab = size_t(N0) * N1;
  const size_t ng = slab * a.n2;
  const cpx<T>* phi = reinterpret_cast<const cpx<T>*>(a.phi) + size_t(a.i0 + ii) * ng + z * slab;
  const cpx<T>* psi0 = reinterpret_cast<const cpx<T>*>(a.psi) + size_t(a.j0) * ng + z * slab;
  const int tid = threadIdx.x;

  cpx<T> ph[BPT0][X0::R], nx[BPT0][X0::R];
  if constexpr (PF) {
    gather<T, GX, X0::R, NT>(ph, [&](int line, int e) { return ldc(phi + unsigned(line * N0 + e)); });
    gather<T, GX, X0::R, NT>(nx, [&](int line, int e) { return ldc(psi0 + unsigned(line * N0 + e)); });
  }
  __syncthreads();

  for (int jj = 0; jj < jend; ++jj) {
    cpx<T>* A = lds + (PP ? (jj & 1) * SL : 0);
    cpx<T>* B = lds + (PP ? (1 - (jj & 1)) * SL : 0);
    cpx<T> cu[BPT0][X0::R];
    if constexpr (PF) {
#pragma unroll
      for (int k = 0; k < BPT0; ++k)
#pragma unroll
        for (int r = 0; r < X0::R; ++r) cu[k][r] = nx[k][r];
      if (jj + 1 < jend) {
        const cpx<T>* pn = psi0 + size_t(jj + 1) * ng;
        gather<T, GX, X0::R, NT>(nx, [&](int line, int e) { return ldc(pn + unsigned(line * N0 + e)); });
      }
    } else {
      const cpx<T>* pc = psi0 + size_t(jj) * ng;
      gather<T, GX, X0::R, NT>(cu, [&](int line, int e) { return ldc(pc + unsigned(line * N0 + e)); });
      gather<T, GX, X0::R, NT>(ph, [&](int line, int e) { return ldc(phi + unsigned(line * N0 + e)); });
    }
    const int p = ii * a.jc + jj;
    double sre = 0.0, sim = 0.0, sen = 0.0;
    T gre = T(0), gim = T(0), gen = T(0);
    // first x stage from registers: product, radix butterfly, LDS
#pragma unroll
    for (int k = 0; k < BPT0; ++k) {
      const int b = tid + k * NT;
      const bool valid = NB0 % NT == 0 || b < NB0;
      int line, j;
      decode<GX, X0::R>(valid ? b : 0, line, j);
      cpx<T> v[X0::R];
      // G = 0 slab sums (FP32 form): the thread's few products are summed in
      // FP32, the partials in FP64.  These are the transform's own inputs;
      // with random rounding the partial sums add about 1e-10 relative to the
      // coefficient of a diagonal pair, far below the FP32 transform's error.
      T fen = T(0);
#pragma unroll
      for (int r = 0; r < X0::R; ++r) {
        v[r] = cmulc(cu[k][r], ph[k][r]);
        if (G0) fen += v[r].x * v[r].x + v[r].y * v[r].y;
      }
      dft<T, X0::R, false>(v);
      // the butterfly's DC output is the FP32 sum of its R inputs
      const T fre = v[0].x, fim = v[0].y;
      if (G0 && valid) {
        if constexpr (GL) {
          gre = fre;
          gim = fim;
          gen = fen;
        } else {
          sre += double(fre);
          sim += double(fim);
          sen += double(fen);
        }
      }
      if (valid) {
#pragma unroll
        for (int r = 0; r < X0::R; ++r) A[line * P0 + out_pos<X0::R, 1>(j, r)] = v[r];
      }
    }
    if constexpr (GL) {
      gpart[tid] = gre;
      gpart[NT + tid] = gim;
      gpart[2 * NT + tid] = gen;
    } else if constexpr (G0) {
      sre = wave_sum(sre);
      sim = wave_sum(sim);
      sen = wave_sum(sen);
      if ((tid & 63) == 0) {
        red[0][tid >> 6] = sre;
        red[1][tid >> 6] = sim;
        red[2][tid >> 6] = sen;
      }
    }
    __syncthreads();
    if constexpr (GL) {
      // sum c (re, im, energy) is added by wave c mod NW; the partials are
      // read before this wave reaches the next barrier, so the next pair
      // cannot overwrite them earlier
      const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
      double* g = reinterpret_cast<double*>(a.g0 + size_t(p) * a.n2 + z);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (w == c % NW) {
          double sc = 0.0;
#pragma unroll
          for (int q = 0; q < NW; ++q) sc += double(gpart[c * NT + q * 64 + (tid & 63)]);
          sc = wave_sum(sc);
          if ((tid & 63) == 0) gst(g + c, sc);
        }
      }
    } else if constexpr (G0) {
      if (tid == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          s0 += red[0][w];
          s1 += red[1][w];
          s2 += red[2][w];
        }
        double* g = reinterpret_cast<double*>(a.g0 + size_t(p) * a.n2 + z);
        gst(g, s0);
        gst(g + 1, s1);
        gst(g + 2, s2);
      }
    }
    if constexpr (PP) {
      stage_pp<T, GX, X1::R, X1::NS, false, NT>(A, B, tw0);
      __syncthreads();
      stage_pp<T, GY, Y0::R, Y0::NS, false, NT>(B, A, tw1);
      __syncthreads();
    } else {
      stages_lds<T, GX, false, NT, 1, NSX, true>(A, tw0);
      stages_lds<T, GY, false, NT, 0, NSY - 1>(A, tw1);
    }
    // last y stage: LDS -> global pair buffer
    cpx<T>* out = reinterpret_cast<cpx<T>*>(a.t) + size_t(p) * ng + z * slab;
#pragma unroll
    for (int k = 0; k < BPTL; ++k) {
      const int b = tid + k * NT;
      if (NBL % NT == 0 || b < NBL) {
        int line, j;
        decode<GY, YL::R>(b, line, j);
        cpx<T> v[YL::R];
#pragma unroll
        for (int r = 0; r < YL::R; ++r) v[r] = A[line + (j + r * (N1 / YL::R)) * P0];
        twiddle<T, N1, YL::R, YL::NS, false>(v, j, tw1);
        dft<T, YL::R, false>(v);
#pragma unroll
        for (int r = 0; r < YL::R; ++r) stn(out + unsigned(line + (j + r * (N1 / YL::R)) * N0), v[r]);
      }
    }
    if constexpr (!PP) __syncthreads();
  }
}

// ============================================================== pass 2
// Plane tile (y, pair group) of a pass-2 workgroup in a grid of n1 x groups
// (with XS x-sections per plane, "y" here is y * XS + section).  Workgroups
// go to the 8 XCDs in turn by linear id; for n1 a multiple of 8, XCD x takes
// the contiguous tiles [x n1/8, (x+1) n1/8), so that the cache lines that
// neighbouring tiles share at the ends of their rows are fetched through one
// L2 instead of two.  The set of tiles in flight is unchanged.  Otherwise,
// when n1 x groups is a multiple of 8, XCD x takes the contiguous eighth
// [x T, (x+1) T) of the tiles in pair-major order (T = n1 x groups / 8): every
// pair's planes then go through one L2, and the XCDs work on different pairs.
// (The plane-major form stays where both apply: pair-major was no faster at
// 72^3 and 96^3 and 6 % slower in pass 2 at 64^3.)
#ifndef PX_PLANE_MAP
#define PX_PLANE_MAP 1
#endif
__device__ __forceinline__ void plane_tile(int& y, int& g) {
  const int ny = int(gridDim.x);
  const int b = int(blockIdx.x) + ny * int(blockIdx.y);
  if (ny % 8 == 0) {
    const int k = b >> 3, per = ny >> 3;
    y = (b & 7) * per + k % per;
    g = k / per;
  } else if (PX_PLANE_MAP && (ny * int(gridDim.y)) % 8 == 0) {
    const int t = (ny * int(gridDim.y)) >> 3;
    const int idx = (b & 7) * t + (b >> 3);
    y = idx % ny;
    g = idx / ny;
  } else {
    y = blockIdx.x;
    g = blockIdx.y;
  }
}

// One workgroup takes the same tile of a y-plane of PQ consecutive pairs:
// the kernel values of the tile are loaded once and, with PF, the next pair's
// tile is in flight while the current one is transformed.  A tile is x-section
// xs of XS: the NX = N0/XS z-lines x in [xs NX, (xs+1) NX) of the plane (XS > 1
// gives more, smaller workgroups per CU).  Energy partials go to slot
// y * XS + xs of the pair (N1 * XS slots per pair).
template <typename T, int N0, int N1, int N2, int NT, bool G0, bool EX, int PQ, bool PF, int XS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    lds_waves_per_simd(N2 * (N0 / XS + 1) * int(sizeof(cpx<T>)) + 1024, NT, pass2_wave_cap<T, N2>()))))
void pass2_z_kernel(ChunkArgs a0, const ChunkArgs* tasks) {
  static_assert(N0 % XS == 0, "x-sections must divide the plane");
  constexpr int NX = N0 / XS;
  const ChunkArgs a = chunk_args(a0, tasks);
  // pairs q in [qbeg, qend) of the chunk; pair q owns slot pair_slot(a, q)
  const int np = chunk_pairs(a);
  int yt, grp;
  plane_tile(yt, grp);
  const int y = yt / XS, xs = yt % XS, x0 = xs * NX;
  const int qbeg = grp * PQ;
  if (qbeg >= np) return;
  const int qend = qbeg + PQ < np ? qbeg + PQ : np;
  constexpr int P0 = NX + 1;
  // energy partials: as the G = 0 sums of pass 1 (EL: per thread in LDS, one
  // wave per sum), else a wave reduction in every wave
  constexpr int NW = NT / 64, NE = G0 ? 2 : 1;
  constexpr bool EL = EX && NT % 64 == 0 && ex_lds_fits<T, NX, N2, NT, G0>();
  __shared__ cpx<T> lds[N2 * P0];
  __shared__ cpx<T> tw2[N2];
  __shared__ double red[EL ? 1 : 2][NW];
  __shared__ double epart[EL ? NE * NT : 1];
  using GZ = Lines<N2, NX, 1, P0, true>;  // tile [z][x], lines along z
  constexpr int NS = Plan<N2>::nst;
  using F0 = StageOf<N2, 0, false>;
  using FL = StageOf<N2, NS - 1, false>;
  using I0 = StageOf<N2, 0, true>;
  using IL = StageOf<N2, NS - 1, true>;
  static_assert(I0::R == FL::R, "inverse must start with the forward's last radix");
  constexpr int NB0 = NX * (N2 / F0::R), BPT0 = (NB0 + NT - 1) / NT;
  constexpr int NBL = NX * (N2 / FL::R), BPTL = (NBL + NT - 1) / NT;
  constexpr int NBI = NX * (N2 / IL::R), BPTI = (NBI + NT - 1) / NT;

  const size_t slab = size_t(N0) * N1;
  cpx<T>* const buf0 = reinterpret_cast<cpx<T>*>(a.t) + size_t(y) * N0 + x0;
  // kernel values: the FP32 copy in the FP32 form (G = 0 comes from kern)
  using KT = typename std::conditional<G0, float, double>::type;
  const KT* kern = (G0 ? reinterpret_cast<const KT*>(a.kern32) : reinterpret_cast<const KT*>(a.kern)) +
                   size_t(y) * N0 + x0;
  const int tid = threadIdx.x;

  // global loads first: the first plane (at stage-0 positions) and the kernel
  // values at the positions the last forward stage produces
  cpx<T> nx[BPT0][F0::R];
  gather_live<T, GZ, F0::R, NT>(nx, [&](int line, int e) {
    return ld_pair2(buf0 + size_t(pair_slot(a, qbeg)) * slab * N2 + unsigned(e * int(slab) + line));
  });
  KT kv[BPTL][FL::R];
  const int wave0 = __builtin_amdgcn_readfirstlane(tid & ~63);
#pragma unroll
  for (int k = 0; k < BPTL; ++k) {
    if (NBL % NT != 0 && wave0 + k * NT >= NBL) continue;  // no live slot in this wave
    int b = tid + k * NT;
    if (NBL % NT != 0) b = b < NBL ? b : NBL - 1;
    int line, j;
    decode<GZ, FL::R>(b, line, j);
#pragma unroll
    for (int r = 0; r < FL::R; ++r) kv[k][r] = gld(kern + unsigned((j + r * (N2 / FL::R)) * int(slab) + line));
  }
  fill_twiddles<T, N2, NT>(tw2);
  for (int q = qbeg; q < qend; ++q) {
  const int p = pair_slot(a, q);
  cpx<T>* const buf = buf0 + size_t(p) * slab * N2;
  cpx<T> v0[BPT0][F0::R];
  if (PQ == 1 || PF || q == qbeg) {
#pragma unroll
    for (int k = 0; k < BPT0; ++k)
#pragma unroll
      for (int r = 0; r < F0::R; ++r) v0[k][r] = nx[k][r];
  } else {
    gather_live<T, GZ, F0::R, NT>(v0, [&](int line, int e) { return ld_pair2(buf + unsigned(e * int(slab) + line)); });
  }
  if (PF && q + 1 < qend) {
    cpx<T>* const bn = buf0 + size_t(pair_slot(a, q + 1)) * slab * N2;
    gather<T, GZ, F0::R, NT>(nx, [&](int line, int e) { return ld_pair2(bn + unsigned(e * int(slab) + line)); });
  }
  if (q > qbeg) __syncthreads();  // the previous pair's last stage has read LDS
#pragma unroll
  for (int k = 0; k < BPT0; ++k) {
    const int b = tid + k * NT;
    if (NB0 % NT == 0 || b < NB0) {
      int line, j;
      decode<GZ, F0::R>(b, line, j);
      dft<T, F0::R, false>(v0[k]);
#pragma unroll
      for (int r = 0; r < F0::R; ++r) lds[out_pos<F0::R, 1>(j, r) * P0 + line] = v0[k][r];
    }
  }
  __syncthreads();
  stages_lds<T, GZ, false, NT, 1, NS - 1>(lds, tw2);
  // last forward stage into registers, kernel multiply, first inverse stage
  cpx<T> v[BPTL][FL::R];
  double ex = 0.0, en = 0.0, ex0 = 0.0;  // FP32 form: sum_{G!=0} K|rho|^2, sum_{G!=0} |rho|^2, G = 0 term
#pragma unroll
  for (int k = 0; k < BPTL; ++k) {
    const int b = tid + k * NT;
    if (NBL % NT == 0 || b < NBL) {
      int line, j;
      decode<GZ, FL::R>(b, line, j);
#pragma unroll
      for (int r = 0; r < FL::R; ++r) v[k][r] = lds[(j + r * (N2 / FL::R)) * P0 + line];
      twiddle<T, N2, FL::R, FL::NS, false>(v[k], j, tw2);
      dft<T, FL::R, false>(v[k]);
      T fex = T(0), fen = T(0);  // FP32 form: the thread's partial energy sums
#pragma unroll
      for (int r = 0; r < FL::R; ++r) {
        const int kz = j + r * (N2 / FL::R);
        const double kg = kv[k][r];
        cpx<T> c = v[k][r];
        if (G0 && y == 0 && x0 + line == 0 && kz == 0) {
          const double k0 = gld(a.kern);
          // G = 0 from the FP64 slab sums of pass 1
          double s0 = 0.0, s1 = 0.0;
          const G0Part* g = a.g0 + size_t(p) * N2;
          for (int zz = 0; zz < N2; ++zz) {
            s0 += gld(&g[zz].re);
            s1 += gld(&g[zz].im);
          }
          if (EX) ex0 = k0 * (s0 * s0 + s1 * s1);
          v[k][r] = {T(k0 * s0), T(k0 * s1)};
        } else if constexpr (G0) {
          // FP32 form: K(G) rounded to FP32; the energy terms of the
          // thread's few values are summed in FP32, the partials in FP64
          // (random rounding: about 1e-10 relative on a pair's energy)
          const T kf = kv[k][r];
          const T c2 = c.x * c.x + c.y * c.y;
          if (EX) {
            fex += kf * c2;
            fen += c2;
          }
          v[k][r] = {kf * c.x, kf * c.y};
        } else {
          const double c2 = double(c.x) * double(c.x) + double(c.y) * double(c.y);
          if (EX) ex += kg * c2;
          v[k][r] = {T(kg * double(c.x)), T(kg * double(c.y))};
        }
      }
      if constexpr (G0 && EX) {
        ex += double(fex);
        en += double(fen);
      }
    }
  }
  if constexpr (EL) {
    epart[tid] = ex;
    if constexpr (G0) epart[NT + tid] = en;
  } else if constexpr (EX) {
    ex = wave_sum(ex);
    if ((tid & 63) == 0) red[0][tid >> 6] = ex;
    if constexpr (G0) {
      // the G = 0 term lives in thread 0 (slot 0 holds line 0, kz = 0)
      en = wave_sum(en);
      if ((tid & 63) == 0) red[1][tid >> 6] = en;
    }
  }
  __syncthreads();  // every thread is done reading LDS before it is overwritten
#pragma unroll
  for (int k = 0; k < BPTL; ++k) {
    const int b = tid + k * NT;
    if (NBL % NT == 0 || b < NBL) {
      int line, j;
      decode<GZ, I0::R>(b, line, j);
      dft<T, I0::R, true>(v[k]);
#pragma unroll
      for (int r = 0; r < I0::R; ++r) lds[out_pos<I0::R, 1>(j, r) * P0 + line] = v[k][r];
    }
  }
  __syncthreads();
  if constexpr (EL) {
    // sum c is added by wave c mod NW, which reads the partials before it
    // reaches the next barrier; the G = 0 term lives in thread 0
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    double* e = G0 ? a.expart + (size_t(p) * N1 * XS + yt) * 3 : a.expart + size_t(p) * N1 * XS + yt;
#pragma unroll
    for (int c = 0; c < NE; ++c) {
      if (w == c % NW) {
        double sc = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) sc += epart[c * NT + q * 64 + (tid & 63)];
        sc = wave_sum(sc);
        if ((tid & 63) == 0) gst(e + c, sc);
      }
    }
    if (G0 && tid == 0) gst(e + 2, ex0);
  } else if constexpr (EX) {
    if (tid == 0) {
      double s2 = 0.0, s3 = 0.0;
      const double s4 = ex0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) {
        s2 += red[0][w];
        if (G0) s3 += red[1][w];
      }
      if constexpr (G0) {
        double* e = a.expart + (size_t(p) * N1 * XS + yt) * 3;
        gst(e, s2);
        gst(e + 1, s3);
        gst(e + 2, s4);
      } else {
        gst(a.expart + size_t(p) * N1 * XS + yt, s2);
      }
    }
  }
  stages_lds<T, GZ, true, NT, 1, NS - 1>(lds, tw2);
  // last inverse stage back to global, in place
#pragma unroll
  for (int k = 0; k < BPTI; ++k) {
    const int b = tid + k * NT;
    if (NBI % NT == 0 || b < NBI) {
      int line, j;
      decode<GZ, IL::R>(b, line, j);
      cpx<T> w[IL::R];
#pragma unroll
      for (int r = 0; r < IL::R; ++r) w[r] = lds[(j + r * (N2 / IL::R)) * P0 + line];
      twiddle<T, N2, IL::R, IL::NS, true>(w, j, tw2);
      dft<T, IL::R, true>(w);
#pragma unroll
      for (int r = 0; r < IL::R; ++r) stn(buf + unsigned((j + r * (N2 / IL::R)) * int(slab) + line), w[r]);
    }
  }
  }  // pairs
}

// Pass 3 with PF: also prefetch the next psi_j slab (a second register set),
// FP32 only.  Measured on the same box: 72^3 -4 %, 32^3 and 40^3 -1 to -2 %;
// 48^3 +11 % and 64^3 +7 % (the larger register set costs occupancy there).
template <typename T, int N> constexpr bool psi_prefetch3_for() {
  return sizeof(T) == 4 && (N == 72 || N <= 40);
}

// ============================================================== pass 3
// PF: prefetch the next pair slab and the next psi_j slab during the transform.
// PP as in pass 1.
// SV: symmetric mode, keep N_g v_ij in the pair slab for pass 4 (a compile-time
// switch, so that the loop has the same stores on every path).
template <typename T, int N0, int N1, int NT, bool PF, bool SV, bool PP>
__global__ __launch_bounds__(NT) void pass3_inv_xy_acc(ChunkArgs a0, const ChunkArgs* tasks) {
  static_assert(!PP || pingpong_fits<T, N0, N1>(), "two slabs do not fit in LDS");
  const ChunkArgs a = chunk_args(a0, tasks);
  if (int(blockIdx.y) >= a.ic) return;
  constexpr int P0 = N0 + 1;
  constexpr int SL = N1 * P0;
  __shared__ cpx<T> lds[PP ? 2 * SL : SL];
  __shared__ cpx<T> tw0[N0];
  __shared__ cpx<T> tw1[N1];
  using GX = Lines<N0, N1, P0, 1, false>;
  using GY = Lines<N1, N0, 1, P0, true>;
  constexpr int NSX = Plan<N0>::nst, NSY = Plan<N1>::nst;
  static_assert(!PP || (NSX == 2 && NSY == 2), "ping-pong path assumes two-stage plans");
  using X0 = StageOf<N0, 0, true>;
  using X1 = StageOf<N0, 1, true>;
  // FP32: y stages in the order whose last radix leaves fewer butterflies
  // per thread, since the last stage's values stay in registers for the
  // accumulation (96: 12 last, one butterfly per thread instead of two; 6 %
  // faster).  Ties, and the FP64 form (slower that way at 96), keep the
  // reversed order.
  constexpr int RF = StageOf<N1, NSY - 1, false>::R, RR = StageOf<N1, NSY - 1, true>::R;
  constexpr bool YREV = sizeof(T) == 8 ||
                        (N0 * (N1 / RR) + NT - 1) / NT <= (N0 * (N1 / RF) + NT - 1) / NT;
  using Y0 = StageOf<N1, 0, YREV>;
  using YL = StageOf<N1, NSY - 1, YREV>;
  constexpr int NB0 = N1 * (N0 / X0::R), BPT0 = (NB0 + NT - 1) / NT;
  constexpr int NBL = N0 * (N1 / YL::R), BPTL = (NBL + NT - 1) / NT;
  constexpr bool PSI = PF && psi_prefetch3_for<T, N0>();

  fill_twiddles<T, N0, NT>(tw0);
  fill_twiddles<T, N1, NT>(tw1);
  const int z = blockIdx.x, ii = blockIdx.y;
  const int jend = a.tri ? ii + 1 : a.jc;  // pairs jj < jend of row ii
  const size_t slab = size_t(N0) * N1;
  const size_t ng = slab * a.n2;
  const int tid = threadIdx.x;
  const cpx<T>* t0 = reinterpret_cast<const cpx<T>*>(a.t) + size_t(ii * a.jc) * ng + z * slab;
  const cpx<T>* psi0 = reinterpret_cast<const cpx<T>*>(a.psi) + size_t(a.j0) * ng + z * slab;
  auto tload = [](const cpx<T>* base) {
    return [base](int line, int e) { return ldg(base + unsigned(line * N0 + e)); };
  };
  auto pload = [](const cpx<T>* base) {
    return [base](int line, int e) { return ldc(base + unsigned(line + e * N0)); };
  };
  cpx<T>* const outz = reinterpret_cast<cpx<T>*>(a.out) + size_t(a.i0 + ii) * ng + z * slab;
  cpx<T> acc[BPTL][YL::R];
#pragma unroll
  for (int k = 0; k < BPTL; ++k)
#pragma unroll
    for (int r = 0; r < YL::R; ++r) acc[k][r] = {T(0), T(0)};
  auto weight = [&](int jj) { return T(gld(a.occ + a.j0 + jj) * a.inv_ng); };

  // One pair: inverse x and y transforms of the pair slab held in tc, then
  // the psi_j-weighted accumulation with the psi_j slab in pc.  With PF the
  // next pair slab is requested at the start (into tn).  With PSI the next
  // psi_j slab is requested too (into pn), after the last stage and before
  // this pair's stores: memory requests complete in order, so the wait for
  // psi_j then never waits for stores.  Otherwise psi_j is requested at the
  // start, before the next pair slab, or without PF in the last stage.
  auto step = [&](int jj, cpx<T>(&tc)[BPT0][X0::R], cpx<T>(&tn)[BPT0][X0::R],
                  cpx<T>(&pc)[BPTL][YL::R], cpx<T>(&pn)[BPTL][YL::R]) {
    cpx<T>* A = lds + (PP ? (jj & 1) * SL : 0);
    cpx<T>* B = lds + (PP ? (1 - (jj & 1)) * SL : 0);
    const T wj = weight(jj);  // requested before the slabs: waiting for it waits for nothing else
    // the last pair re-requests its own slabs: the loop stays branch free
    const int jn = jj + 1 < jend ? jj + 1 : jj;
    if constexpr (PF) {
      if constexpr (!PSI) gather<T, GY, YL::R, NT>(pc, pload(psi0 + size_t(jj) * ng));
      gather<T, GX, X0::R, NT>(tn, tload(t0 + size_t(jn) * ng));
    }
#pragma unroll
    for (int k = 0; k < BPT0; ++k) {
      const int b = tid + k * NT;
      if (NB0 % NT == 0 || b < NB0) {
        int line, j;
        decode<GX, X0::R>(b, line, j);
        dft<T, X0::R, true>(tc[k]);
#pragma unroll
        for (int r = 0; r < X0::R; ++r) A[line * P0 + out_pos<X0::R, 1>(j, r)] = tc[k][r];
      }
    }
    __syncthreads();
    if constexpr (PP) {
      stage_pp<T, GX, X1::R, X1::NS, true, NT>(A, B, tw0);
      __syncthreads();
      stage_pp<T, GY, Y0::R, Y0::NS, true, NT>(B, A, tw1);
      __syncthreads();
    } else {
      stages_lds<T, GX, true, NT, 1, NSX>(A, tw0);
      stages_lds<T, GY, true, NT, 0, NSY - 1, YREV>(A, tw1);
    }
    // last stage: slots past the last butterfly repeat it (same values to the
    // same addresses), so every thread issues the same loads and stores.
    // Symmetric mode (SV) keeps N_g * v_ij (real space) for the transposed pass.
    cpx<T>* tv = reinterpret_cast<cpx<T>*>(a.t) + size_t(ii * a.jc + jj) * ng + z * slab;
    cpx<T> v[BPTL][YL::R];
#pragma unroll
    for (int k = 0; k < BPTL; ++k) {
      int b = tid + k * NT;
      if (NBL % NT != 0) b = b < NBL ? b : NBL - 1;
      int line, j;
      decode<GY, YL::R>(b, line, j);
      if constexpr (!PF) {
        const cpx<T>* pj = psi0 + size_t(jj) * ng;
#pragma unroll
        for (int r = 0; r < YL::R; ++r) pc[k][r] = ldc(pj + unsigned(line + (j + r * (N1 / YL::R)) * N0));
      }
#pragma unroll
      for (int r = 0; r < YL::R; ++r) v[k][r] = A[line + (j + r * (N1 / YL::R)) * P0];
      twiddle<T, N1, YL::R, YL::NS, true>(v[k], j, tw1);
      dft<T, YL::R, true>(v[k]);
#pragma unroll
      for (int r = 0; r < YL::R; ++r) {
        cpx<T> t = cmul(pc[k][r], v[k][r]);
        acc[k][r].x += wj * t.x;
        acc[k][r].y += wj * t.y;
      }
      if constexpr (SV && !PSI) {
#pragma unroll
        for (int r = 0; r < YL::R; ++r) stn(tv + unsigned(line + (j + r * (N1 / YL::R)) * N0), v[k][r]);
      }
    }
    if constexpr (PSI) {
      gather<T, GY, YL::R, NT>(pn, pload(psi0 + size_t(jn) * ng));
      if constexpr (SV) {
#pragma unroll
        for (int k = 0; k < BPTL; ++k) {
          int b = tid + k * NT;
          if (NBL % NT != 0) b = b < NBL ? b : NBL - 1;
          int line, j;
          decode<GY, YL::R>(b, line, j);
#pragma unroll
          for (int r = 0; r < YL::R; ++r) stn(tv + unsigned(line + (j + r * (N1 / YL::R)) * N0), v[k][r]);
        }
      }
    }
    if constexpr (!PP) __syncthreads();
  };

  if constexpr (PF) {
    // two register sets for the pair slab, used alternately: the next slab
    // loads into the idle set while the current one is transformed (no
    // copies between iterations, so the loads stay in flight)
    cpx<T> tA[BPT0][X0::R], tB[BPT0][X0::R];
    cpx<T> pA[BPTL][YL::R], pB[PSI ? BPTL : 1][YL::R];
    gather<T, GX, X0::R, NT>(tA, tload(t0));
    if constexpr (PSI) gather<T, GY, YL::R, NT>(pA, pload(psi0));
    __syncthreads();
    for (int jj = 0; jj < jend; jj += 2) {
      if constexpr (PSI) {
        step(jj, tA, tB, pA, pB);
        if (jj + 1 < jend) step(jj + 1, tB, tA, pB, pA);
      } else {
        step(jj, tA, tB, pA, pA);
        if (jj + 1 < jend) step(jj + 1, tB, tA, pA, pA);
      }
    }
  } else {
    __syncthreads();
    for (int jj = 0; jj < jend; ++jj) {
      cpx<T> tc[BPT0][X0::R];
      cpx<T> pc[BPTL][YL::R];
      gather<T, GX, X0::R, NT>(tc, tload(t0 + size_t(jj) * ng));
      step(jj, tc, tc, pc, pc);
    }
  }
  // one read-modify-write of the output slab, all loads issued before the
  // first store
  cpx<T> po[BPTL][YL::R];
  if (!a.first) gather<T, GY, YL::R, NT>(po, pload(outz));
#pragma unroll
  for (int k = 0; k < BPTL; ++k) {
    const int b = tid + k * NT;
    if (NBL % NT == 0 || b < NBL) {
      int line, j;
      decode<GY, YL::R>(b, line, j);
#pragma unroll
      for (int r = 0; r < YL::R; ++r) {
        const cpx<T> prev = a.first ? cpx<T>{T(0), T(0)} : po[k][r];
        stg(outz + unsigned(line + (j + r * (N1 / YL::R)) * N0), csub(prev, acc[k][r]));
      }
    }
  }
}

// ============================================================== pass 3, staged form
// A workgroup barrier that waits only for this wave's LDS accesses: global ->
// LDS transfers in flight stay in flight across it.  (The fence of
// __syncthreads would wait for every outstanding vector memory operation,
// those transfers included.)  The signal fences keep the compiler from moving
// memory accesses across it.
__device__ __forceinline__ void lds_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0); vmcnt and expcnt not waited for
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// A workgroup barrier after all of this wave's memory operations, global ->
// LDS transfers included (vmcnt(0) lgkmcnt(0)).
__device__ __forceinline__ void dma_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0070);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Copies BYTES contiguous bytes (a multiple of 16) from global memory into LDS
// with 16-byte global -> LDS transfers: wave w moves the 1 KiB pieces w,
// w + NW, ..., lane l bytes [16 l, 16 l + 16) of each (the LDS destination of
// a transfer is wave-uniform, its lanes fill consecutive 16-byte slots).
// Cache-policy bits of the slab transfers (a build may set PX_DMA_AUX to time
// alternatives).
#ifndef PX_DMA_AUX
#define PX_DMA_AUX 2
#endif
template <int BYTES, int NT>
__device__ __forceinline__ void dma_to_lds(const void* src, void* dst) {
  static_assert(BYTES % 16 == 0, "16-byte pieces");
  constexpr int NW = NT / 64, NCH = (BYTES + 1023) / 1024;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = int(threadIdx.x) & 63;
  const char PX_GLOBAL* g = (const char PX_GLOBAL*)(src);
  char __attribute__((address_space(3)))* l = (char __attribute__((address_space(3)))*)(dst);
#pragma unroll
  for (int q0 = 0; q0 < NCH; q0 += NW) {
    const int q = q0 + w;
    const int off = q * 1024 + lane * 16;
    // whole pieces for every wave: no branch (the same transfers on every path)
    if (NCH % NW == 0 && BYTES % 1024 == 0 ? true : (q < NCH && off < BYTES))
      __builtin_amdgcn_global_load_lds((const void PX_GLOBAL*)(g + off),
                                       (void __attribute__((address_space(3)))*)(l + q * 1024), 16, 0,
                                       PX_DMA_AUX);
  }
}

// One in-place LDS stage like stage_lds, with lds_sync barriers.
template <typename T, class G, int R, int NS, bool INV, int NT>
__device__ __forceinline__ void stage_inplace(cpx<T>* lds, const cpx<T>* tw) {
  constexpr int NB = G::nl * (G::n / R);
  constexpr int BPT = (NB + NT - 1) / NT;
  cpx<T> v[BPT][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = tid + k * NT;
    if (NB % NT == 0 || b < NB) {
      int line, j;
      decode<G, R>(b, line, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = lds[line * G::ls + (j + r * (G::n / R)) * G::es];
    }
  }
  lds_sync();
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = tid + k * NT;
    if (NB % NT == 0 || b < NB) {
      int line, j;
      decode<G, R>(b, line, j);
      twiddle<T, G::n, R, NS, INV>(v[k], j, tw);
      dft<T, R, INV>(v[k]);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[line * G::ls + out_pos<R, NS>(j, r) * G::es] = v[k][r];
    }
  }
  lds_sync();
}

// Pass 3 with the pair slab staged through LDS (FP32): one working slab A
// (padded rows, stages in place) and one staging slab S (the pair slab as
// stored).  While pair jj is transformed, the next pair's slab moves into S by
// global -> LDS transfers, so neither the registers of a second slab (which at
// 96^3 would cost the occupancy of the 12-wave workgroup) nor a wait at the
// start of each pair are needed.  The psi_j slab of the pair is requested at
// the start of the pair, before the transfer, so that waiting for it never
// waits for the transfer.  Same arithmetic and results as pass3_inv_xy_acc.
template <typename T, int N0, int N1, int NT, bool SV>
__global__ __launch_bounds__(NT) void pass3_staged(ChunkArgs a0, const ChunkArgs* tasks) {
  const ChunkArgs a = chunk_args(a0, tasks);
  if (int(blockIdx.y) >= a.ic) return;
  constexpr int P0 = N0 + 1;
  constexpr int SL = N1 * P0;
  constexpr int SLAB_BYTES = N0 * N1 * int(sizeof(cpx<T>));
  __shared__ cpx<T> lds[SL];
  __shared__ __attribute__((aligned(16))) cpx<T> sbuf[N0 * N1];
  __shared__ cpx<T> tw0[N0];
  __shared__ cpx<T> tw1[N1];
  using GX = Lines<N0, N1, P0, 1, false>;
  using GY = Lines<N1, N0, 1, P0, true>;
  constexpr int NSX = Plan<N0>::nst, NSY = Plan<N1>::nst;
  static_assert(NSX == 2 && NSY == 2, "staged pass 3 assumes two-stage plans");
  using X0 = StageOf<N0, 0, true>;
  using X1 = StageOf<N0, 1, true>;
  constexpr int RF = StageOf<N1, NSY - 1, false>::R, RR = StageOf<N1, NSY - 1, true>::R;
  constexpr bool YREV = sizeof(T) == 8 ||
                        (N0 * (N1 / RR) + NT - 1) / NT <= (N0 * (N1 / RF) + NT - 1) / NT;
  using Y0 = StageOf<N1, 0, YREV>;
  using YL = StageOf<N1, NSY - 1, YREV>;
  constexpr int NB0 = N1 * (N0 / X0::R), BPT0 = (NB0 + NT - 1) / NT;
  constexpr int NBL = N0 * (N1 / YL::R), BPTL = (NBL + NT - 1) / NT;

  fill_twiddles<T, N0, NT>(tw0);
  fill_twiddles<T, N1, NT>(tw1);
  const int z = blockIdx.x, ii = blockIdx.y;
  const int jend = a.tri ? ii + 1 : a.jc;  // pairs jj < jend of row ii
  const size_t slab = size_t(N0) * N1;
  const size_t ng = slab * a.n2;
  const int tid = threadIdx.x;
  const cpx<T>* t0 = reinterpret_cast<const cpx<T>*>(a.t) + size_t(ii * a.jc) * ng + z * slab;
  const cpx<T>* psi0 = reinterpret_cast<const cpx<T>*>(a.psi) + size_t(a.j0) * ng + z * slab;
  auto pload = [](const cpx<T>* base) {
    return [base](int line, int e) { return ldc(base + unsigned(line + e * N0)); };
  };
  cpx<T>* const outz = reinterpret_cast<cpx<T>*>(a.out) + size_t(a.i0 + ii) * ng + z * slab;
  cpx<T> acc[BPTL][YL::R];
#pragma unroll
  for (int k = 0; k < BPTL; ++k)
#pragma unroll
    for (int r = 0; r < YL::R; ++r) acc[k][r] = {T(0), T(0)};

  dma_to_lds<SLAB_BYTES, NT>(t0, sbuf);
  dma_sync();
  for (int jj = 0; jj < jend; ++jj) {
    // the weight is uniform: a scalar load (counted with the LDS operations,
    // so that waiting for it never waits for the slab transfer)
    const T wj = T(*(const __attribute__((address_space(4))) double*)(a.occ + a.j0 + jj) * a.inv_ng);
    cpx<T> pc[BPTL][YL::R];
    gather<T, GY, YL::R, NT>(pc, pload(psi0 + size_t(jj) * ng));
    // first inverse x stage: staging slab -> registers -> working slab
#pragma unroll
    for (int k = 0; k < BPT0; ++k) {
      const int b = tid + k * NT;
      if (NB0 % NT == 0 || b < NB0) {
        int line, j;
        decode<GX, X0::R>(b, line, j);
        cpx<T> v[X0::R];
#pragma unroll
        for (int r = 0; r < X0::R; ++r) v[r] = sbuf[line * N0 + j + r * (N0 / X0::R)];
        dft<T, X0::R, true>(v);
#pragma unroll
        for (int r = 0; r < X0::R; ++r) lds[line * P0 + out_pos<X0::R, 1>(j, r)] = v[r];
      }
    }
    lds_sync();  // the staging slab has been read by every thread
    // the next pair's slab (the last pair moves its own slab again: the same
    // transfers on every pair, so that the compiler's wait for the psi_j slab
    // counts them and does not wait for them)
    dma_to_lds<SLAB_BYTES, NT>(t0 + size_t(jj + 1 < jend ? jj + 1 : jj) * ng, sbuf);
    stage_inplace<T, GX, X1::R, X1::NS, true, NT>(lds, tw0);
    stage_inplace<T, GY, Y0::R, Y0::NS, true, NT>(lds, tw1);
    // last stage: registers, psi_j-weighted accumulation, kept v_ij (SV)
    cpx<T>* tv = reinterpret_cast<cpx<T>*>(a.t) + size_t(ii * a.jc + jj) * ng + z * slab;
#pragma unroll
    for (int k = 0; k < BPTL; ++k) {
      int b = tid + k * NT;
      if (NBL % NT != 0) b = b < NBL ? b : NBL - 1;
      int line, j;
      decode<GY, YL::R>(b, line, j);
      cpx<T> v[YL::R];
#pragma unroll
      for (int r = 0; r < YL::R; ++r) v[r] = lds[line + (j + r * (N1 / YL::R)) * P0];
      twiddle<T, N1, YL::R, YL::NS, true>(v, j, tw1);
      dft<T, YL::R, true>(v);
#pragma unroll
      for (int r = 0; r < YL::R; ++r) {
        cpx<T> t = cmul(pc[k][r], v[r]);
        acc[k][r].x += wj * t.x;
        acc[k][r].y += wj * t.y;
      }
      if constexpr (SV) {
#pragma unroll
        for (int r = 0; r < YL::R; ++r) stn(tv + unsigned(line + (j + r * (N1 / YL::R)) * N0), v[r]);
      }
    }
    // the next pair's slab has arrived and the working slab is free
    dma_sync();
  }
  // one read-modify-write of the output slab, all loads issued before the
  // first store
  cpx<T> po[BPTL][YL::R];
  if (!a.first) gather<T, GY, YL::R, NT>(po, pload(outz));
#pragma unroll
  for (int k = 0; k < BPTL; ++k) {
    const int b = tid + k * NT;
    if (NBL % NT == 0 || b < NBL) {
      int line, j;
      decode<GY, YL::R>(b, line, j);
#pragma unroll
      for (int r = 0; r < YL::R; ++r) {
        const cpx<T> prev = a.first ? cpx<T>{T(0), T(0)} : po[k][r];
        stg(outz + unsigned(line + (j + r * (N1 / YL::R)) * N0), csub(prev, acc[k][r]));
      }
    }
  }
}

// ============================================================== host launcher
// Threads per workgroup: close to the butterfly count of each stage of a slab
// (N * N / R), so that most stages take one butterfly per thread.
template <int N> constexpr int threads_for() {
  return N == 16 ? 64 : N == 24 ? 192 : N == 32 ? 256 : N == 40 ? 320 : N == 48 ? 384
       : N == 60 ? 640 : N == 64 ? 512 : N == 72 ? 704 : N == 80 ? 832 : 768;
}
// Per-pass configuration of passes 1 and 3: threads per workgroup, the
// ping-pong form (two LDS slabs, one barrier per stage) or one slab updated in
// place, and prefetch across pair iterations where the doubled register set
// fits without spilling (checked with the compiler's resource report).  The
// defaults were chosen by measurement; a build may override them for one grid
// size, PX_P13_N, to time alternatives (PX_P1_NT32, PX_P1_PP32, PX_P1_PF32,
// PX_P3_NT32, PX_P3_PP32, PX_P3_PF32 and the same with 64 for FP64).
#if defined(PX_P13_N)
#define PX_OVR(M32, M64)                                    \
  if (sizeof(T) == 4 && N == PX_P13_N) return M32;          \
  if (sizeof(T) == 8 && N == PX_P13_N) return M64;
#endif
template <typename T, int N> constexpr int pass1_threads() {
#if defined(PX_P13_N) && defined(PX_P1_NT32) && defined(PX_P1_NT64)
  PX_OVR(PX_P1_NT32, PX_P1_NT64)
#endif
  return threads_for<N>();
}
template <typename T, int N> constexpr int pass3_threads() {
#if defined(PX_P13_N) && defined(PX_P3_NT32) && defined(PX_P3_NT64)
  PX_OVR(PX_P3_NT32, PX_P3_NT64)
#endif
  return threads_for<N>();
}
template <typename T, int N> constexpr bool pass1_pingpong() {
#if defined(PX_P13_N) && defined(PX_P1_PP32) && defined(PX_P1_PP64)
  PX_OVR(bool(PX_P1_PP32), bool(PX_P1_PP64))
#endif
  return pingpong_fits<T, N, N>();
}
template <typename T, int N> constexpr bool pass3_pingpong() {
#if defined(PX_P13_N) && defined(PX_P3_PP32) && defined(PX_P3_PP64)
  PX_OVR(bool(PX_P3_PP32), bool(PX_P3_PP64))
#endif
  return pingpong_fits<T, N, N>();
}
template <typename T, int N> constexpr bool prefetch1_for() {
#if defined(PX_P13_N) && defined(PX_P1_PF32) && defined(PX_P1_PF64)
  PX_OVR(bool(PX_P1_PF32), bool(PX_P1_PF64))
#endif
  return sizeof(T) == 4 ? true : (N <= 72 && N != 60);  // FP32 at 96^3: -21 % with it
}
// Pass 3 in the staged form (pass3_staged) instead of pass3_inv_xy_acc: FP32
// at 72^3 to 96^3 (per 1,024-pair launch, same box: 96^3 3.52 -> 3.14 ms,
// where the 12-wave workgroup has no registers for a second slab; 80^3 2.11 ->
// 1.78 ms; 72^3 1.51 -> 1.36 ms).  Pass 4 then runs 4-9 % slower, so at 64^3
// and below, where pass 3 gained nothing, the register form stays.
template <typename T, int N> constexpr bool pass3_staged_for() {
#if defined(PX_P13_N) && defined(PX_P3_STG32)
  if (sizeof(T) == 4 && N == PX_P13_N) return bool(PX_P3_STG32);
#endif
  return sizeof(T) == 4 && (N == 72 || N == 80 || N == 96);
}
template <typename T, int N> constexpr bool prefetch3_for() {
#if defined(PX_P13_N) && defined(PX_P3_PF32) && defined(PX_P3_PF64)
  PX_OVR(bool(PX_P3_PF32), bool(PX_P3_PF64))
#endif
  return sizeof(T) == 4 ? N <= 72 : N <= 48;
}

// Threads of a pass-2 workgroup.  FP32 at 72^3: 512 (two butterflies per
// thread in each stage) lets three workgroups share a CU instead of two.  With
// two x-sections per plane (see pass2_sections): 192 at 96^3 in both forms
// (2-3 butterflies per thread; FP32 four workgroups per CU; measured against
// 128-384 threads and one to four sections on the same box), FP32 256 at
// 64^3 and 320 at 80^3 (half the single-section counts).
template <typename T, int N> constexpr int pass2_threads_default() {
  return N == 96 ? 192
       : sizeof(T) == 4 && N == 72 ? 512
       : sizeof(T) == 4 && N == 64 ? 256
       : sizeof(T) == 4 && N == 80 ? 320
       : threads_for<N>();
}
template <typename T, int N> constexpr int pass2_threads_for() {
#if defined(PX_P2_N) && defined(PX_P2_NT32)
  if (sizeof(T) == 4 && N == PX_P2_N) return PX_P2_NT32;
#endif
#if defined(PX_P2_N) && defined(PX_P2_NT64)
  if (sizeof(T) == 8 && N == PX_P2_N) return PX_P2_NT64;
#endif
  return pass2_threads_default<T, N>();
}

// Threads of pass-2 configuration CFG (see pass2_sections_cfg): the default,
// or for the alternative with two sections half the default (a multiple of
// 64), with one section the single-section counts.
template <typename T, int N, int CFG> constexpr int pass2_threads_cfg() {
  if constexpr (CFG == 0) {
    return pass2_threads_for<T, N>();
  } else if constexpr (pass2_sections_cfg(sizeof(T) == 4, N, 1) == 2) {
    constexpr int t = (pass2_threads_for<T, N>() / 2 + 63) / 64 * 64;
    return t < 64 ? 64 : t;
  } else {
    return sizeof(T) == 4 && N == 72 ? 512 : sizeof(T) == 4 && N == 96 ? 384 : threads_for<N>();
  }
}

// Pairs per pass-2 workgroup, with prefetch of the next plane: FP64 at 72^3,
// where the plane's LDS already limits a CU to one workgroup and the loop
// fits the registers.  Elsewhere two workgroups per CU overlap better than one
// with a loop (FP32 at 72^3), or the loop would spill (FP64 at 80^3, 96^3).
template <typename T, int N> constexpr int pass2_pairs_per_wg() {
  return sizeof(T) == 8 && N == 72 ? 8 : 1;
}

// Pass 1, 2, 3 for the cubic grid N^3: one chunk (tasks == nullptr, the
// chunk in `a`), or ntasks chunks of a task table in device memory, one per
// blockIdx.z (max_ic / max_pairs: the largest chunk of the table).  The FP32
// form always takes the G = 0 coefficient from FP64 slab sums.
// ev (optional, 4 events) brackets the passes: ev[0] | pass 1 | ev[1] | pass 2 | ev[2] | pass 3 | ev[3].
// Pass 2 of one chunk or task table in configuration CFG.
template <int N, int CFG>
void launch_pass2(bool fp32, const ChunkArgs& a, int npairs, bool ex, hipStream_t s,
                  const ChunkArgs* tasks, int ntasks) {
  constexpr int Q32 = pass2_pairs_per_wg<float, N>(), Q64 = pass2_pairs_per_wg<double, N>();
  constexpr int X32 = pass2_sections_cfg(true, N, CFG), X64 = pass2_sections_cfg(false, N, CFG);
  const int pq = fp32 ? Q32 : Q64;
  const dim3 g2(N * (fp32 ? X32 : X64), (npairs + pq - 1) / pq, ntasks);
  if (fp32) {
    constexpr int NT2 = pass2_threads_cfg<float, N, CFG>();
    if (ex) hipLaunchKernelGGL((pass2_z_kernel<float, N, N, N, NT2, true, true, Q32, (Q32 > 1), X32>), g2, dim3(NT2), 0, s, a, tasks);
    else hipLaunchKernelGGL((pass2_z_kernel<float, N, N, N, NT2, true, false, Q32, (Q32 > 1), X32>), g2, dim3(NT2), 0, s, a, tasks);
  } else {
    constexpr int NT2 = pass2_threads_cfg<double, N, CFG>();
    if (ex) hipLaunchKernelGGL((pass2_z_kernel<double, N, N, N, NT2, false, true, Q64, (Q64 > 1), X64>), g2, dim3(NT2), 0, s, a, tasks);
    else hipLaunchKernelGGL((pass2_z_kernel<double, N, N, N, NT2, false, false, Q64, (Q64 > 1), X64>), g2, dim3(NT2), 0, s, a, tasks);
  }
}

template <int N>
hipError_t launch_chunk_n(bool fp32, const ChunkArgs& a, int npairs, bool ex, bool store_v,
                          int p2cfg, hipStream_t s, hipEvent_t* ev, const ChunkArgs* tasks,
                          int ntasks, int max_ic) {
  if (!tasks) {
    ntasks = 1;
    max_ic = a.ic;
  }
  dim3 g1(N, max_ic, ntasks), g3(N, max_ic, ntasks);
  if (ev) (void)hipEventRecord(ev[0], s);
  constexpr int NT1F = pass1_threads<float, N>(), NT1D = pass1_threads<double, N>();
  if (fp32)
    hipLaunchKernelGGL((pass1_fwd_xy<float, N, N, NT1F, true, prefetch1_for<float, N>(), pass1_pingpong<float, N>()>),
                       g1, dim3(NT1F), 0, s, a, tasks);
  else
    hipLaunchKernelGGL((pass1_fwd_xy<double, N, N, NT1D, false, prefetch1_for<double, N>(), pass1_pingpong<double, N>()>),
                       g1, dim3(NT1D), 0, s, a, tasks);
  if (ev) (void)hipEventRecord(ev[1], s);
  if (p2cfg == 0) launch_pass2<N, 0>(fp32, a, npairs, ex, s, tasks, ntasks);
  else launch_pass2<N, 1>(fp32, a, npairs, ex, s, tasks, ntasks);
  if (ev) (void)hipEventRecord(ev[2], s);
  constexpr bool P32 = prefetch3_for<float, N>(), P64 = prefetch3_for<double, N>();
  constexpr bool Q3F = pass3_pingpong<float, N>(), Q3D = pass3_pingpong<double, N>();
  constexpr int NT3F = pass3_threads<float, N>(), NT3D = pass3_threads<double, N>();
  constexpr bool S3F = pass3_staged_for<float, N>();
  if (fp32 && S3F && store_v)
    hipLaunchKernelGGL((pass3_staged<float, N, N, NT3F, true>), g3, dim3(NT3F), 0, s, a, tasks);
  else if (fp32 && S3F)
    hipLaunchKernelGGL((pass3_staged<float, N, N, NT3F, false>), g3, dim3(NT3F), 0, s, a, tasks);
  else if (fp32 && store_v)
    hipLaunchKernelGGL((pass3_inv_xy_acc<float, N, N, NT3F, P32, true, Q3F>), g3, dim3(NT3F), 0, s, a, tasks);
  else if (fp32)
    hipLaunchKernelGGL((pass3_inv_xy_acc<float, N, N, NT3F, P32, false, Q3F>), g3, dim3(NT3F), 0, s, a, tasks);
  else if (store_v)
    hipLaunchKernelGGL((pass3_inv_xy_acc<double, N, N, NT3D, P64, true, Q3D>), g3, dim3(NT3D), 0, s, a, tasks);
  else
    hipLaunchKernelGGL((pass3_inv_xy_acc<double, N, N, NT3D, P64, false, Q3D>), g3, dim3(NT3D), 0, s, a, tasks);
  if (ev) (void)hipEventRecord(ev[3], s);
  return hipGetLastError();
}

// ---------------------------------------------------------------- other grids
// Grids whose three lengths differ (the wavefunction grids of the paper's
// 768- and 1536-atom cells, 60 x 60 x 90 and 60 x 90 x 120): configurations
// derived from the plans plus a few choices measured at 60 x 90 x 120 (FP32,
// per 1,024-pair launch, same box).  Slab kernels (passes 1, 3): threads = the
// largest stage's butterfly count rounded up to whole waves, at most 768 (12
// waves leave 170 registers per thread at one workgroup per CU; 960 threads
// spilled in pass 3, 512 were 25 % slower); ping-pong slabs where two fit; the
// FP32 form prefetches the next density orbital in pass 1 (2.27 -> 1.90 ms) and
// runs pass 3 staged through LDS (3.55 -> 2.23 ms).  Pass 2: see
// shape_sections; one pair per workgroup.  A build may override these for
// timing (PX_SH_* below).
#ifndef PX_SH_NT_CAP
#define PX_SH_NT_CAP 768
#endif
#ifndef PX_SH_PF1
#define PX_SH_PF1 1
#endif
#ifndef PX_SH_STG3
#define PX_SH_STG3 1
#endif
constexpr int wave_threads(int butterflies, int cap) {
  const int t = (butterflies + 63) / 64 * 64;
  return t < cap ? t : cap;
}
template <int N0, int N1> constexpr int slab_threads() {
  int m = 0;
  for (int s = 0; s < Plan<N0>::nst; ++s) m = m > N1 * (N0 / Plan<N0>::rad[s]) ? m : N1 * (N0 / Plan<N0>::rad[s]);
  for (int s = 0; s < Plan<N1>::nst; ++s) m = m > N0 * (N1 / Plan<N1>::rad[s]) ? m : N0 * (N1 / Plan<N1>::rad[s]);
  return wave_threads(m, PX_SH_NT_CAP);
}
template <int NX, int N2> constexpr int plane_threads() {
  int m = 0;
  for (int s = 0; s < Plan<N2>::nst; ++s) m = m > NX * (N2 / Plan<N2>::rad[s]) ? m : NX * (N2 / Plan<N2>::rad[s]);
  return wave_threads(m, 1024);
}

template <int N0, int N1, int N2>
hipError_t launch_chunk_shape(bool fp32, const ChunkArgs& a, int npairs, bool ex, bool store_v,
                              hipStream_t s, hipEvent_t* ev, const ChunkArgs* tasks, int ntasks,
                              int max_ic) {
  if (!tasks) {
    ntasks = 1;
    max_ic = a.ic;
  }
  constexpr int NT1 = slab_threads<N0, N1>();
  constexpr bool PPF = pingpong_fits<float, N0, N1>(), PPD = pingpong_fits<double, N0, N1>();
  constexpr int XF = shape_sections(true, N0, N2), XD = shape_sections(false, N0, N2);
  constexpr int NT2F = plane_threads<N0 / XF, N2>(), NT2D = plane_threads<N0 / XD, N2>();
  const dim3 g1(N2, max_ic, ntasks), g2f(N1 * XF, npairs, ntasks), g2d(N1 * XD, npairs, ntasks);
  if (ev) (void)hipEventRecord(ev[0], s);
  if (fp32)
    hipLaunchKernelGGL((pass1_fwd_xy<float, N0, N1, NT1, true, bool(PX_SH_PF1), PPF>), g1, dim3(NT1), 0, s, a, tasks);
  else
    hipLaunchKernelGGL((pass1_fwd_xy<double, N0, N1, NT1, false, false, PPD>), g1, dim3(NT1), 0, s, a, tasks);
  if (ev) (void)hipEventRecord(ev[1], s);
  if (fp32 && ex)
    hipLaunchKernelGGL((pass2_z_kernel<float, N0, N1, N2, NT2F, true, true, 1, false, XF>), g2f, dim3(NT2F), 0, s, a, tasks);
  else if (fp32)
    hipLaunchKernelGGL((pass2_z_kernel<float, N0, N1, N2, NT2F, true, false, 1, false, XF>), g2f, dim3(NT2F), 0, s, a, tasks);
  else if (ex)
    hipLaunchKernelGGL((pass2_z_kernel<double, N0, N1, N2, NT2D, false, true, 1, false, XD>), g2d, dim3(NT2D), 0, s, a, tasks);
  else
    hipLaunchKernelGGL((pass2_z_kernel<double, N0, N1, N2, NT2D, false, false, 1, false, XD>), g2d, dim3(NT2D), 0, s, a, tasks);
  if (ev) (void)hipEventRecord(ev[2], s);
  if (fp32) {
    if constexpr (PX_SH_STG3 != 0) {
      if (store_v)
        hipLaunchKernelGGL((pass3_staged<float, N0, N1, NT1, true>), g1, dim3(NT1), 0, s, a, tasks);
      else
        hipLaunchKernelGGL((pass3_staged<float, N0, N1, NT1, false>), g1, dim3(NT1), 0, s, a, tasks);
    } else {
      if (store_v)
        hipLaunchKernelGGL((pass3_inv_xy_acc<float, N0, N1, NT1, false, true, PPF>), g1, dim3(NT1), 0, s, a, tasks);
      else
        hipLaunchKernelGGL((pass3_inv_xy_acc<float, N0, N1, NT1, false, false, PPF>), g1, dim3(NT1), 0, s, a, tasks);
    }
  } else if (store_v)
    hipLaunchKernelGGL((pass3_inv_xy_acc<double, N0, N1, NT1, false, true, PPD>), g1, dim3(NT1), 0, s, a, tasks);
  else
    hipLaunchKernelGGL((pass3_inv_xy_acc<double, N0, N1, NT1, false, false, PPD>), g1, dim3(NT1), 0, s, a, tasks);
  if (ev) (void)hipEventRecord(ev[3], s);
  return hipGetLastError();
}

}  // namespace px
