// Complex contractions of the ACE construction and application on MFMA
// (gfx950 matrix cores):
//
//   xhy:  M[a][b] = scale * sum_r conj(X[a][r]) Y[b][r]     (M = dV Psi^H W,
//                                                           C = dV xi^H Phi)
//   xc :  Z[b][r] = alpha * sum_a X[a][r] C[a][b]           (xi = W U,
//                                                           Y = -xi C)
//
// X, Y, Z are orbital blocks [orb][N_g] (complex128 or complex64), C and M are
// small complex128 matrices.  A complex product takes three real MFMAs
// (Gauss): for (a + ib)(c + id), k1 = (a + b) c, k2 = a (d - c),
// k3 = b (c + d), re = k1 - k3, im = k1 + k2, with b = -Im x for the
// conjugated left operand of xhy.  The operand sums are formed in registers
// from the loaded values; against four MFMAs per product this is 9 % faster
// for the ACE application in both forms (512 x 512 x 72^3), at a few more
// accumulator registers.  MFMA: v_mfma_f64_16x16x4f64 (FP64 form) or
// v_mfma_f32_16x16x4f32 (FP32 form).  Operand layout of both 16x16x4 instructions: lane l supplies
// A[l%16][l/16] and B[l/16][l%16].  The result layouts differ: item t of lane
// l holds D[4*(l/16)+t][l%16] for f32 but D[l/16+4*t][l%16] for f64 (checked
// on gfx950 with a one-hot B operand).
//
// xhy splits the long r sum across workgroups; each writes FP64 partials that
// a second kernel adds in a fixed order (deterministic).  In the FP32 form
// the MFMA accumulators cover at most 1024 consecutive r before they are
// added into FP64 registers, which keeps the contraction error near 1e-8.
#include "fft_core.hpp"
#include "px_internal.hpp"

namespace px {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double vd2g __attribute__((ext_vector_type(2)));
typedef float vf2g __attribute__((ext_vector_type(2)));

template <typename T> struct Acc;
template <> struct Acc<double> { using t = d4; };
template <> struct Acc<float> { using t = f4; };

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ cpx<T> load_c(const cpx<T>* p) {
  if constexpr (sizeof(T) == 8) {
    vd2g v = *reinterpret_cast<const vd2g*>(p);
    return {v.x, v.y};
  } else {
    vf2g v = *reinterpret_cast<const vf2g*>(p);
    return {v.x, v.y};
  }
}

typedef float vf4g __attribute__((ext_vector_type(4)));
// Two consecutive complex64 values (16-byte aligned).
__device__ __forceinline__ vf4g gload4(const cpx<float>* p) {
  return *reinterpret_cast<const vf4g*>(p);
}

// Row of the 16x16 result held in item t of a lane with l/16 = q.
template <typename T> __device__ __forceinline__ int drow(int q, int t) {
  return sizeof(T) == 8 ? q + 4 * t : 4 * q + t;
}

constexpr int XHY_SUB = 1024;  // FP32 form: r-span of one FP32 accumulation
constexpr int XHY_KU = 4;      // k-steps of 4 per unrolled iteration (16 r)
constexpr int XC_KU = 4;       // k-steps of 4 per group in xc (16 a)

// ---------------------------------------------------------------- xhy
// grid (ceil(na/64), ceil(nb/64), nsplit), 256 threads; wave w covers the
// 32x32 sub-block (w&1, w>>1) as 2x2 MFMA tiles.  Occupancy target of two
// waves per SIMD: the three accumulator sets fit in 256 registers without
// spills, where the default allocation (FP64) left one wave per SIMD.
// tri > 0 (a Hermitian result, na = nb): only the tiles (ta, tb) with ta <= tb
// of the tri x tri tile grid are computed, blockIdx.x enumerating them row by
// row; the reduction mirrors the others.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_xhy_k(int na, int nb, size_t ng, const cpx<T>* X,
                                                  const cpx<T>* Y, double* part, size_t kchunk,
                                                  int tri) {
  using A = typename Acc<T>::t;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int ta = blockIdx.x, tb = blockIdx.y;
  if (tri > 0) {  // wave-uniform decode of the upper-triangle tile index
    int k = blockIdx.x;
    ta = 0;
    while (k >= tri - ta) {
      k -= tri - ta;
      ++ta;
    }
    tb = ta + k;
  }
  const int a_base = ta * 64 + (w & 1) * 32;
  const int b_base = tb * 64 + (w >> 1) * 32;
  const size_t r_begin = size_t(blockIdx.z) * kchunk;
  const size_t r_end = (r_begin + kchunk < ng) ? r_begin + kchunk : ng;
  const int q = lane >> 4, m = lane & 15;

  const cpx<T>* xrow[2];
  const cpx<T>* yrow[2];
  bool xv[2], yv[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int a = a_base + 16 * t + m, b = b_base + 16 * t + m;
    xv[t] = a < na;
    yv[t] = b < nb;
    xrow[t] = X + size_t(xv[t] ? a : 0) * ng;
    yrow[t] = Y + size_t(yv[t] ? b : 0) * ng;
  }
  // Gauss's three products: with x = a + ib (a = xr, b = -xi) and y = c + id,
  // k1 = (a + b) c, k2 = a (d - c), k3 = b (c + d); re = k1 - k3, im = k1 + k2
  A k1[2][2], k2[2][2], k3[2][2];
  double dre[2][2][4], dim[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      k1[i][j] = k2[i][j] = k3[i][j] = A{0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < 4; ++t) dre[i][j][t] = dim[i][j][t] = 0.0;
    }

  // Groups of 4*XHY_KU consecutive r.  Two register sets alternate: the next
  // group loads into the idle set while the current one feeds the MFMAs.
  // Loads past the chunk end read a valid address and are masked to zero, so
  // every iteration issues the same loads (the group count is padded to even).
  constexpr size_t GR = 4 * XHY_KU;
  constexpr size_t GPS = XHY_SUB / GR;  // groups per FP32 accumulation span
  const size_t ngroups = r_end > r_begin ? (r_end - r_begin + GR - 1) / GR : 0;
  // (FP32: each lane's four consecutive complex values of a row come in two
  // 16-byte loads, which halves the address work of the gather; the grids
  // have N_g and the chunk bounds even, so a pair never straddles the end)
  auto load = [&](size_t g, cpx<T>(&xa)[2][XHY_KU], cpx<T>(&yb)[2][XHY_KU]) {
    const size_t rl = r_begin + g * GR + 4 * q;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int s = 0; s < XHY_KU; s += 2) {
          const size_t r = rl + s;
          const bool in = r < r_end;
          const size_t rc = in ? r : r_begin;
          const vf4g x = gload4(xrow[t] + rc), y = gload4(yrow[t] + rc);
          const bool ux = in && xv[t], uy = in && yv[t];
          xa[t][s] = ux ? cpx<T>{x.x, x.y} : cpx<T>{T(0), T(0)};
          xa[t][s + 1] = ux ? cpx<T>{x.z, x.w} : cpx<T>{T(0), T(0)};
          yb[t][s] = uy ? cpx<T>{y.x, y.y} : cpx<T>{T(0), T(0)};
          yb[t][s + 1] = uy ? cpx<T>{y.z, y.w} : cpx<T>{T(0), T(0)};
        }
      } else {
#pragma unroll
        for (int s = 0; s < XHY_KU; ++s) {
          const size_t r = rl + s;
          const bool in = r < r_end;
          const size_t rc = in ? r : r_begin;
          const cpx<T> x = load_c(xrow[t] + rc), y = load_c(yrow[t] + rc);
          xa[t][s] = (in && xv[t]) ? x : cpx<T>{T(0), T(0)};
          yb[t][s] = (in && yv[t]) ? y : cpx<T>{T(0), T(0)};
        }
      }
    }
  };
  auto compute = [&](size_t g, cpx<T>(&xa)[2][XHY_KU], cpx<T>(&yb)[2][XHY_KU]) {
#pragma unroll
    for (int s = 0; s < XHY_KU; ++s) {
      T xs[2], yd[2], ys[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        xs[t] = xa[t][s].x - xa[t][s].y;
        yd[t] = yb[t][s].y - yb[t][s].x;
        ys[t] = yb[t][s].x + yb[t][s].y;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          k1[i][j] = mfma(xs[i], yb[j][s].x, k1[i][j]);
          k2[i][j] = mfma(xa[i][s].x, yd[j], k2[i][j]);
          k3[i][j] = mfma(-xa[i][s].y, ys[j], k3[i][j]);
        }
    }
    if constexpr (sizeof(T) == 4) {
      // FP32 accumulators span at most XHY_SUB values of r, then go to FP64
      // (a padding group adds zeros, so a repeated flush is harmless)
      if ((g + 1) % GPS == 0 || g + 1 >= ngroups) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              dre[i][j][t] += double(k1[i][j][t]) - double(k3[i][j][t]);
              dim[i][j][t] += double(k1[i][j][t]) + double(k2[i][j][t]);
            }
            k1[i][j] = k2[i][j] = k3[i][j] = A{0, 0, 0, 0};
          }
      }
    }
  };
  if (ngroups > 0) {
    cpx<T> xa0[2][XHY_KU], yb0[2][XHY_KU], xa1[2][XHY_KU], yb1[2][XHY_KU];
    load(0, xa0, yb0);
    for (size_t g = 0; g < ngroups; g += 2) {
      load(g + 1, xa1, yb1);
      compute(g, xa0, yb0);
      load(g + 2, xa0, yb0);
      compute(g + 1, xa1, yb1);
    }
  }
  double* out = part + size_t(blockIdx.z) * na * nb * 2;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int a = a_base + 16 * i + drow<T>(q, t), b = b_base + 16 * j + m;
        if (a < na && b < nb) {
          double re, im;
          if constexpr (sizeof(T) == 4) {
            re = dre[i][j][t];
            im = dim[i][j][t];
          } else {
            re = k1[i][j][t] - k3[i][j][t];
            im = k1[i][j][t] + k2[i][j][t];
          }
          out[(size_t(a) * nb + b) * 2] = re;
          out[(size_t(a) * nb + b) * 2 + 1] = im;
        }
      }
}

__global__ void xhy_reduce_k(int na, int nb, const double* part, int nsplit, double scale,
                             double* M, int ldm, float* M32, int herm) {
  const size_t n = size_t(na) * nb;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
       e += size_t(gridDim.x) * blockDim.x) {
    const size_t a = e / nb, b = e % nb;
    // a Hermitian result keeps only the tiles on and above the diagonal:
    // entries below it are the conjugates of their mirror images
    const bool mirror = herm && (a / 64) > (b / 64);
    const size_t src = mirror ? b * nb + a : e;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < nsplit; ++s) {
      re += part[(size_t(s) * n + src) * 2];
      im += part[(size_t(s) * n + src) * 2 + 1];
    }
    if (mirror) im = -im;
    M[(a * ldm + b) * 2] = scale * re;
    M[(a * ldm + b) * 2 + 1] = scale * im;
    if (M32) {  // the same, rounded to FP32 (operand of an FP32 contraction)
      M32[(a * ldm + b) * 2] = float(scale * re);
      M32[(a * ldm + b) * 2 + 1] = float(scale * im);
    }
  }
}

// r-span of one split: aim at ~2048 workgroups, at least 1024 values of r,
// and at most max_split splits (the partials need max_split * na * nb
// complex128 values of scratch).  Among 1 to 2 times the aimed split count the
// one whose workgroups best fill whole rounds of the resident ones (two per CU
// on 256 CUs) is taken: the workgroups of a launch all run about equally long,
// so a last round half full idles half the chip for one workgroup's time
// (ACE application at 96^3 x 1536: 4 -> 8 splits, about -2 %).  herm counts
// the tiles on and above the diagonal that the Hermitian form launches.
static size_t xhy_kchunk(int na, int nb, size_t ng, int max_split, bool herm, int* nsplit) {
  constexpr size_t kResident = 2 * 256;
  const size_t ta = size_t(na + 63) / 64, tb = size_t(nb + 63) / 64;
  const size_t tiles = herm ? ta * (ta + 1) / 2 : ta * tb;
  const size_t want0 = (2048 + tiles - 1) / tiles;
  size_t want = want0;
  double best = 0.0;
  for (size_t s = want0; s <= 2 * want0; ++s) {
    const size_t wg = tiles * s, rounds = (wg + kResident - 1) / kResident;
    const double fill = double(wg) / double(rounds * kResident);
    if (fill > best + 1e-9) {
      best = fill;
      want = s;
    }
  }
  size_t kchunk = (ng + want - 1) / want;
  if (kchunk < 1024) kchunk = 1024;
  if (max_split > 0 && (ng + kchunk - 1) / kchunk > size_t(max_split))
    kchunk = (ng + size_t(max_split) - 1) / size_t(max_split);
  kchunk = (kchunk + 15) / 16 * 16;
  *nsplit = int((ng + kchunk - 1) / kchunk);
  return kchunk;
}

size_t gemm_xhy_part_elems(int na, int nb, size_t ng, int* nsplit) {
  xhy_kchunk(na, nb, ng, 0, false, nsplit);
  return size_t(*nsplit) * na * nb;
}

int gemm_xhy_splits(int na, int nb, size_t ng, int max_split) {
  int nsplit = 0;
  xhy_kchunk(na, nb, ng, max_split, false, &nsplit);
  return nsplit;
}

static hipError_t xhy_launch(bool fp32, int na, int nb, size_t ng, const void* X, const void* Y,
                             double scale, double* M, int ldm, double* part, int nsplit_avail,
                             float* M32, bool herm, hipStream_t s) {
  int nsplit;
  const size_t kchunk = xhy_kchunk(na, nb, ng, nsplit_avail, herm, &nsplit);
  if (nsplit > nsplit_avail || (herm && na != nb)) return hipErrorInvalidValue;
  const int ta = (na + 63) / 64, tb = (nb + 63) / 64;
  const int tri = herm ? ta : 0;
  dim3 grid(herm ? ta * (ta + 1) / 2 : ta, herm ? 1 : tb, nsplit);
  if (fp32)
    hipLaunchKernelGGL(gemm_xhy_k<float>, grid, dim3(256), 0, s, na, nb, ng,
                       static_cast<const cpx<float>*>(X), static_cast<const cpx<float>*>(Y), part,
                       kchunk, tri);
  else
    hipLaunchKernelGGL(gemm_xhy_k<double>, grid, dim3(256), 0, s, na, nb, ng,
                       static_cast<const cpx<double>*>(X), static_cast<const cpx<double>*>(Y),
                       part, kchunk, tri);
  const size_t n = size_t(na) * nb;
  const int blocks = int((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(xhy_reduce_k, dim3(blocks), dim3(256), 0, s, na, nb, part, nsplit, scale, M,
                     ldm, M32, int(herm));
  return hipGetLastError();
}

hipError_t launch_gemm_xhy(bool fp32, int na, int nb, size_t ng, const void* X, const void* Y,
                           double scale, double* M, int ldm, double* part, int nsplit_avail,
                           float* M32, hipStream_t s) {
  return xhy_launch(fp32, na, nb, ng, X, Y, scale, M, ldm, part, nsplit_avail, M32, false, s);
}

hipError_t launch_gemm_xhy_herm(bool fp32, int n, size_t ng, const void* X, const void* Y,
                                double scale, double* M, double* part, int nsplit_avail,
                                hipStream_t s) {
  return xhy_launch(fp32, n, n, ng, X, Y, scale, M, n, part, nsplit_avail, nullptr, true, s);
}

// ---------------------------------------------------------------- xc
// grid ceil(ng/64) * ceil(nb/64) in one dimension.  Dense C: the b tile
// varies fastest, so the workgroups that share an r tile of X run together
// and read it through the caches once, and each XCD (every eighth workgroup)
// keeps a few b column blocks of C in its L2 (ACE application at 96^3 x 1536
// -2 %, at 72^3 x 512 -6 %, against r tiles fastest).  Upper-triangular C
// (upper): the r tile varies fastest, so the workgroups in flight share one b
// tile and the same sum length (b-fastest mixes lengths 1 to nb/64 and was
// 21 % slower for xi = W U at 96^3 x 1536).  256 threads; wave w covers
// r-block (w&1) and b-block (w>>1) of 32 each, as 2x2 MFMA tiles (i: r,
// j: b).  Occupancy
// targets (no spills): three waves per SIMD in the FP32 form, two in FP64
// (one by default; ACE application in FP64 -15 %).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 2))) void gemm_xc_k(int na, int nb, size_t ng, const cpx<T>* X,
                                                 const T* C, int ldc, double alpha,
                                                 cpx<T>* Z, int upper) {
  using A = typename Acc<T>::t;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned nbt = unsigned(nb + 63) / 64, nrt = unsigned((ng + 63) / 64);
  const int bt = int(upper ? blockIdx.x / nrt : blockIdx.x % nbt);
  const size_t rt = upper ? blockIdx.x % nrt : blockIdx.x / nbt;
  const size_t r_base = rt * 64 + (w & 1) * 32;
  const int b_base = bt * 64 + (w >> 1) * 32;
  const int q = lane >> 4, m = lane & 15;
  int a_end = na;
  if (upper) {
    const int lim = bt * 64 + 64;
    a_end = lim < na ? lim : na;
  }
  bool rv[2], bv[2];
  size_t rr[2];
  int bb[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    rr[t] = r_base + 16 * t + m;
    rv[t] = rr[t] < ng;
    bb[t] = b_base + 16 * t + m;
    bv[t] = bb[t] < nb;
  }
  // Gauss's three products (x = a + ib, C entry c + id): k1 = (a + b) c,
  // k2 = a (d - c), k3 = b (c + d); re = k1 - k3, im = k1 + k2
  A k1[2][2], k2[2][2], k3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) k1[i][j] = k2[i][j] = k3[i][j] = A{0, 0, 0, 0};
  // Groups of 4*XC_KU consecutive a (4 per MFMA k-step); two register sets
  // alternate as in xhy, with masked loads from clamped addresses.
  const size_t rc[2] = {rv[0] ? rr[0] : 0, rv[1] ? rr[1] : 0};
  const int bc[2] = {bv[0] ? bb[0] : 0, bv[1] ? bb[1] : 0};
  constexpr int GA = 4 * XC_KU;
  const int ngroups = (a_end + GA - 1) / GA;
  auto load = [&](int g, cpx<T>(&xa)[2][XC_KU], cpx<T>(&cb)[2][XC_KU]) {
#pragma unroll
    for (int s = 0; s < XC_KU; ++s) {
      const int a = g * GA + 4 * s + q;
      const bool av = a < a_end;
      const int ac = av ? a : 0;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const cpx<T> x = load_c(X + size_t(ac) * ng + rc[t]);
        const T* c = C + (size_t(ac) * ldc + bc[t]) * 2;
        const T c0 = c[0], c1 = c[1];
        xa[t][s] = (av && rv[t]) ? x : cpx<T>{T(0), T(0)};
        cb[t][s] = (av && bv[t]) ? cpx<T>{c0, c1} : cpx<T>{T(0), T(0)};
      }
    }
  };
  auto compute = [&](cpx<T>(&xa)[2][XC_KU], cpx<T>(&cb)[2][XC_KU]) {
#pragma unroll
    for (int s = 0; s < XC_KU; ++s) {
      T xs[2], cd[2], cs[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        xs[t] = xa[t][s].x + xa[t][s].y;
        cd[t] = cb[t][s].y - cb[t][s].x;
        cs[t] = cb[t][s].x + cb[t][s].y;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          k1[i][j] = mfma(xs[i], cb[j][s].x, k1[i][j]);
          k2[i][j] = mfma(xa[i][s].x, cd[j], k2[i][j]);
          k3[i][j] = mfma(xa[i][s].y, cs[j], k3[i][j]);
        }
    }
  };
  if (ngroups > 0) {
    cpx<T> xa0[2][XC_KU], cb0[2][XC_KU], xa1[2][XC_KU], cb1[2][XC_KU];
    load(0, xa0, cb0);
    for (int g = 0; g < ngroups; g += 2) {
      load(g + 1, xa1, cb1);
      compute(xa0, cb0);
      load(g + 2, xa0, cb0);
      compute(xa1, cb1);
    }
  }
  const T al = T(alpha);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int b = b_base + 16 * j + m;
      if (b >= nb) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const size_t r = r_base + 16 * i + drow<T>(q, t);
        if (r < ng) {
          cpx<T>* o = Z + size_t(b) * ng + r;
          o->x = al * (k1[i][j][t] - k3[i][j][t]);
          o->y = al * (k1[i][j][t] + k2[i][j][t]);
        }
      }
    }
}

hipError_t launch_gemm_xc(bool fp32, int na, int nb, size_t ng, const void* X, const void* C,
                          int ldc, double alpha, void* Z, bool upper, hipStream_t s) {
  dim3 grid(unsigned((ng + 63) / 64) * unsigned((nb + 63) / 64));
  if (fp32)
    hipLaunchKernelGGL(gemm_xc_k<float>, grid, dim3(256), 0, s, na, nb, ng,
                       static_cast<const cpx<float>*>(X), static_cast<const float*>(C), ldc,
                       alpha, static_cast<cpx<float>*>(Z), int(upper));
  else
    hipLaunchKernelGGL(gemm_xc_k<double>, grid, dim3(256), 0, s, na, nb, ng,
                       static_cast<const cpx<double>*>(X), static_cast<const double*>(C), ldc,
                       alpha, static_cast<cpx<double>*>(Z), int(upper));
  return hipGetLastError();
}

}  // namespace px
