// Internal interfaces between the host orchestration (px_api.cpp) and the
// kernel translation units.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace px {

// FP64 per-slab sums of one pair product (FP32 form): sum of rho, and sum
// of |rho|^2 of the values handed to the transform.
struct G0Part {
  double re, im, en, pad;
};

// One chunk of orbital pairs: i in [i0, i0+ic) (output orbitals phi_i) times
// j in [j0, j0+jc) (density orbitals psi_j).  Pair p = (i-i0)*jc + (j-j0)
// owns slab p of the pair buffer t ([pairs][n2][n1][n0]).
struct ChunkArgs {
  const void* psi;      // [n_psi][N_g] complex (precision of the call)
  const void* phi;      // [n_phi][N_g]
  void* t;              // pair buffer, >= ic*jc*N_g complex
  void* out;            // [n_phi][N_g]
  const double* occ;    // [n_psi]
  const double* kern;   // [N_g] FP64, FFT order
  const float* kern32;  // [N_g] the same rounded to FP32 (FP32 form; K(0) is read from kern)
  G0Part* g0;           // [ic*jc][n2] FP64 slab sums (FP32 form)
  double* expart;       // FP64 energy partials per (pair, y-plane): sum K|rho(G)|^2 (FP64
                        // form), or {sum_{G!=0} K|rho|^2, sum_{G!=0} |rho|^2, G=0 term} (FP32 form)
  int n2;
  int i0, ic, j0, jc;
  int first;            // pass 3 overwrites the output instead of accumulating
  double* S;            // pair-energy matrix of the instance (task-table mode)
  int s_ld;             // its row stride
  int store_v;          // pass 3 also writes N_g * v_ij back into the pair slab (symmetric mode)
  double inv_ng;
  int tri;              // diagonal block of the symmetric mode (i0 == j0, ic == jc) solved as
                        // its lower triangle jj <= ii: passes 1 and 3 run jj = 0..ii, pass 2
                        // takes the ic (ic + 1) / 2 pairs of the triangle (slots keep the
                        // square layout p = ii jc + jj), pass 4 adds the pairs jj < ii
};

#if defined(__HIPCC__)
// Pairs of a chunk, and the pair slot of the q-th of them (row-major over the
// triangle jj <= ii when tri is set).
__host__ __device__ inline int chunk_pairs(const ChunkArgs& a) {
  return a.tri ? a.ic * (a.ic + 1) / 2 : a.ic * a.jc;
}
__device__ __forceinline__ int pair_slot(const ChunkArgs& a, int q) {
  if (!a.tri) return q;
  int ii = int((sqrt(8.0 * double(q) + 1.0) - 1.0) * 0.5);
  if ((ii + 1) * (ii + 2) / 2 <= q) ++ii;  // rounding of the square root
  if (ii * (ii + 1) / 2 > q) --ii;
  return ii * a.jc + (q - ii * (ii + 1) / 2);
}
#endif

// The chunk of a kernel launch: the launch argument, or entry blockIdx.z of a
// task table in device memory.  A table entry is read through the constant
// address space (scalar loads), so that its fields are known to be uniform:
// the compiler then keeps the base pointers in scalar registers and forms
// addresses from 32-bit per-lane offsets.
#if defined(__HIPCC__)
__device__ __forceinline__ ChunkArgs chunk_args(const ChunkArgs& a0, const ChunkArgs* tasks) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (tasks) {
    typedef const __attribute__((address_space(4))) ChunkArgs CChunk;
    CChunk* c = (CChunk*)(tasks + blockIdx.z);
    ChunkArgs a;
    a.psi = c->psi;
    a.phi = c->phi;
    a.t = c->t;
    a.out = c->out;
    a.occ = c->occ;
    a.kern = c->kern;
    a.kern32 = c->kern32;
    a.g0 = c->g0;
    a.expart = c->expart;
    a.n2 = c->n2;
    a.i0 = c->i0;
    a.ic = c->ic;
    a.j0 = c->j0;
    a.jc = c->jc;
    a.first = c->first;
    a.S = c->S;
    a.s_ld = c->s_ld;
    a.store_v = c->store_v;
    a.inv_ng = c->inv_ng;
    a.tri = c->tri;
    return a;
  }
  return a0;
#else
  return tasks ? tasks[blockIdx.z] : a0;
#endif
}
#endif

// Grids with compiled pipelines: the cubic sizes and the non-cubic shapes.
bool grid_supported(int n0, int n1, int n2);
bool grid_cubic(int n0, int n1, int n2);

// x-sections per y-plane tile of pass 2 (the z transforms, kernel multiply and
// the exchange-energy partials): a pass-2 workgroup takes N0/XS of the plane's
// N0 z-lines, and a pair has N1 * XS energy-partial slots.  Chosen per grid
// size and form by measurement (per 1,024-pair launch, same box): at 96^3 two
// sections of 48 lines (37 KB of LDS in FP32, four workgroups of 192 threads
// per CU instead of two of 384) take FP32 pass 2 from 3.67 to 2.62 ms and FP64
// from 5.47 to 5.11 ms; FP32 at 80^3 2.13 -> 1.74 ms, at 64^3 0.76 -> 0.68 ms;
// at 48^3 and 72^3, and FP64 below 96^3, sections were slower or no faster.
// The build may override the choice for one size (PX_P2_N with PX_P2_XS32 /
// PX_P2_XS64).
constexpr int pass2_sections(bool fp32, int n) {
#if defined(PX_P2_N) && defined(PX_P2_XS32)
  if (fp32 && n == PX_P2_N) return PX_P2_XS32;
#endif
#if defined(PX_P2_N) && defined(PX_P2_XS64)
  if (!fp32 && n == PX_P2_N) return PX_P2_XS64;
#endif
  return n == 96 || (fp32 && (n == 64 || n == 80)) ? 2 : 1;
}
// Pass-2 configuration cfg: 0 the measured default, 1 the alternative that the
// autotuner times as well (one section where the default has two, else two).
constexpr int pass2_sections_cfg(bool fp32, int n, int cfg) {
  return cfg == 0 ? pass2_sections(fp32, n) : (pass2_sections(fp32, n) == 1 ? 2 : 1);
}
// Non-cubic grids: the fewest x-sections (a divisor of n0) that keep a pass-2
// tile (n2 lines of n0/XS + 1 padded values) within 64 KB of LDS in the FP32
// form (two 768-thread workgroups per CU) and within 40 KB in FP64.  Measured
// at 60 x 90 x 120 per 1,024-pair launch: FP32 one section 2.88 ms against
// 3.03 with two; FP64 three sections 4.28 ms against 4.82 with one and 6.00
// with two.  PX_SH_XS32 / PX_SH_XS64 override for timing.
constexpr int shape_sections(bool fp32, int n0, int n2) {
#if defined(PX_SH_XS32)
  if (fp32) return PX_SH_XS32;
#endif
#if defined(PX_SH_XS64)
  if (!fp32) return PX_SH_XS64;
#endif
  for (int xs = 1; xs <= n0; ++xs)
    if (n0 % xs == 0 && n2 * (n0 / xs + 1) * (fp32 ? 8 : 16) <= (fp32 ? 64 : 40) * 1024) return xs;
  return n0;
}
// The same for any grid n[3]: non-cubic grids have one configuration.
inline int pass2_sections_grid(bool fp32, const int* n, int cfg) {
  return grid_cubic(n[0], n[1], n[2]) ? pass2_sections_cfg(fp32, n[0], cfg)
                                      : shape_sections(fp32, n[0], n[2]);
}
// Pass-2 configurations the autotuner can choose from on grid n[3].
inline int pass2_configs(const int* n) { return grid_cubic(n[0], n[1], n[2]) ? 2 : 1; }
// Launches pass 1, 2, 3 of one chunk on grid n[3]; ev (nullable) = 4 events
// recorded before pass 1, between the passes and after pass 3.
hipError_t launch_chunk(bool fp32, const int* n, const ChunkArgs& a, int npairs, bool ex, int p2cfg,
                        hipStream_t s, hipEvent_t* ev);

// The same passes over a task table in device memory (ntasks chunks of one
// grid, all with ic <= max_ic and at most max_pairs solved pairs
// (chunk_pairs), and all with the given store_v), one launch each.
hipError_t launch_chunk_tasks(bool fp32, const int* n, const ChunkArgs* tasks, int ntasks, int max_ic,
                              int max_pairs, bool ex, bool store_v, int p2cfg, hipStream_t s);
// Pass 4 over a task table (tasks without kept v_ij are skipped).
hipError_t launch_pass4_tasks(bool fp32, const ChunkArgs* tasks, int ntasks, int max_jc, size_t ng,
                              hipStream_t s);
// Energy partials -> S for every task of a table (see launch_expart_reduce).
// max_slots: the largest ic * jc of the table.
hipError_t launch_expart_reduce_tasks(bool fp32, const ChunkArgs* tasks, int ntasks, int max_slots,
                                      int n1, int n2, double ng, hipStream_t s);

// Pass 4 (symmetric mode): out[j] -= sum_i f_i/N_g psi_i conj(v_ij) from the
// pair slabs that pass 3 left in the pair buffer.
hipError_t launch_pass4(bool fp32, const ChunkArgs& a, size_t ng, hipStream_t s);

// misc_kernels.hip
hipError_t launch_kernel_hse(int n0, int n1, int n2, double L0, double L1, double L2, double mu,
                             double* kern, hipStream_t s);
hipError_t launch_convert_c128_c64(size_t n, const void* src, void* dst, hipStream_t s);
// n real FP64 values -> FP32 (round to nearest even)
hipError_t launch_convert_f64_f32(size_t n, const double* src, float* dst, hipStream_t s);
hipError_t launch_stream_copy(size_t bytes, const void* src, void* dst, hipStream_t s);
// S[i][j] (row stride lds) from the chunk's energy partials (see ChunkArgs);
// FP32 form (g0 non-null): the G != 0 part is rescaled so that its energy
// matches Parseval's identity with the FP64 energy of the transform input.
hipError_t launch_expart_reduce(const double* expart, const G0Part* g0, int n1, int n2, double ng,
                                int i0, int ic, int j0, int jc, double* S, int lds, bool mirror,
                                bool tri, hipStream_t s);
// e_x = scale * sum_i sum_j f_i f_j S[i][j]
hipError_t launch_energy(const double* S, const double* occ, int n, double scale, double* e_x,
                         hipStream_t s);

// PT-IM-style loop pieces (n = complex element count)
hipError_t launch_midpoint(bool fp32, size_t n, const void* a, const void* b, void* mid,
                           hipStream_t s);
// nxt = phi_n - i*c*(y + y2) (y2 nullable); res = ||nxt - cur|| / ||nxt|| accumulated in FP64
hipError_t launch_ptim_update(bool fp32, size_t n, const void* phi_n, const void* y,
                              const void* y2, const void* cur, void* nxt, double c, double* partial,
                              double* res, hipStream_t s);
int ptim_update_blocks();

// rho[r] = sum_i w[i] |phi_i(r)|^2 (FP64), phi [n][ng] complex in the form's precision
hipError_t launch_density(bool fp32, size_t ng, int n, const void* phi, const double* w,
                          double* rho, hipStream_t s);

// eig_kernels.hip: sigma = Q diag(d) Q^H (FP64, complex128 n x n row-major), d ascending;
// status[0] = 0 when converged within max_sweeps Jacobi sweeps, else the sweeps made.
// work: eig_work_bytes(n).
size_t eig_work_bytes(int n);
hipError_t launch_eig_hermitian(const double* sigma, int n, double* Q, double* d, int32_t* status,
                                void* work, int max_sweeps, hipStream_t s);

// gemm_kernels.hip: complex GEMMs on MFMA
// M[a][b] (a < na, b < nb, row-major ldm) = scale * sum_r conj(X[a][r]) Y[b][r]
//   X: [na][ng], Y: [nb][ng]; FP64 result.  part: workspace of nsplit*na*nb complex128,
//   where nsplit (the splits available) may be below gemm_xhy_part_elems' count: the
//   sum over r then runs in fewer, longer splits.
//   M32 (nullable): the result rounded to complex64 as well, same layout.
hipError_t launch_gemm_xhy(bool fp32, int na, int nb, size_t ng, const void* X, const void* Y,
                           double scale, double* M, int ldm, double* part, int nsplit,
                           float* M32, hipStream_t s);
// The same for a result known to be Hermitian (n x n, ldm = n, e.g. M = dV
// Psi^H W of the ACE construction): only the 64 x 64 tiles on and above the
// diagonal are contracted (about half the flops); each tile below the diagonal
// is the conjugate transpose of its mirror.  The diagonal tiles are computed in
// full, so they keep their (rounding-level) non-Hermitian part.
hipError_t launch_gemm_xhy_herm(bool fp32, int n, size_t ng, const void* X, const void* Y,
                                double scale, double* M, double* part, int nsplit,
                                hipStream_t s);
size_t gemm_xhy_part_elems(int na, int nb, size_t ng, int* nsplit);
// Splits launch_gemm_xhy uses when at most max_split are available (fewer,
// longer splits than the default when max_split is below it).
int gemm_xhy_splits(int na, int nb, size_t ng, int max_split);
// Z[b][r] = alpha * sum_a X[a][r] C[a][b]
//   X: [na][ng], C: [na][ldc] row-major in the precision of the form (complex128, or
//   complex64 rounded from the FP64 matrix), Z: [nb][ng]; upper: C upper triangular
hipError_t launch_gemm_xc(bool fp32, int na, int nb, size_t ng, const void* X, const void* C,
                          int ldc, double alpha, void* Z, bool upper, hipStream_t s);

// chol_kernels.hip: FP64 Hermitian tools on an n x n complex128 matrix (row-major)
hipError_t launch_hermitize(double* M, int n, hipStream_t s);
// U = L^{-H} where -M = L L^H; status[0] = 0 on success or the 1-based failing column
// dinv: workspace of chol_dinv_bytes(n) (inverses of the 32 x 32 diagonal blocks)
size_t chol_dinv_bytes(int n);
hipError_t launch_chol_inv(const double* M, int n, double* L, double* U, int32_t* status,
                           double* dinv, hipStream_t s);
// One factorisation of a group: its matrices and status word (M is hermitized in place).
struct CholJob {
  double* M;
  double* L;
  double* U;
  double* dinv;
  int32_t* status;
  int n;
  int pad;
};
// hermitize + launch_chol_inv for every job of a device-resident table, one
// launch per step for the whole group (blockIdx.z = job); max_n >= every n.
hipError_t launch_chol_inv_group(const CholJob* jobs, int njobs, int max_n, hipStream_t s);
// C = op(A) B, n x n complex128 row-major, op(A) = A^H when ah
hipError_t launch_zgemm(bool ah, int n, const double* A, const double* B, double* C, hipStream_t s);
// C = alpha op(A) B: op(A) m x k (A^H of a k x m A when ah), B k x n, C m x n,
// complex128 row-major with leading dimensions lda, ldb, ldc (elements)
hipError_t launch_zgemm_gen(bool ah, int m, int n, int k, const double* A, int lda, const double* B,
                            int ldb, double* C, int ldc, double alpha, hipStream_t s);
// dst = alpha * src, n real FP64 values
hipError_t launch_scale(size_t n, const double* src, double alpha, double* dst, hipStream_t s);
// nxt = sigma_n - i c (A1 - A2) (n x n complex128); *res = ||nxt - cur|| / ||nxt|| (FP64)
hipError_t launch_sigma_update(int n, const double* sigma_n, const double* A1, const double* A2,
                               const double* cur, double* nxt, double c, double* res, hipStream_t s);
// out[0] = first non-zero of st[0 .. k), else 0
hipError_t launch_status_first(const int32_t* st, int k, int32_t* out, hipStream_t s);

}  // namespace px
