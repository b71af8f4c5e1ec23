/* px.h -- C ABI of libpx: the Fock exchange operator with fractional
 * occupations and its adaptively compressed (ACE) form on AMD MI355X (gfx950).
 *
 * Problem statement (arXiv 2501.03061):
 *   Sec. II-B, Eq. (8)-(10): the exchange operator Vx[P](r,r') = -P(r,r') K(r,r')
 *     with a (possibly screened) interaction kernel K.
 *   Sec. IV-A-1, Eq. (11)-(13): once the occupation matrix is diagonalised,
 *     P = sum_j f_j psi_j psi_j^*, and
 *       (Vx phi_i)(r) = -sum_j f_j psi_j(r) IFFT[ K(G) FFT(conj(psi_j) phi_i) ](r),
 *     N_phi * N_psi pair solves.
 *   Sec. IV-A-2, Eq. (14): ACE, W = Vx Psi reproduced exactly by
 *     V_ACE = -xi xi^H on span(Psi).
 *
 * Conventions shared by every entry point
 *   Grid and cell: orthorhombic cell of edge lengths L[0..2] (bohr), grid
 *     n[0] x n[1] x n[2]; Omega = L0 L1 L2, N_g = n0 n1 n2, dV = Omega/N_g.
 *   Layout: every orbital block is orbital-major and C-ordered
 *     [orbital][n2][n1][n0] (x = n0 fastest), interleaved complex (re, im):
 *     complex128 for PX_PREC_FP64, complex64 for PX_PREC_FP32.
 *     occ is float64 [n_psi]; kernel_G is float64 [n2][n1][n0] in FFT index
 *     order (index m has frequency m if m < n/2, else m - n).
 *     Small matrices (M) are complex128, row-major, n x n.
 *   Units: atomic units.  The hybrid mixing fraction alpha of Eq. (8) is NOT
 *     applied (the library returns Vx); there is no spin factor.
 *   FFT convention: forward exp(-iG.r) unnormalised, inverse exp(+iG.r) with
 *     1/N_g; for a real even kernel the result does not depend on the sign.
 *   Alignment: orbital blocks (psi, phi, xi and the outputs) must be 16-byte
 *     aligned; every orbital of a block then is too, since N_g is even on the
 *     grids with FFT plans (all their axes are even) and must be even for FP32
 *     blocks in the contraction-only entry points.  Misaligned blocks:
 *     PX_ERR_INVALID_ARG.
 *   Memory: all array arguments are DEVICE pointers owned by the caller.  The
 *     library never allocates or frees device memory; scratch space comes from
 *     the workspace the caller attaches with px_set_workspace, sized by
 *     px_workspace_bytes.  Outputs must not alias inputs.
 *   Streams: every compute call only enqueues work on `stream` (a
 *     hipStream_t; NULL = default stream) and returns; no host synchronisation
 *     except in px_sync.
 *   Errors: arguments are validated on the host before anything is enqueued;
 *     a non-PX_OK return means nothing was enqueued.  px_last_error gives a
 *     message.  Device-side failures (Cholesky breakdown, a diagonalisation
 *     that did not converge) are reported through the caller's status word
 *     and surfaced by px_sync.
 *   Precision forms: PX_PREC_FP64 runs everything in FP64.  PX_PREC_FP32 runs
 *     pair products, FFTs and contractions in FP32 (FP32 MFMA accumulation)
 *     while the G = 0 coefficient, the exchange energy sums, the reductions of
 *     contraction partials, the Cholesky factorisation and the triangular
 *     inverse stay FP64.
 */
#ifndef PX_H_
#define PX_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PX_ABI_VERSION 1

typedef enum {
  PX_OK = 0,
  PX_ERR_INVALID_ARG = 1,           /* null pointer, bad size, bad aliasing      */
  PX_ERR_UNSUPPORTED_GRID = 2,      /* grid shape without a compiled FFT plan    */
  PX_ERR_WORKSPACE = 3,             /* no workspace attached or too small        */
  PX_ERR_DEVICE = 4,                /* a HIP runtime call failed                 */
  PX_ERR_NOT_POSITIVE_DEFINITE = 5, /* -M is not positive definite (px_sync)     */
  PX_ERR_NOT_CONVERGED = 6          /* sigma diagonalisation did not converge    */
} px_status;

typedef enum { PX_PREC_FP64 = 0, PX_PREC_FP32 = 1 } px_precision;

typedef enum {
  PX_OP_EXCHANGE = 0,
  PX_OP_ACE_BUILD = 1,
  PX_OP_ACE_APPLY = 2,
  PX_OP_PTIM_LOOP = 3,
  PX_OP_EXCHANGE_SIGMA = 4,  /* n_psi = n (Phi and sigma), n_phi = n_tgt */
  PX_OP_SIGMA_DIAG = 5,      /* n_psi = n; n_phi ignored                 */
  PX_OP_DENSITY_SIGMA = 6,   /* n_psi = n; n_phi ignored                 */
  PX_OP_PTIM_STEP = 7,       /* n_psi = n (rank of xi), n_phi            */
  PX_OP_ACE_BUILD_SIGMA = 8, /* n_psi = n (Phi and sigma); n_phi ignored */
  PX_OP_ROTATE = 9,          /* n_psi = n; n_phi ignored                 */
  PX_OP_DENSITY_FINE = 10    /* n_psi = n; n_phi ignored                 */
} px_op;

/* Orthorhombic cell: edge lengths in bohr and the real-space grid, n[0] = x. */
typedef struct {
  double L[3];
  int32_t n[3];
} px_cell;

typedef struct px_context px_context;

/* Returns PX_ABI_VERSION of the loaded library. */
int32_t px_abi_version(void);

/* Creates a context bound to HIP device `device` (host state only: tuning
 * table, latched errors, attached workspace).  *ctx receives the handle. */
px_status px_create(int32_t device, px_context** ctx);

/* Destroys a context; NULL is accepted.  Does not free the workspace. */
void px_destroy(px_context* ctx);

/* Message of the last failure on this context (never NULL). */
const char* px_last_error(const px_context* ctx);

/* Whether the grid of `cell` has compiled FFT plans in precision `prec`
 * (1 = yes).  Supported: cubic n in {16,24,32,40,48,60,64,72,80,96}, and the
 * non-cubic (n[0], n[1], n[2]) = (60, 60, 90) and (60, 90, 120), the
 * wavefunction grids of the 768- and 1536-atom cells of Sec. VI (their
 * pipelines use configurations derived from the FFT plans, without per-size
 * tuning). */
int32_t px_grid_supported(const px_cell* cell, px_precision prec);

/* Bytes of workspace that `op` needs for this problem with the context's
 * current tuning; 0 if the arguments are invalid.  n_phi is ignored for
 * PX_OP_ACE_BUILD (Phi = Psi). */
size_t px_workspace_bytes(const px_context* ctx, px_op op, const px_cell* cell, px_precision prec,
                          int32_t n_psi, int32_t n_phi);

/* Attaches caller-owned device memory as the workspace (256-byte aligned).
 * The same buffer serves every later call on the context; calls that overlap
 * in time on different streams must not share a context. */
px_status px_set_workspace(px_context* ctx, void* dev_ptr, size_t bytes);

/* Pair-chunk tuning: a chunk is ic output orbitals x jc density orbitals whose
 * pair slabs are in flight together (Sec. III-B(b) batches 16 pairs on its
 * GPU).  0 restores the default.  Changes px_workspace_bytes.  The pass-2
 * configuration that px_autotune chose for the grid is kept. */
px_status px_set_tuning(px_context* ctx, const px_cell* cell, px_precision prec, int32_t ic,
                        int32_t jc);

/* Fills kernel_G (device, float64 [n2][n1][n0], FFT order) with the HSE06
 * screened interaction K(G) = 4 pi (1 - exp(-G^2/(4 mu^2)))/G^2, K(0) = pi/mu^2
 * (Sec. II-B: "possibly screened" kernel; Sec. VI: HSE06). */
px_status px_kernel_hse(px_context* ctx, const px_cell* cell, double mu, double* kernel_G,
                        hipStream_t stream);

/* Rounds n_elems complex128 values to complex64 (round to nearest even):
 * the staging step of the FP32 form.  src and dst are device pointers. */
px_status px_convert_c128_to_c64(px_context* ctx, size_t n_elems, const void* src, void* dst,
                                 hipStream_t stream);

/* Plain device-to-device copy of `bytes` (a multiple of 16; 16-byte aligned
 * pointers).  Not part of the method: it is the reference kernel whose
 * measured bandwidth and HBM counters calibrate the roofline figures. */
px_status px_stream_copy(px_context* ctx, const void* src, void* dst, size_t bytes,
                         hipStream_t stream);

/* Exchange operator applied to a block, Eq. (13) with occupations f_j:
 *   vx_phi[i] = (Vx phi_i) = -sum_j occ[j] psi_j IFFT[K FFT(conj(psi_j) phi_i)]
 * psi [n_psi][N_g], phi [n_phi][N_g], vx_phi [n_phi][N_g] in the element type
 * of `prec`; occ, kernel_G FP64.  e_x (nullable, device, one float64) receives
 *   E_x = 1/2 sum_i f_i <psi_i|Vx psi_i> = -Omega/(2 N_g^2) sum_ij f_i f_j sum_G K |FFT(conj(psi_j) psi_i)|^2,
 * accumulated in FP64; it requires phi == psi and n_phi == n_psi. */
px_status px_exchange_apply(px_context* ctx, const px_cell* cell, px_precision prec,
                            int32_t n_psi, const void* psi, const double* occ, int32_t n_phi,
                            const void* phi, const double* kernel_G, void* vx_phi, double* e_x,
                            hipStream_t stream);

/* ACE construction (Eq. 14; steps: W = Vx Psi, M = dV Psi^H W, M <- (M+M^H)/2,
 * -M = L L^H with L lower and real positive diagonal, xi = W L^{-H}).
 * psi [n][N_g] (element type of prec), occ FP64 [n], kernel_G FP64.
 * Outputs: xi [n][N_g] (element type of prec); M (nullable) complex128 [n][n]
 * after Hermitisation; e_x (nullable) as in px_exchange_apply; status (device
 * int32, required): 0 on success, else the 1-based column where the Cholesky
 * factorisation of -M broke down (xi is then undefined).
 * In the Hermitian-pair mode (px_set_symmetry, on by default) each unordered
 * pair is solved once and v_ji = conj(v_ij) is used for the other; that holds
 * only for a real kernel with K(G) = K(-G) (true of px_kernel_hse and of any
 * radial interaction).  For another kernel turn the mode off: with it on, the
 * pairs (i, j) with j <= i use K(G) and the transposed pairs (j, i) use
 * conj(K(-G)) instead (they reuse conj(v_ij)). */
px_status px_ace_build(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                       const void* psi, const double* occ, const double* kernel_G, void* xi,
                       double* M, double* e_x, int32_t* status, hipStream_t stream);

/* ACE application (Eq. 14): out = V_ACE phi = -xi (dV xi^H phi).
 * xi [n][N_g], phi and out [n_phi][N_g], element type of prec.  Only
 * contractions: any grid in the FP64 form; the FP32 form needs an even N_g
 * (PX_ERR_UNSUPPORTED_GRID otherwise). */
px_status px_ace_apply(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                       const void* xi, int32_t n_phi, const void* phi, void* out,
                       hipStream_t stream);

/* ACE application without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight loops and harnesses that
 * forbid allocation).  Same operation, arguments and errors as px_ace_apply;
 * the contraction scratch (C = dV xi^H phi, its complex64 copy and the split
 * partials of the N_g sum) is a 64 MiB array in the library's device memory,
 * one per GPU, held until the process ends, instead of the workspace.  Needs
 * 40 * n * n_phi bytes of it at least (n * n_phi <= 1,677,721; larger:
 * PX_ERR_WORKSPACE); when the default number of splits does not fit, the N_g
 * sum runs in fewer, longer splits.  No device memory is allocated or freed.
 * Calls on one GPU share its array: calls that overlap in time on one GPU
 * (other streams, other contexts, other threads) race and give undefined
 * results; nothing in the array needs to be cleared between calls. */
px_status px_ace_apply_noalloc(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                               const void* xi, int32_t n_phi, const void* phi, void* out,
                               hipStream_t stream);

/* Exchange-only implicit-midpoint fixed point with the ACE operator (the
 * orbital update of Eq. 6 at the midpoint of Eq. 4, keeping only alpha*Vx of
 * Eq. 8 and no projector, iterated as x = T(x) of Eq. 7):
 *   Phi^(k+1) = Phi_n - i*dt_alpha * V_ACE (Phi_n + Phi^(k))/2,  Phi^(0) = Phi_n,
 * for k = 0 .. n_iter-1, with residual R_k = ||Phi^(k+1) - Phi^(k)||_F / ||Phi^(k+1)||_F
 * accumulated in FP64.  dt_alpha = dt * alpha (e.g. 50 as * 0.25).
 * xi [n][N_g], phi_n and phi_out [n_phi][N_g] (element type of prec),
 * residuals: device float64 [n_iter].  Grids as in px_ace_apply. */
px_status px_ptim_exchange_loop(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                                const void* xi, int32_t n_phi, const void* phi_n, int32_t n_iter,
                                double dt_alpha, void* phi_out, double* residuals,
                                hipStream_t stream);

/* Occupation-matrix diagonalisation (Sec. IV-A-1, Eq. 11): sigma = Q D Q^H
 * for a Hermitian sigma (the input is Hermitised as (sigma + sigma^H)/2 first),
 * in FP64 by cyclic Jacobi rotations (blocked: pairs of 16-index blocks per
 * round, each pair's 32 x 32 subproblem rotated in LDS).  sigma and Q: complex128 [n][n]
 * row-major (device; Q[a][k] is component a of eigenvector k); d: float64 [n],
 * the eigenvalues in ascending order.  Eigenvectors are unique up to a phase
 * (and a rotation within a degenerate eigenspace); Q D Q^H is unique.
 * status (device int32, required): 0 when the off-diagonal Frobenius norm fell
 * below 64 eps sqrt(n) ||sigma||_F within 40 sweeps, else the sweeps made
 * (Q, d then approximate; px_sync returns PX_ERR_NOT_CONVERGED).  Workspace:
 * px_workspace_bytes(PX_OP_SIGMA_DIAG, cell (any), FP64, n, 0). */
px_status px_sigma_diagonalize(px_context* ctx, int32_t n, const double* sigma, double* Q, double* d,
                               int32_t* status, hipStream_t stream);

/* Mixed-state exchange operator with a full occupation matrix (Eq. 10),
 *   vx_tgt[j] = -sum_{i,k} sigma_ik Phi_i IFFT[K FFT(conj(Phi_k) tgt_j)],
 * evaluated as the paper does after Eq. 11: sigma = Q D Q^H, phi = Phi Q
 * (a contraction over the orbitals, in the form's precision), then Eq. 13 on
 * (phi, d): N^2 pair solves instead of N^3.  Phi [n][N_g], tgt and vx_tgt
 * [n_tgt][N_g] (element type of prec; tgt may be Phi itself), sigma
 * complex128 [n][n], kernel_G as in px_exchange_apply.  status as in
 * px_sigma_diagonalize.  Workspace: PX_OP_EXCHANGE_SIGMA with (n, n_tgt). */
px_status px_exchange_apply_sigma(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                                  const void* phi_basis, const double* sigma, int32_t n_tgt,
                                  const void* tgt, const double* kernel_G, void* vx_tgt,
                                  int32_t* status, hipStream_t stream);

/* Electron density of orbitals with occupations (Eq. 12 with sigma
 * diagonalised: rho(r) = sum_i occ_i |phi_i(r)|^2, the density the paper
 * evaluates with N products after the diagonalisation instead of N^2).
 * phi [n][N_g] (element type of prec), occ float64 [n] (any real weights, e.g.
 * the d of px_sigma_diagonalize), rho float64 [N_g] on the wavefunction grid.
 * Products and sums in FP64 in both forms.  No workspace.  Grids as in
 * px_ace_apply. */
px_status px_density(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                     const void* phi, const double* occ, double* rho, hipStream_t stream);

/* The density of px_density on the charge-density grid, twice as fine per
 * axis as the wavefunction grid (Sec. VI: 120 x 180 x 240 for 60 x 90 x 120):
 * rho_fine = sum_i occ_i |phi_i^f|^2 with phi_i^f the trigonometric
 * interpolation of phi_i onto the fine grid (its spectrum zero-padded; the
 * Nyquist coefficient of each axis split evenly between +n/2 and -n/2), so
 * that rho_fine at even indices equals the density on the wavefunction grid
 * and no product aliases.  phi [n][N_g] (element type of prec), occ float64
 * [n], rho_fine float64 [2 n2][2 n1][2 n0].  The interpolation runs in the
 * form's precision, the squares and sums in FP64.  Every axis must be even
 * and at most 120 points (PX_ERR_UNSUPPORTED_GRID otherwise; any such grid,
 * with or without an FFT plan).  Workspace: PX_OP_DENSITY_FINE with n
 * (10 N_g values of the form's type for each of 16 orbitals in flight). */
px_status px_density_fine(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                          const void* phi, const double* occ, double* rho_fine, hipStream_t stream);

/* Density with a full occupation matrix (Sec. III-C:
 * rho(r) = sum_{i,j} Phi_i(r) sigma_ij conj(Phi_j(r))), evaluated as
 * diagonalisation, phi = Phi Q and px_density on (phi, d).  Phi [n][N_g],
 * sigma complex128 [n][n], rho float64 [N_g]; status as in
 * px_sigma_diagonalize.  Workspace: PX_OP_DENSITY_SIGMA with n. */
px_status px_density_sigma(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                           const void* phi_basis, const double* sigma, double* rho, int32_t* status,
                           hipStream_t stream);

/* The orbitals of the diagonal form (Eq. 11): phi = Phi Q, orbital b of phi
 * being sum_a Q[a][b] Phi_a (with Q from px_sigma_diagonalize, phi and d
 * feed px_ace_build, px_exchange_apply and px_density, so that one
 * diagonalisation serves both the density of a state and the exchange
 * operator of the next step).  Phi and phi_out [n][N_g] (element type of
 * prec, no aliasing), Q complex128 [n][n] row-major (device).  A contraction
 * over the orbitals on the matrix cores, in the form's precision (the FP32
 * form rounds Q to complex64 in the workspace, PX_OP_ROTATE with n; the FP64
 * form reads Q directly and needs no workspace).  Grids as in px_ace_apply. */
px_status px_rotate_orbitals(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                             const void* phi_basis, const double* Q, void* phi_out, hipStream_t stream);

/* ACE construction for a full occupation matrix (Eq. 10 compressed as in
 * Eq. 14, evaluated through Eq. 11-13): sigma = Q D Q^H, phi = Phi Q, then
 * the construction of px_ace_build on (phi, d).  phi spans the space of Phi,
 * so V_ACE = -xi xi^H reproduces Vx[sigma] on every vector of span(Phi).
 * Phi [n][N_g] (element type of prec), sigma complex128 [n][n] (Hermitian;
 * its eigenvalues are the occupations d, normally in [0, 1]), kernel_G as in
 * px_exchange_apply.  Outputs: xi [n][N_g]; M (nullable) complex128 [n][n],
 * dV phi^H W in the eigenbasis of sigma (it depends on the phases chosen for
 * Q; xi xi^H does not); e_x (nullable) = (1/2) Tr(sigma Phi^H Vx[sigma] Phi) dV,
 * the exchange energy of Eq. 10.  status (device int32 [2], required):
 * status[0] as in px_sigma_diagonalize, status[1] as the status of
 * px_ace_build; px_sync reports either.  Workspace: PX_OP_ACE_BUILD_SIGMA with
 * n.  Kernel evenness as for px_ace_build (the Hermitian-pair mode applies). */
px_status px_ace_build_sigma(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                             const void* phi_basis, const double* sigma, const double* kernel_G,
                             void* xi, double* M, double* e_x, int32_t* status,
                             hipStream_t stream);

/* Exchange-only PT-IM step with the projector and the occupation matrix
 * (Sec. II-A: the scheme of Eq. 6 at the midpoints of Eq. 4 with the
 * projector P~ of Eq. 5, H reduced to alpha * V_ACE (Eq. 8, Eq. 14), iterated
 * as the fixed point x = T(x) of Eq. 7 from x^(0) = (Phi_n, sigma_n)):
 *   Phi_mid = (Phi_n + Phi^(k))/2,  sigma_mid = (sigma_n + sigma^(k))/2,
 *   Y = V_ACE Phi_mid,  S = dV Phi_mid^H Phi_mid,  Hm = dV Phi_mid^H Y
 *   (with V_ACE = -xi dV xi^H, Hm = -C^H C for C = dV xi^H Phi_mid, which
 *   the application of V_ACE forms anyway: Hm costs an n_phi x n_phi product
 *   over n instead of a contraction over the grid, and is Hermitian),
 *   Phi^(k+1)   = Phi_n   - i dt_alpha (Y - Phi_mid S^{-1} Hm),
 *   sigma^(k+1) = sigma_n - i dt_alpha (Hm sigma_mid - sigma_mid Hm),
 * for k = 0 .. n_iter-1 (n_iter <= 64), dt_alpha = dt * alpha.  Orbital
 * contractions in the form's precision (C and S with FP64 results); Hm,
 * S^{-1} Hm (Cholesky of S, U = L^{-H}, X = U U^H Hm), the sigma algebra and
 * the residuals in FP64.
 * xi [n][N_g], phi_n and phi_out [n_phi][N_g] (element type of prec);
 * sigma_n, sigma_out complex128 [n_phi][n_phi]; residuals float64
 * [2][n_iter]: R_Phi,k = ||Phi^(k+1) - Phi^(k)||_F / ||Phi^(k+1)||_F in
 * residuals[k], the same for sigma in residuals[n_iter + k].  status (device
 * int32, required): 0, or the 1-based column where the Cholesky factorisation
 * of an overlap S broke down (Phi_mid linearly dependent; results undefined;
 * px_sync returns PX_ERR_NOT_POSITIVE_DEFINITE).  Anderson mixing and the
 * other terms of H are not part of the step.  Workspace: PX_OP_PTIM_STEP
 * with (n, n_phi).  Grids as in px_ace_apply. */
px_status px_ptim_step(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                       const void* xi, int32_t n_phi, const void* phi_n, const double* sigma_n,
                       int32_t n_iter, double dt_alpha, void* phi_out, double* sigma_out,
                       double* residuals, int32_t* status, hipStream_t stream);

/* Hermitian pair symmetry of the ACE build (default on).  With Phi = Psi and a
 * real even kernel, v_ji = conj(v_ij): the orbitals are cut into square blocks,
 * only blocks J <= I are transformed, and a diagonal block only for its pairs
 * j <= i; the real-space v_ij is kept and a streaming pass adds the transposed
 * contribution -f_i psi_i conj(v_ij) to W_j for j < i.  Every unordered pair
 * is solved once (N (N + 1) / 2 pair solves instead of N^2). */
px_status px_set_symmetry(px_context* ctx, int32_t enable);

/* Measurement mode.  When enabled, px_exchange_apply and px_ace_build record
 * HIP events on their stream around pass 1 (pair product + forward xy
 * transforms), pass 2 (z transforms + kernel multiply) and pass 3 (inverse xy
 * transforms + weighted accumulation) of every pair chunk, and synchronise on
 * the last event before returning (the only host synchronisation outside
 * px_sync).  Off by default. */
px_status px_set_profiling(px_context* ctx, int32_t enable);

/* Totals since the last reset, per pass k = 0..3 (arrays of 4): ms[k] summed
 * event time (pass 4: the time from the end of pass 3 to the end of the
 * chunk, which is the transposed accumulation), bytes[k] algorithmic HBM
 * bytes of the 6 * N_g * b pair model (b = element size), 2 * N_g * b per
 * solved pair in each of passes 1-3: pass 1 reads psi_j and writes the pair
 * slab, pass 2 reads and rewrites it, pass 3 reads it and psi_j.  The
 * Hermitian-pair mode keeps v_ij outside that model: pass 3 also writes it
 * (N_g * b per solved pair, not counted in bytes[2]) and pass 4 reads it back,
 * bytes[3] = N_g * b per pair below the diagonal.  launches[k] kernel
 * launches.  reset != 0 zeroes the totals. */
px_status px_profile_read(px_context* ctx, double* ms, double* bytes, int64_t* launches,
                          int32_t reset);

/* Stage times of the ACE builds (px_ace_build) made while profiling was on,
 * since the last reset (Sec. IV-A-2, Eq. (14)), ms an array of 4: ms[0] the
 * contraction M = dV Psi^H W, ms[1] the factorisation (Hermitising, Cholesky
 * of -M and U = L^{-H}), ms[2] the contraction xi = W U, ms[3] the whole
 * build from its first enqueued work (W = Vx Psi) to its last; *calls the
 * number of builds.  The passes of the pair pipeline are in px_profile_read.
 * Each profiled build synchronises on its last event.  reset != 0 zeroes. */
px_status px_profile_read_ace(px_context* ctx, double* ms, int64_t* calls, int32_t reset);

/* One instance of the batched form: the exchange operator of an orbital block
 * applied to the same block (Phi = Psi), optionally followed by its ACE
 * construction.  Arrays as in px_exchange_apply / px_ace_build, element type
 * of the call's precision. */
typedef struct {
  px_cell cell;
  int32_t n;               /* orbitals */
  const void* psi;         /* [n][N_g] */
  const double* occ;       /* [n] */
  const double* kernel_G;  /* [N_g] FP64 */
  void* out;               /* Vx psi (ace == 0) or xi (ace != 0), [n][N_g] */
  double* e_x;             /* nullable: exchange energy */
  double* M;               /* nullable, ace only: Hermitised M, complex128 [n][n] */
  int32_t* status;         /* ace only, required: Cholesky status word */
} px_instance;

/* Workspace for px_exchange_apply_batched with these instances (0 if invalid). */
size_t px_workspace_bytes_batched(const px_context* ctx, int32_t n_inst, const px_instance* inst,
                                  px_precision prec, int32_t ace);

/* Batched form (Sec. III-B(b) batches pairs to fill the GPU): all block pairs
 * of all instances (Hermitian-pair mode, always on here, so every kernel_G
 * must be real and even, K(G) = K(-G); square blocks from the tuning) are
 * grouped by grid and scheduled by block diagonal, so each pass runs as
 * one launch over a task table for many chunks of many instances; then the
 * per-instance energies and, with ace != 0, the ACE construction.  In ACE
 * mode the instances whose last chunk ran in one wave form a group whose
 * tail (Gram matrices, one factorisation launch sequence for the whole
 * group, xi) runs on one of two side streams of the context while `stream`
 * goes on with the next waves; `stream` waits for both before the call's
 * work ends.  The whole call is captured once into a HIP graph and replayed
 * while the instance descriptors, the workspace and the tuning stay the same
 * (rebuilding it synchronises `stream` once).  Results equal those of
 * per-instance px_exchange_apply / px_ace_build calls up to summation order.
 * Calls on one context must not overlap (they share the side streams and the
 * workspace). */
px_status px_exchange_apply_batched(px_context* ctx, int32_t n_inst, const px_instance* inst,
                                    px_precision prec, int32_t ace, hipStream_t stream);

/* Pair-buffer bytes of one wave of the batched form (0 = default 4 GiB). */
px_status px_set_batch_capacity(px_context* ctx, size_t pair_buffer_bytes);

/* Graph capture of the batched form on (default) or off (direct enqueue). */
px_status px_set_graph(px_context* ctx, int32_t enable);

/* Autotuner: times the Hermitian-pair pipeline on this instance (Phi = Psi)
 * for square pair blocks B in {16, 24, 32, 48, 64, 96, 128, 192, 256} (up to
 * the first B >= n, which solves the instance as one triangular block) that
 * fit the attached workspace, each with both compiled
 * configurations of pass 2 (the z transforms: its workgroup shape, x-sections
 * per plane and threads, fixed per grid size at compile time; one
 * configuration on the non-cubic grids), keeps the
 * fastest pair as the context's tuning for this grid and precision, writes B
 * to *best_block (nullable) and appends a JSON line (block, "p2"
 * configuration, per-candidate times) to cache_path (nullable).
 * Synchronises `stream`; `out` receives Vx psi. */
px_status px_autotune(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                      const void* psi, const double* occ, const double* kernel_G, void* out,
                      const char* cache_path, int32_t* best_block, hipStream_t stream);

/* Applies the tuning lines of a px_autotune cache file (last entry per grid
 * and precision wins); *applied (nullable) receives the number of lines used. */
px_status px_load_tuning(px_context* ctx, const char* cache_path, int32_t* applied);

/* Synchronises `stream`, then reads the status word(s) of the last call on
 * this context that reports through one: PX_ERR_NOT_POSITIVE_DEFINITE if an
 * ACE build reported a breakdown, PX_ERR_NOT_CONVERGED if a diagonalisation of
 * sigma did not converge (the error stays latched until px_clear_error),
 * PX_ERR_DEVICE on a HIP error. */
px_status px_sync(px_context* ctx, hipStream_t stream);

/* Clears a latched error. */
void px_clear_error(px_context* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PX_H_ */
