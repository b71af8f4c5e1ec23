// Host side of libpx: argument validation, workspace carving and the
// stream-ordered orchestration of the exchange and ACE kernels.  No call here
// allocates device memory or synchronises the host, except px_sync.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/px.h"
#include <cstdint>

#include "px_internal.hpp"
#include "density_fine.hpp"

struct px_context {
  int device = 0;
  std::string err = "";
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // device status words of the last calls that report through one: the
  // error each stands for when non-zero (a Cholesky breakdown, or no
  // convergence of the occupation-matrix diagonalisation) and what it belongs to
  struct StatusWord {
    int32_t* word;
    px_status kind;
    std::string what;
  };
  std::vector<StatusWord> last_status;
  int latched = PX_OK;
  // (n0,n1,n2,prec) -> pair chunk ic x jc and the pass-2 configuration (0, 1)
  std::map<std::tuple<int, int, int, int>, std::tuple<int, int, int>> tuning;
  // measurement mode: HIP events around each pass of each chunk
  bool profiling = false;
  std::vector<hipEvent_t> events;
  double prof_ms[4] = {0, 0, 0, 0};
  double prof_bytes[4] = {0, 0, 0, 0};
  int64_t prof_launches[4] = {0, 0, 0, 0};
  // ACE build stages: start of the build, start of M, after M, after the
  // factorisation, after xi
  hipEvent_t ace_events[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double ace_ms[4] = {0, 0, 0, 0};
  int64_t ace_calls = 0;
  bool symmetric_ace = true;  // ACE build solves only pairs j <= i (block level)
  bool tri_diag = true;       // ... and within the diagonal blocks (pair level)
  // batched form: the graph of the last batched call, replayed while the call
  // signature (instances, pointers, workspace) stays the same
  bool use_graph = true;
  size_t batch_cap_bytes = size_t(4) << 30;  // pair buffer of one wave
  std::vector<unsigned char> graph_key;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  void* pinned_tasks = nullptr;  // host copy of the task and job tables (page-locked)
  size_t pinned_bytes = 0;
  // ACE tails of the batched form (Gram matrix, factorisation, xi) run on
  // side streams beside the later pair-pipeline waves
  static constexpr int kTailLanes = 2;
  hipStream_t lanes[kTailLanes] = {nullptr, nullptr};
  hipEvent_t lane_done[kTailLanes] = {nullptr, nullptr};
  std::vector<hipEvent_t> fork_events;
  ~px_context() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (hipEvent_t e : ace_events)
      if (e) (void)hipEventDestroy(e);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (pinned_tasks) (void)hipHostFree(pinned_tasks);
    for (int l = 0; l < kTailLanes; ++l) {
      if (lanes[l]) (void)hipStreamDestroy(lanes[l]);
      if (lane_done[l]) (void)hipEventDestroy(lane_done[l]);
    }
    for (hipEvent_t e : fork_events) (void)hipEventDestroy(e);
  }
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

px_status fail(px_context* c, px_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
px_status fail(px_context* c, px_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

px_status hip_check(px_context* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return PX_OK;
  return fail(c, PX_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool cell_ok(const px_cell* cell) {
  if (!cell) return false;
  for (int a = 0; a < 3; ++a)
    if (!(cell->L[a] > 0.0) || cell->n[a] <= 0) return false;
  return true;
}

size_t ngrid(const px_cell* c) { return size_t(c->n[0]) * c->n[1] * c->n[2]; }
// Orbital blocks are read with 16-byte vector loads.
bool misaligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) != 0; }
size_t elem_bytes(px_precision p) { return p == PX_PREC_FP32 ? 8 : 16; }

void default_tuning(const px_cell* cell, px_precision prec, int* ic, int* jc) {
  // ic output orbitals x jc density orbitals per chunk.  Pass 1 and 3 launch
  // n2 * ic workgroups and loop over jc pairs each; larger chunks amortise the
  // phi slab and the output read-modify-write (measured best near 32 x 16 at
  // 72^3 in both precisions).  The pair buffer holds ic*jc slabs.
  (void)cell;
  (void)prec;
  *ic = 32;
  *jc = 16;
}

void tuning_for(const px_context* c, const px_cell* cell, px_precision prec, int* ic, int* jc,
                int* p2 = nullptr) {
  auto it = c->tuning.find({cell->n[0], cell->n[1], cell->n[2], int(prec)});
  if (it != c->tuning.end()) {
    *ic = std::get<0>(it->second);
    *jc = std::get<1>(it->second);
    if (p2) *p2 = std::get<2>(it->second);
  } else {
    default_tuning(cell, prec, ic, jc);
    if (p2) *p2 = 0;
  }
}

// Workspace layout of one exchange application.
struct ExLayout {
  size_t t, g0, expart, S, k32, end;
};

ExLayout ex_layout(const px_cell* cell, px_precision prec, int n_psi, int n_phi, int ic, int jc,
                   bool energy, int p2 = 0) {
  ExLayout l{};
  const int icc = ic < n_phi ? ic : n_phi, jcc = jc < n_psi ? jc : n_psi;
  const size_t pairs = size_t(icc) * jcc;
  size_t off = 0;
  l.t = off;
  off = align_up(off + pairs * ngrid(cell) * elem_bytes(prec));
  l.g0 = off;
  if (prec == PX_PREC_FP32) off = align_up(off + pairs * cell->n[2] * sizeof(px::G0Part));
  l.expart = off;
  l.S = off;
  if (energy) {
    const size_t slots = size_t(cell->n[1]) * px::pass2_sections_grid(prec == PX_PREC_FP32, cell->n, p2);
    off = align_up(off + pairs * slots * 8 * (prec == PX_PREC_FP32 ? 3 : 1));
    l.S = off;
    off = align_up(off + size_t(n_phi) * n_psi * 8);
  }
  l.k32 = off;
  if (prec == PX_PREC_FP32) off = align_up(off + ngrid(cell) * sizeof(float));
  l.end = off;
  return l;
}

struct AceLayout {
  ExLayout ex;
  size_t W, M, L, U, dinv, part, end;
};

AceLayout ace_layout(const px_cell* cell, px_precision prec, int n, int ic, int jc,
                     bool symmetric, int p2 = 0) {
  AceLayout a{};
  if (symmetric) ic = jc = (ic > jc ? ic : jc);
  a.ex = ex_layout(cell, prec, n, n, ic, jc, true, p2);
  size_t off = a.ex.end;
  a.W = off;
  off = align_up(off + size_t(n) * ngrid(cell) * elem_bytes(prec));
  a.M = off;
  off = align_up(off + size_t(n) * n * 16);
  a.L = off;
  off = align_up(off + size_t(n) * n * 16);
  a.U = off;
  off = align_up(off + size_t(n) * n * 16);
  a.dinv = off;
  off = align_up(off + px::chol_dinv_bytes(n));
  int nsplit = 0;
  const size_t pe = px::gemm_xhy_part_elems(n, n, ngrid(cell), &nsplit);
  a.part = off;
  off = align_up(off + pe * 16);
  a.end = off;
  return a;
}

struct ApplyLayout {
  size_t C, C32, part, end;
};

ApplyLayout apply_layout(const px_cell* cell, int n, int n_phi) {
  ApplyLayout a{};
  size_t off = 0;
  a.C = off;
  off = align_up(off + size_t(n) * n_phi * 16);
  a.C32 = off;  // C rounded to complex64, the operand of the FP32 form's xi C
  off = align_up(off + size_t(n) * n_phi * 8);
  int nsplit = 0;
  const size_t pe = px::gemm_xhy_part_elems(n, n_phi, ngrid(cell), &nsplit);
  a.part = off;
  off = align_up(off + pe * 16);
  a.end = off;
  return a;
}

struct LoopLayout {
  ApplyLayout ap;
  size_t mid, buf0, buf1, partial, end;
};

LoopLayout loop_layout(const px_cell* cell, px_precision prec, int n, int n_phi) {
  LoopLayout l{};
  l.ap = apply_layout(cell, n, n_phi);
  size_t off = l.ap.end;
  const size_t blk = size_t(n_phi) * ngrid(cell) * elem_bytes(prec);
  l.mid = off;  // the midpoint, then V_ACE of it (xi^H mid is taken before it is overwritten)
  off = align_up(off + blk);
  l.buf0 = off;
  off = align_up(off + blk);
  l.buf1 = off;
  off = align_up(off + blk);
  l.partial = off;
  off = align_up(off + size_t(px::ptim_update_blocks()) * 16);
  l.end = off;
  return l;
}

// Maximum Jacobi sweeps of the occupation-matrix diagonalisation.  The
// method converges quadratically only once the off-diagonal norm is below the
// gaps between distinct eigenvalues; Fermi-Dirac spectra hold eigenvalues
// exponentially close to 0 and 1, and then the off-diagonal norm first falls
// by a factor of only 2-3 per sweep (n = 512 at kT = 0.02 Ha: 21 sweeps).
// Sweeps after convergence cost one no-op launch pair per round.
constexpr int kEigSweeps = 40;
// Most fixed-point iterations of one px_ptim_step call.
constexpr int kStepMaxIter = 64;

// Workspace of the sigma front end from `base` on: the Jacobi work arrays,
// Q (complex128) and its complex64 copy, d, and the rotated orbital block
// phi = Phi Q (element type of the form; omitted with no_phi).
struct SigmaLayout {
  size_t eig, Q, Q32, d, phi, end;
};

SigmaLayout sigma_layout(size_t base, const px_cell* cell, px_precision prec, int n, bool no_phi) {
  SigmaLayout l{};
  size_t off = align_up(base);
  l.eig = off;
  off = align_up(off + px::eig_work_bytes(n));
  l.Q = off;
  off = align_up(off + size_t(n) * n * 16);
  l.Q32 = off;
  off = align_up(off + size_t(n) * n * 8);
  l.d = off;
  off = align_up(off + size_t(n) * 8);
  l.phi = off;
  if (!no_phi) off = align_up(off + size_t(n) * ngrid(cell) * elem_bytes(prec));
  l.end = off;
  return l;
}

// Workspace of the exchange-only PT-IM step: the ACE application's pieces
// (C, C32, partials for n x n_phi), partials of the n_phi x n_phi overlaps,
// five orbital blocks (midpoint, V_ACE of it, its projection, two iterates),
// the residual partials, and the n_phi x n_phi FP64 matrices.
struct StepLayout {
  ApplyLayout ap;
  size_t part2, mid, Y, Z, buf0, buf1, partial;
  size_t S, Hm, Mneg, L, U, dinv, T, X, X32, smid, sbuf0, sbuf1, A1, A2, st;
  size_t end;
};

StepLayout step_layout(const px_cell* cell, px_precision prec, int n, int n_phi, int n_iter) {
  StepLayout l{};
  l.ap = apply_layout(cell, n, n_phi);
  size_t off = l.ap.end;
  int nsplit = 0;
  const size_t pe = px::gemm_xhy_part_elems(n_phi, n_phi, ngrid(cell), &nsplit);
  l.part2 = off;
  off = align_up(off + pe * 16);
  const size_t blk = size_t(n_phi) * ngrid(cell) * elem_bytes(prec);
  size_t* blocks[5] = {&l.mid, &l.Y, &l.Z, &l.buf0, &l.buf1};
  for (size_t* b : blocks) {
    *b = off;
    off = align_up(off + blk);
  }
  l.partial = off;
  off = align_up(off + size_t(px::ptim_update_blocks()) * 16);
  const size_t mat = size_t(n_phi) * n_phi * 16;
  size_t* mats[12] = {&l.S, &l.Hm, &l.Mneg, &l.L, &l.U, &l.T, &l.X, &l.smid, &l.sbuf0, &l.sbuf1,
                      &l.A1, &l.A2};
  for (size_t* m : mats) {
    *m = off;
    off = align_up(off + mat);
  }
  l.X32 = off;
  off = align_up(off + mat / 2);
  l.dinv = off;
  off = align_up(off + px::chol_dinv_bytes(n_phi));
  l.st = off;
  off = align_up(off + size_t(n_iter > 0 ? n_iter : 1) * sizeof(int32_t));
  l.end = off;
  return l;
}

// Grids of the fine-grid density: even axes (the interpolation splits the
// Nyquist coefficient) of at most kFineMaxAxis points (a line tile of the
// FP64 form, 32 lines, must stay within 64 KB of LDS).
constexpr int kFineMaxAxis = 120;
bool fine_grid_ok(const px_cell* cell) {
  for (int a = 0; a < 3; ++a)
    if (cell->n[a] % 2 || cell->n[a] > kFineMaxAxis) return false;
  return true;
}

px_status check_grid(px_context* c, const px_cell* cell) {
  if (!cell_ok(cell))
    return fail(c, PX_ERR_INVALID_ARG, "cell: edge lengths must be > 0 and grid sizes > 0");
  if (!px::grid_supported(cell->n[0], cell->n[1], cell->n[2]))
    return fail(c, PX_ERR_UNSUPPORTED_GRID,
                "grid %dx%dx%d has no compiled FFT plan (cubic n in {16,24,32,40,48,60,64,72,80,96}, "
                "or 60x60x90, 60x90x120)",
                cell->n[0], cell->n[1], cell->n[2]);
  return PX_OK;
}

// Grids of the contraction-only entry points (ACE application, PT-IM-style
// loop): any positive grid in the FP64 form; the FP32 form reads two complex64
// values per 16-byte load, so N_g must be even (every orbital of a block then
// stays 16-byte aligned and a load never straddles two orbitals).
px_status check_gemm_grid(px_context* c, const px_cell* cell, px_precision prec) {
  if (!cell_ok(cell))
    return fail(c, PX_ERR_INVALID_ARG, "cell: edge lengths must be > 0 and grid sizes > 0");
  if (prec == PX_PREC_FP32 && ngrid(cell) % 2 != 0)
    return fail(c, PX_ERR_UNSUPPORTED_GRID,
                "grid %dx%dx%d: the FP32 form needs an even number of grid points", cell->n[0],
                cell->n[1], cell->n[2]);
  return PX_OK;
}

px_status need_ws(px_context* c, size_t bytes) {
  if (c->ws == nullptr || c->ws_bytes < bytes)
    return fail(c, PX_ERR_WORKSPACE, "workspace of %zu bytes attached, %zu needed", c->ws_bytes,
                bytes);
  return PX_OK;
}

// Enqueue the pair pipeline; `out` gets Vx phi.  With energy, S[i][j]
// receives sum_G K |rho_ij(G)|^2 per pair.  Symmetric mode (phi is psi): the
// orbitals are cut into square blocks of B = max(ic, jc); only blocks J <= I
// are solved, and for J < I pass 3 keeps v_ij so that pass 4 adds the
// transposed contributions to the J block (v_ji = conj(v_ij)).  A diagonal
// block J = I is solved as its lower triangle j <= i (pass 4 adds the pairs
// j < i), so every unordered pair is solved once.
px_status run_exchange(px_context* c, const px_cell* cell, px_precision prec, int n_psi,
                       const void* psi, const double* occ, int n_phi, const void* phi,
                       const double* kern, void* out, const ExLayout& l, bool energy, int ic,
                       int jc, bool symmetric, hipStream_t s, int p2 = 0) {
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t ng = ngrid(cell);
  px::ChunkArgs a{};
  a.psi = psi;
  a.phi = phi;
  a.t = c->ws + l.t;
  a.out = out;
  a.occ = occ;
  a.kern = kern;
  if (fp32) {
    // the FP32 form multiplies by K(G) rounded to FP32 (K(0) stays FP64)
    float* k32 = reinterpret_cast<float*>(c->ws + l.k32);
    px_status st = hip_check(c, px::launch_convert_f64_f32(ng, kern, k32, s), "kernel to FP32");
    if (st != PX_OK) return st;
    a.kern32 = k32;
  }
  a.g0 = reinterpret_cast<px::G0Part*>(c->ws + l.g0);
  a.expart = reinterpret_cast<double*>(c->ws + l.expart);
  a.n2 = cell->n[2];
  a.inv_ng = 1.0 / double(ng);
  double* S = reinterpret_cast<double*>(c->ws + l.S);
  if (symmetric) ic = jc = (ic > jc ? ic : jc);
  const size_t nch = size_t((n_phi + ic - 1) / ic) * ((n_psi + jc - 1) / jc);
  if (c->profiling) {
    while (c->events.size() < nch * 5) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return fail(c, PX_ERR_DEVICE, "hipEventCreate failed");
      c->events.push_back(e);
    }
  }
  const double pair_bytes = double(ng * elem_bytes(prec));
  size_t nchunks = 0;
  std::vector<int> has4;
  for (int i0 = 0; i0 < n_phi; i0 += ic) {
    a.i0 = i0;
    a.ic = (n_phi - i0) < ic ? (n_phi - i0) : ic;
    for (int j0 = 0; j0 < n_psi; j0 += jc) {
      if (symmetric && j0 > i0) break;
      a.j0 = j0;
      a.jc = (n_psi - j0) < jc ? (n_psi - j0) : jc;
      a.first = j0 == 0;
      // a diagonal block is solved as its lower triangle and keeps v_ij for
      // the transposed pass like the blocks below it
      a.tri = symmetric && c->tri_diag && j0 == i0 && a.ic == a.jc;
      a.store_v = symmetric && (j0 < i0 || a.tri);
      const int npairs = px::chunk_pairs(a);
      hipEvent_t* ev = c->profiling ? &c->events[5 * nchunks] : nullptr;
      px_status st = hip_check(
          c, px::launch_chunk(fp32, cell->n, a, npairs, energy, p2, s, ev), "pair pipeline");
      if (st != PX_OK) return st;
      if (a.store_v) {
        st = hip_check(c, px::launch_pass4(fp32, a, ng, s), "transposed accumulation");
        if (st != PX_OK) return st;
      }
      if (c->profiling) {
        (void)hipEventRecord(c->events[5 * nchunks + 4], s);
        // algorithmic bytes of the 6 N_g b pair model, 2 N_g b per solved pair
        // in each pass (pass 1: read psi_j, write the pair slab; pass 2: read
        // and rewrite it; pass 3: read it and psi_j).  The symmetric mode's
        // kept v_ij is outside the model: pass 3 writes it (not counted here)
        // and pass 4 reads it back, N_g b per pair below the diagonal (a
        // triangular block keeps v_ij for its npairs pairs; pass 4 reads the
        // npairs - ic of them below the diagonal)
        const double np = double(npairs), np4 = a.tri ? double(npairs - a.ic) : np;
        for (int k = 0; k < 3; ++k) {
          c->prof_bytes[k] += 2.0 * pair_bytes * np;
          c->prof_launches[k] += 1;
        }
        if (a.store_v) {
          c->prof_bytes[3] += pair_bytes * np4;
          c->prof_launches[3] += 1;
        }
        has4.push_back(a.store_v);
      }
      ++nchunks;
      if (energy) {
        st = hip_check(c, px::launch_expart_reduce(a.expart, fp32 ? a.g0 : nullptr,
                                                   cell->n[1] * px::pass2_sections_grid(fp32, cell->n, p2),
                                                   cell->n[2], double(ng), i0, a.ic, j0, a.jc, S,
                                                   n_psi, a.store_v != 0, a.tri != 0, s),
                       "energy partials");
        if (st != PX_OK) return st;
      }
    }
  }
  if (c->profiling && nchunks > 0) {
    hipError_t e = hipEventSynchronize(c->events[5 * nchunks - 1]);
    if (e != hipSuccess) return hip_check(c, e, "profiling sync");
    for (size_t k = 0; k < nchunks; ++k) {
      for (int p = 0; p < 3; ++p) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, c->events[5 * k + p], c->events[5 * k + p + 1]);
        if (e != hipSuccess) return hip_check(c, e, "hipEventElapsedTime");
        c->prof_ms[p] += ms;
      }
      if (has4[k]) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, c->events[5 * k + 3], c->events[5 * k + 4]);
        if (e != hipSuccess) return hip_check(c, e, "hipEventElapsedTime");
        c->prof_ms[3] += ms;
      }
    }
  }
  return PX_OK;
}

}  // namespace

extern "C" {

int32_t px_abi_version(void) { return PX_ABI_VERSION; }

px_status px_create(int32_t device, px_context** ctx) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  *ctx = nullptr;
  if (device < 0) return PX_ERR_INVALID_ARG;
  // No HIP call here: a context can validate arguments on a machine without
  // a GPU.  The device is selected (and checked) by the first compute call.
  px_context* c = new px_context();
  c->device = device;
  *ctx = c;
  return PX_OK;
}

void px_destroy(px_context* ctx) { delete ctx; }

const char* px_last_error(const px_context* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

int32_t px_grid_supported(const px_cell* cell, px_precision prec) {
  (void)prec;
  return cell_ok(cell) && px::grid_supported(cell->n[0], cell->n[1], cell->n[2]) ? 1 : 0;
}

size_t px_workspace_bytes(const px_context* ctx, px_op op, const px_cell* cell, px_precision prec,
                          int32_t n_psi, int32_t n_phi) {
  if (!ctx || !cell_ok(cell) || n_psi <= 0) return 0;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32) return 0;
  const bool fft_grid = px::grid_supported(cell->n[0], cell->n[1], cell->n[2]);
  const bool gemm_grid = prec == PX_PREC_FP64 || ngrid(cell) % 2 == 0;
  const bool fft_op = op == PX_OP_EXCHANGE || op == PX_OP_ACE_BUILD || op == PX_OP_EXCHANGE_SIGMA ||
                      op == PX_OP_ACE_BUILD_SIGMA;
  if (fft_op ? !fft_grid : !gemm_grid) return 0;
  int ic, jc, p2;
  tuning_for(ctx, cell, prec, &ic, &jc, &p2);
  switch (op) {
    case PX_OP_EXCHANGE:
      if (n_phi <= 0) return 0;
      return ex_layout(cell, prec, n_psi, n_phi, ic, jc, true, p2).end;
    case PX_OP_ACE_BUILD:
      return ace_layout(cell, prec, n_psi, ic, jc, ctx->symmetric_ace, p2).end;
    case PX_OP_ACE_APPLY:
      if (n_phi <= 0) return 0;
      return apply_layout(cell, n_psi, n_phi).end;
    case PX_OP_PTIM_LOOP:
      if (n_phi <= 0) return 0;
      return loop_layout(cell, prec, n_psi, n_phi).end;
    case PX_OP_EXCHANGE_SIGMA: {
      if (n_phi <= 0) return 0;
      const ExLayout ex = ex_layout(cell, prec, n_psi, n_phi, ic, jc, false, p2);
      return sigma_layout(ex.end, cell, prec, n_psi, false).end;
    }
    case PX_OP_SIGMA_DIAG:
      return align_up(px::eig_work_bytes(n_psi));
    case PX_OP_DENSITY_SIGMA:
      return sigma_layout(0, cell, prec, n_psi, false).end;
    case PX_OP_PTIM_STEP:
      if (n_phi <= 0) return 0;
      return step_layout(cell, prec, n_psi, n_phi, kStepMaxIter).end;
    case PX_OP_ROTATE:  // Q in complex64 (the FP64 form does not use it)
      return align_up(size_t(n_psi) * n_psi * 8);
    case PX_OP_DENSITY_FINE:
      if (!fine_grid_ok(cell)) return 0;
      return align_up(px::density_fine_work_bytes(prec == PX_PREC_FP32, cell->n, n_psi));
    case PX_OP_ACE_BUILD_SIGMA: {
      const AceLayout a = ace_layout(cell, prec, n_psi, ic, jc, ctx->symmetric_ace, p2);
      return sigma_layout(a.end, cell, prec, n_psi, false).end;
    }
  }
  return 0;
}

px_status px_set_workspace(px_context* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(dev_ptr) % kAlign) != 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
  ctx->ws = static_cast<char*>(dev_ptr);
  ctx->ws_bytes = dev_ptr ? bytes : 0;
  return PX_OK;
}

px_status px_set_tuning(px_context* ctx, const px_cell* cell, px_precision prec, int32_t ic,
                        int32_t jc) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (!cell_ok(cell) || ic < 0 || jc < 0 || ic > 4096 || jc > 4096)
    return fail(ctx, PX_ERR_INVALID_ARG, "tuning: need a valid cell and 0 <= ic, jc <= 4096");
  auto key = std::make_tuple(cell->n[0], cell->n[1], cell->n[2], int(prec));
  auto it = ctx->tuning.find(key);
  const int p2 = it != ctx->tuning.end() ? std::get<2>(it->second) : 0;  // kept from px_autotune
  if (ic == 0 || jc == 0) ctx->tuning.erase(key);
  else ctx->tuning[key] = {ic, jc, p2};
  return PX_OK;
}

px_status px_kernel_hse(px_context* ctx, const px_cell* cell, double mu, double* kernel_G,
                        hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (!cell_ok(cell) || !kernel_G || !(mu > 0.0))
    return fail(ctx, PX_ERR_INVALID_ARG, "kernel_hse: need a valid cell, mu > 0, non-null output");
  return hip_check(ctx,
                   px::launch_kernel_hse(cell->n[0], cell->n[1], cell->n[2], cell->L[0],
                                         cell->L[1], cell->L[2], mu, kernel_G, stream),
                   "kernel_hse");
}

px_status px_convert_c128_to_c64(px_context* ctx, size_t n_elems, const void* src, void* dst,
                                 hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (n_elems > 0 && (!src || !dst)) return fail(ctx, PX_ERR_INVALID_ARG, "convert: null pointer");
  if ((reinterpret_cast<uintptr_t>(src) % 32) != 0 || (reinterpret_cast<uintptr_t>(dst) % 16) != 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "convert: src must be 32-byte and dst 16-byte aligned");
  return hip_check(ctx, px::launch_convert_c128_c64(n_elems, src, dst, stream), "convert");
}

px_status px_stream_copy(px_context* ctx, const void* src, void* dst, size_t bytes,
                         hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (bytes > 0 && (!src || !dst)) return fail(ctx, PX_ERR_INVALID_ARG, "stream_copy: null pointer");
  if (bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(src) % 16) != 0 ||
      (reinterpret_cast<uintptr_t>(dst) % 16) != 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "stream_copy: bytes and pointers must be 16-byte multiples");
  return hip_check(ctx, px::launch_stream_copy(bytes, src, dst, stream), "stream_copy");
}

px_status px_exchange_apply(px_context* ctx, const px_cell* cell, px_precision prec,
                            int32_t n_psi, const void* psi, const double* occ, int32_t n_phi,
                            const void* phi, const double* kernel_G, void* vx_phi, double* e_x,
                            hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_grid(ctx, cell);
  if (st != PX_OK) return st;
  if (n_psi <= 0 || n_phi <= 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "n_psi and n_phi must be > 0 (got %d, %d)", n_psi, n_phi);
  if (!psi || !occ || !phi || !kernel_G || !vx_phi)
    return fail(ctx, PX_ERR_INVALID_ARG, "exchange_apply: null array argument");
  if (vx_phi == psi || vx_phi == phi)
    return fail(ctx, PX_ERR_INVALID_ARG, "exchange_apply: vx_phi must not alias psi or phi");
  if (misaligned(psi) || misaligned(phi) || misaligned(vx_phi))
    return fail(ctx, PX_ERR_INVALID_ARG, "exchange_apply: orbital blocks must be 16-byte aligned");
  if (e_x && (phi != psi || n_phi != n_psi))
    return fail(ctx, PX_ERR_INVALID_ARG, "exchange_apply: e_x requires phi == psi and n_phi == n_psi");
  int ic, jc, p2;
  tuning_for(ctx, cell, prec, &ic, &jc, &p2);
  const ExLayout l = ex_layout(cell, prec, n_psi, n_phi, ic, jc, e_x != nullptr, p2);
  st = need_ws(ctx, l.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  st = run_exchange(ctx, cell, prec, n_psi, psi, occ, n_phi, phi, kernel_G, vx_phi, l,
                    e_x != nullptr, ic, jc, false, stream, p2);
  if (st != PX_OK) return st;
  if (e_x) {
    const double ng = double(ngrid(cell));
    const double omega = cell->L[0] * cell->L[1] * cell->L[2];
    st = hip_check(ctx,
                   px::launch_energy(reinterpret_cast<double*>(ctx->ws + l.S), occ, n_psi,
                                     -0.5 * omega / (ng * ng), e_x, stream),
                   "energy");
  }
  return st;
}

}  // extern "C"

namespace {

// The ACE construction of Eq. 14 from orbitals psi with occupations occ, in
// the workspace layout l (validated arguments, device set): W = Vx psi through
// the pair pipeline, M = dV psi^H W, -M = L L^H, U = L^-H, xi = W U; the
// Cholesky breakdown column goes to *status.
px_status ace_build_run(px_context* ctx, const px_cell* cell, px_precision prec, int n,
                        const void* psi, const double* occ, const double* kernel_G, void* xi,
                        double* M, double* e_x, int32_t* status, const AceLayout& l, int ic,
                        int jc, int p2, hipStream_t stream) {
  px_status st = PX_OK;
  hipError_t he = hipSuccess;
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t ng = ngrid(cell);
  const double omega = cell->L[0] * cell->L[1] * cell->L[2];
  const double dV = omega / double(ng);
  hipEvent_t* ev = ctx->ace_events;
  if (ctx->profiling) {
    for (int k = 0; k < 5; ++k)
      if (!ev[k] && hipEventCreate(&ev[k]) != hipSuccess)
        return fail(ctx, PX_ERR_DEVICE, "hipEventCreate failed");
    (void)hipEventRecord(ev[0], stream);
  }
  void* W = ctx->ws + l.W;
  double* Mw = M ? M : reinterpret_cast<double*>(ctx->ws + l.M);
  double* L = reinterpret_cast<double*>(ctx->ws + l.L);
  double* U = reinterpret_cast<double*>(ctx->ws + l.U);
  double* part = reinterpret_cast<double*>(ctx->ws + l.part);
  // W = Vx Psi (pair pipeline) and the energy sums
  st = run_exchange(ctx, cell, prec, n, psi, occ, n, psi, kernel_G, W, l.ex, true, ic, jc,
                    ctx->symmetric_ace, stream, p2);
  if (st != PX_OK) return st;
  if (e_x) {
    st = hip_check(ctx,
                   px::launch_energy(reinterpret_cast<double*>(ctx->ws + l.ex.S), occ, n,
                                     -0.5 * omega / (double(ng) * double(ng)), e_x, stream),
                   "energy");
    if (st != PX_OK) return st;
  }
  int nsplit = 0;
  px::gemm_xhy_part_elems(n, n, ng, &nsplit);
  if (ctx->profiling) (void)hipEventRecord(ev[1], stream);
  // M = dV Psi^H W, Hermitised; -M = L L^H; U = L^{-H}; xi = W U
  // M is Hermitian up to rounding: the tiles above the diagonal are mirrored
  st = hip_check(ctx, px::launch_gemm_xhy_herm(fp32, n, ng, psi, W, dV, Mw, part, nsplit, stream),
                 "M = dV Psi^H W");
  if (st != PX_OK) return st;
  if (ctx->profiling) (void)hipEventRecord(ev[2], stream);
  st = hip_check(ctx, px::launch_hermitize(Mw, n, stream), "hermitize");
  if (st != PX_OK) return st;
  st = hip_check(ctx,
                 px::launch_chol_inv(Mw, n, L, U, status,
                                     reinterpret_cast<double*>(ctx->ws + l.dinv), stream),
                 "cholesky");
  if (st != PX_OK) return st;
  if (ctx->profiling) (void)hipEventRecord(ev[3], stream);
  // FP32 form: U rounded to complex64 into L's place (L is not read again)
  const void* Uc = U;
  if (fp32) {
    st = hip_check(ctx, px::launch_convert_f64_f32(size_t(2) * n * n, U, reinterpret_cast<float*>(L),
                                                   stream),
                   "U to FP32");
    if (st != PX_OK) return st;
    Uc = L;
  }
  st = hip_check(ctx, px::launch_gemm_xc(fp32, n, n, ng, W, Uc, n, 1.0, xi, true, stream),
                 "xi = W L^-H");
  if (st != PX_OK) return st;
  if (ctx->profiling) {
    (void)hipEventRecord(ev[4], stream);
    he = hipEventSynchronize(ev[4]);
    if (he != hipSuccess) return hip_check(ctx, he, "profiling sync");
    for (int k = 0; k < 4; ++k) {
      float ms = 0.f;
      // stages M, factorisation, xi; then the whole build
      he = k < 3 ? hipEventElapsedTime(&ms, ev[k + 1], ev[k + 2]) : hipEventElapsedTime(&ms, ev[0], ev[4]);
      if (he != hipSuccess) return hip_check(ctx, he, "hipEventElapsedTime");
      ctx->ace_ms[k] += ms;
    }
    ctx->ace_calls += 1;
  }
  return PX_OK;
}

}  // namespace

extern "C" {

px_status px_ace_build(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                       const void* psi, const double* occ, const double* kernel_G, void* xi,
                       double* M, double* e_x, int32_t* status, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_grid(ctx, cell);
  if (st != PX_OK) return st;
  if (n <= 0) return fail(ctx, PX_ERR_INVALID_ARG, "n must be > 0 (got %d)", n);
  if (!psi || !occ || !kernel_G || !xi || !status)
    return fail(ctx, PX_ERR_INVALID_ARG, "ace_build: null array argument");
  if (xi == psi) return fail(ctx, PX_ERR_INVALID_ARG, "ace_build: xi must not alias psi");
  if (misaligned(psi) || misaligned(xi))
    return fail(ctx, PX_ERR_INVALID_ARG, "ace_build: orbital blocks must be 16-byte aligned");
  int ic, jc, p2;
  tuning_for(ctx, cell, prec, &ic, &jc, &p2);
  const AceLayout l = ace_layout(cell, prec, n, ic, jc, ctx->symmetric_ace, p2);
  st = need_ws(ctx, l.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  st = ace_build_run(ctx, cell, prec, n, psi, occ, kernel_G, xi, M, e_x, status, l, ic, jc, p2, stream);
  if (st == PX_OK) ctx->last_status.assign(1, {status, PX_ERR_NOT_POSITIVE_DEFINITE, "ace_build: -M"});
  return st;
}

px_status px_ace_apply(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                       const void* xi, int32_t n_phi, const void* phi, void* out,
                       hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_gemm_grid(ctx, cell, prec);
  if (st != PX_OK) return st;
  if (n <= 0 || n_phi <= 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "n and n_phi must be > 0 (got %d, %d)", n, n_phi);
  if (!xi || !phi || !out) return fail(ctx, PX_ERR_INVALID_ARG, "ace_apply: null array argument");
  if (out == phi || out == xi)
    return fail(ctx, PX_ERR_INVALID_ARG, "ace_apply: out must not alias xi or phi");
  if (misaligned(xi) || misaligned(phi) || misaligned(out))
    return fail(ctx, PX_ERR_INVALID_ARG, "ace_apply: orbital blocks must be 16-byte aligned");
  const ApplyLayout l = apply_layout(cell, n, n_phi);
  st = need_ws(ctx, l.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t ng = ngrid(cell);
  const double dV = cell->L[0] * cell->L[1] * cell->L[2] / double(ng);
  double* C = reinterpret_cast<double*>(ctx->ws + l.C);
  float* C32 = fp32 ? reinterpret_cast<float*>(ctx->ws + l.C32) : nullptr;
  double* part = reinterpret_cast<double*>(ctx->ws + l.part);
  int nsplit = 0;
  px::gemm_xhy_part_elems(n, n_phi, ng, &nsplit);
  st = hip_check(ctx, px::launch_gemm_xhy(fp32, n, n_phi, ng, xi, phi, dV, C, n_phi, part, nsplit,
                                          C32, stream),
                 "C = dV xi^H phi");
  if (st != PX_OK) return st;
  const void* Cc = fp32 ? static_cast<const void*>(C32) : C;
  return hip_check(ctx, px::launch_gemm_xc(fp32, n, n_phi, ng, xi, Cc, n_phi, -1.0, out, false, stream),
                   "out = -xi C");
}

px_status px_ptim_exchange_loop(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                                const void* xi, int32_t n_phi, const void* phi_n, int32_t n_iter,
                                double dt_alpha, void* phi_out, double* residuals,
                                hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_gemm_grid(ctx, cell, prec);
  if (st != PX_OK) return st;
  if (n <= 0 || n_phi <= 0 || n_iter <= 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "n, n_phi and n_iter must be > 0");
  if (!xi || !phi_n || !phi_out || !residuals)
    return fail(ctx, PX_ERR_INVALID_ARG, "ptim_exchange_loop: null array argument");
  if (phi_out == phi_n || phi_out == xi)
    return fail(ctx, PX_ERR_INVALID_ARG, "ptim_exchange_loop: phi_out must not alias xi or phi_n");
  if (misaligned(xi) || misaligned(phi_n) || misaligned(phi_out))
    return fail(ctx, PX_ERR_INVALID_ARG,
                "ptim_exchange_loop: orbital blocks must be 16-byte aligned");
  const LoopLayout l = loop_layout(cell, prec, n, n_phi);
  st = need_ws(ctx, l.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t ng = ngrid(cell);
  const size_t nel = size_t(n_phi) * ng;
  const double dV = cell->L[0] * cell->L[1] * cell->L[2] / double(ng);
  double* C = reinterpret_cast<double*>(ctx->ws + l.ap.C);
  float* C32 = fp32 ? reinterpret_cast<float*>(ctx->ws + l.ap.C32) : nullptr;
  const void* Cc = fp32 ? static_cast<const void*>(C32) : C;
  double* part = reinterpret_cast<double*>(ctx->ws + l.ap.part);
  void* mid = ctx->ws + l.mid;
  void* y = mid;
  void* bufs[2] = {ctx->ws + l.buf0, ctx->ws + l.buf1};
  double* partial = reinterpret_cast<double*>(ctx->ws + l.partial);
  int nsplit = 0;
  px::gemm_xhy_part_elems(n, n_phi, ng, &nsplit);
  const void* cur = phi_n;
  for (int k = 0; k < n_iter; ++k) {
    void* nxt = (k == n_iter - 1) ? phi_out : bufs[k & 1];
    st = hip_check(ctx, px::launch_midpoint(fp32, nel, phi_n, cur, mid, stream), "midpoint");
    if (st != PX_OK) return st;
    st = hip_check(ctx, px::launch_gemm_xhy(fp32, n, n_phi, ng, xi, mid, dV, C, n_phi, part,
                                            nsplit, C32, stream),
                   "C = dV xi^H mid");
    if (st != PX_OK) return st;
    st = hip_check(ctx, px::launch_gemm_xc(fp32, n, n_phi, ng, xi, Cc, n_phi, -1.0, y, false, stream),
                   "y = -xi C");
    if (st != PX_OK) return st;
    st = hip_check(ctx, px::launch_ptim_update(fp32, nel, phi_n, y, nullptr, cur, nxt, dt_alpha,
                                               partial, residuals + k, stream),
                   "update");
    if (st != PX_OK) return st;
    cur = nxt;
  }
  return PX_OK;
}

px_status px_sigma_diagonalize(px_context* ctx, int32_t n, const double* sigma, double* Q, double* d,
                               int32_t* status, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (n <= 0) return fail(ctx, PX_ERR_INVALID_ARG, "n must be > 0 (got %d)", n);
  if (!sigma || !Q || !d || !status)
    return fail(ctx, PX_ERR_INVALID_ARG, "sigma_diagonalize: null array argument");
  if (Q == sigma) return fail(ctx, PX_ERR_INVALID_ARG, "sigma_diagonalize: Q must not alias sigma");
  if (misaligned(sigma) || misaligned(Q))
    return fail(ctx, PX_ERR_INVALID_ARG, "sigma_diagonalize: matrices must be 16-byte aligned");
  px_status st = need_ws(ctx, align_up(px::eig_work_bytes(n)));
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  st = hip_check(ctx, px::launch_eig_hermitian(sigma, n, Q, d, status, ctx->ws, kEigSweeps, stream),
                 "sigma = Q D Q^H");
  if (st == PX_OK) ctx->last_status.assign(1, {status, PX_ERR_NOT_CONVERGED, "sigma_diagonalize"});
  return st;
}

}  // extern "C"

namespace {

// sigma = Q D Q^H into the layout's Q and d, then phi = Phi Q (Eq. 11): the
// orbitals of the diagonal form that Eq. 12 and Eq. 13 sum over.
px_status rotate_orbitals(px_context* c, const SigmaLayout& l, const px_cell* cell, px_precision prec,
                          int n, const void* phi_basis, const double* sigma, int32_t* status,
                          hipStream_t s) {
  const bool fp32 = prec == PX_PREC_FP32;
  double* Q = reinterpret_cast<double*>(c->ws + l.Q);
  double* d = reinterpret_cast<double*>(c->ws + l.d);
  px_status st = hip_check(
      c, px::launch_eig_hermitian(sigma, n, Q, d, status, c->ws + l.eig, kEigSweeps, s),
      "sigma = Q D Q^H");
  if (st != PX_OK) return st;
  const void* Qc = Q;
  if (fp32) {  // the FP32 contraction reads Q rounded to complex64
    float* Q32 = reinterpret_cast<float*>(c->ws + l.Q32);
    st = hip_check(c, px::launch_convert_f64_f32(size_t(2) * n * n, Q, Q32, s), "Q to FP32");
    if (st != PX_OK) return st;
    Qc = Q32;
  }
  return hip_check(c, px::launch_gemm_xc(fp32, n, n, ngrid(cell), phi_basis, Qc, n, 1.0,
                                         c->ws + l.phi, false, s),
                   "phi = Phi Q");
}

}  // namespace

extern "C" {

px_status px_exchange_apply_sigma(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                                  const void* phi_basis, const double* sigma, int32_t n_tgt,
                                  const void* tgt, const double* kernel_G, void* vx_tgt,
                                  int32_t* status, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_grid(ctx, cell);
  if (st != PX_OK) return st;
  if (n <= 0 || n_tgt <= 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "n and n_tgt must be > 0 (got %d, %d)", n, n_tgt);
  if (!phi_basis || !sigma || !tgt || !kernel_G || !vx_tgt || !status)
    return fail(ctx, PX_ERR_INVALID_ARG, "exchange_apply_sigma: null array argument");
  if (vx_tgt == phi_basis || vx_tgt == tgt)
    return fail(ctx, PX_ERR_INVALID_ARG, "exchange_apply_sigma: vx_tgt must not alias Phi or tgt");
  if (misaligned(phi_basis) || misaligned(tgt) || misaligned(vx_tgt) || misaligned(sigma))
    return fail(ctx, PX_ERR_INVALID_ARG,
                "exchange_apply_sigma: orbital blocks and sigma must be 16-byte aligned");
  int ic, jc, p2;
  tuning_for(ctx, cell, prec, &ic, &jc, &p2);
  const ExLayout ex = ex_layout(cell, prec, n, n_tgt, ic, jc, false, p2);
  const SigmaLayout sl = sigma_layout(ex.end, cell, prec, n, false);
  st = need_ws(ctx, sl.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  st = rotate_orbitals(ctx, sl, cell, prec, n, phi_basis, sigma, status, stream);
  if (st != PX_OK) return st;
  // Eq. 13 on (phi, d): the double loop over the rotated orbitals
  st = run_exchange(ctx, cell, prec, n, ctx->ws + sl.phi, reinterpret_cast<double*>(ctx->ws + sl.d),
                    n_tgt, tgt, kernel_G, vx_tgt, ex, false, ic, jc, false, stream, p2);
  if (st == PX_OK) ctx->last_status.assign(1, {status, PX_ERR_NOT_CONVERGED, "exchange_apply_sigma"});
  return st;
}

px_status px_density(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                     const void* phi, const double* occ, double* rho, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_gemm_grid(ctx, cell, prec);
  if (st != PX_OK) return st;
  if (n <= 0) return fail(ctx, PX_ERR_INVALID_ARG, "n must be > 0 (got %d)", n);
  if (!phi || !occ || !rho) return fail(ctx, PX_ERR_INVALID_ARG, "density: null array argument");
  if (misaligned(phi) || (reinterpret_cast<uintptr_t>(rho) & 7) != 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "density: phi must be 16-byte and rho 8-byte aligned");
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  return hip_check(ctx, px::launch_density(prec == PX_PREC_FP32, ngrid(cell), n, phi, occ, rho, stream),
                   "density");
}

px_status px_density_fine(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                          const void* phi, const double* occ, double* rho_fine, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  if (!cell_ok(cell))
    return fail(ctx, PX_ERR_INVALID_ARG, "cell: edge lengths must be > 0 and grid sizes > 0");
  if (!fine_grid_ok(cell))
    return fail(ctx, PX_ERR_UNSUPPORTED_GRID, "density_fine: grid %dx%dx%d needs even axes of at most %d",
                cell->n[0], cell->n[1], cell->n[2], kFineMaxAxis);
  if (n <= 0) return fail(ctx, PX_ERR_INVALID_ARG, "n must be > 0 (got %d)", n);
  if (!phi || !occ || !rho_fine) return fail(ctx, PX_ERR_INVALID_ARG, "density_fine: null array argument");
  if (misaligned(phi) || (reinterpret_cast<uintptr_t>(rho_fine) & 7) != 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "density_fine: phi must be 16-byte and rho 8-byte aligned");
  const bool fp32 = prec == PX_PREC_FP32;
  px_status st = need_ws(ctx, align_up(px::density_fine_work_bytes(fp32, cell->n, n)));
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  return hip_check(ctx, px::launch_density_fine(fp32, cell->n, n, phi, occ, rho_fine, ctx->ws, stream),
                   "density on the fine grid");
}

px_status px_density_sigma(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                           const void* phi_basis, const double* sigma, double* rho, int32_t* status,
                           hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_gemm_grid(ctx, cell, prec);
  if (st != PX_OK) return st;
  if (n <= 0) return fail(ctx, PX_ERR_INVALID_ARG, "n must be > 0 (got %d)", n);
  if (!phi_basis || !sigma || !rho || !status)
    return fail(ctx, PX_ERR_INVALID_ARG, "density_sigma: null array argument");
  if (misaligned(phi_basis) || misaligned(sigma) || (reinterpret_cast<uintptr_t>(rho) & 7) != 0)
    return fail(ctx, PX_ERR_INVALID_ARG,
                "density_sigma: Phi and sigma must be 16-byte and rho 8-byte aligned");
  const SigmaLayout sl = sigma_layout(0, cell, prec, n, false);
  st = need_ws(ctx, sl.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  st = rotate_orbitals(ctx, sl, cell, prec, n, phi_basis, sigma, status, stream);
  if (st != PX_OK) return st;
  st = hip_check(ctx, px::launch_density(prec == PX_PREC_FP32, ngrid(cell), n, ctx->ws + sl.phi,
                                         reinterpret_cast<double*>(ctx->ws + sl.d), rho, stream),
                 "density");
  if (st == PX_OK) ctx->last_status.assign(1, {status, PX_ERR_NOT_CONVERGED, "density_sigma"});
  return st;
}

px_status px_rotate_orbitals(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                             const void* phi_basis, const double* Q, void* phi_out, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_gemm_grid(ctx, cell, prec);
  if (st != PX_OK) return st;
  if (n <= 0) return fail(ctx, PX_ERR_INVALID_ARG, "n must be > 0 (got %d)", n);
  if (!phi_basis || !Q || !phi_out) return fail(ctx, PX_ERR_INVALID_ARG, "rotate_orbitals: null array argument");
  if (phi_out == phi_basis)
    return fail(ctx, PX_ERR_INVALID_ARG, "rotate_orbitals: phi_out must not alias Phi");
  if (misaligned(phi_basis) || misaligned(Q) || misaligned(phi_out))
    return fail(ctx, PX_ERR_INVALID_ARG, "rotate_orbitals: arrays must be 16-byte aligned");
  const bool fp32 = prec == PX_PREC_FP32;
  if (fp32) {
    st = need_ws(ctx, align_up(size_t(n) * n * 8));
    if (st != PX_OK) return st;
  }
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  const void* Qc = Q;
  if (fp32) {  // the FP32 contraction reads Q rounded to complex64
    st = hip_check(ctx, px::launch_convert_f64_f32(size_t(2) * n * n, Q, reinterpret_cast<float*>(ctx->ws),
                                                   stream),
                   "Q to FP32");
    if (st != PX_OK) return st;
    Qc = ctx->ws;
  }
  return hip_check(ctx, px::launch_gemm_xc(fp32, n, n, ngrid(cell), phi_basis, Qc, n, 1.0, phi_out, false,
                                           stream),
                   "phi = Phi Q");
}

px_status px_ace_build_sigma(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                             const void* phi_basis, const double* sigma, const double* kernel_G,
                             void* xi, double* M, double* e_x, int32_t* status,
                             hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_grid(ctx, cell);
  if (st != PX_OK) return st;
  if (n <= 0) return fail(ctx, PX_ERR_INVALID_ARG, "n must be > 0 (got %d)", n);
  if (!phi_basis || !sigma || !kernel_G || !xi || !status)
    return fail(ctx, PX_ERR_INVALID_ARG, "ace_build_sigma: null array argument");
  if (xi == phi_basis) return fail(ctx, PX_ERR_INVALID_ARG, "ace_build_sigma: xi must not alias Phi");
  if (misaligned(phi_basis) || misaligned(xi) || misaligned(sigma))
    return fail(ctx, PX_ERR_INVALID_ARG,
                "ace_build_sigma: orbital blocks and sigma must be 16-byte aligned");
  int ic, jc, p2;
  tuning_for(ctx, cell, prec, &ic, &jc, &p2);
  const AceLayout l = ace_layout(cell, prec, n, ic, jc, ctx->symmetric_ace, p2);
  const SigmaLayout sl = sigma_layout(l.end, cell, prec, n, false);
  st = need_ws(ctx, sl.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  // sigma = Q D Q^H and phi = Phi Q (Eq. 11); then Eq. 14 on (phi, d), which
  // span the same space as Phi, so V_ACE is exact on span(Phi)
  st = rotate_orbitals(ctx, sl, cell, prec, n, phi_basis, sigma, status, stream);
  if (st != PX_OK) return st;
  st = ace_build_run(ctx, cell, prec, n, ctx->ws + sl.phi, reinterpret_cast<double*>(ctx->ws + sl.d),
                     kernel_G, xi, M, e_x, status + 1, l, ic, jc, p2, stream);
  if (st == PX_OK)
    ctx->last_status = {{status, PX_ERR_NOT_CONVERGED, "ace_build_sigma"},
                        {status + 1, PX_ERR_NOT_POSITIVE_DEFINITE, "ace_build_sigma: -M"}};
  return st;
}

px_status px_ptim_step(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                       const void* xi, int32_t n_phi, const void* phi_n, const double* sigma_n,
                       int32_t n_iter, double dt_alpha, void* phi_out, double* sigma_out,
                       double* residuals, int32_t* status, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_gemm_grid(ctx, cell, prec);
  if (st != PX_OK) return st;
  if (n <= 0 || n_phi <= 0 || n_iter <= 0 || n_iter > kStepMaxIter)
    return fail(ctx, PX_ERR_INVALID_ARG, "n, n_phi > 0 and 0 < n_iter <= %d needed", kStepMaxIter);
  if (!xi || !phi_n || !sigma_n || !phi_out || !sigma_out || !residuals || !status)
    return fail(ctx, PX_ERR_INVALID_ARG, "ptim_step: null array argument");
  if (phi_out == phi_n || phi_out == xi || sigma_out == sigma_n)
    return fail(ctx, PX_ERR_INVALID_ARG, "ptim_step: outputs must not alias the inputs");
  if (misaligned(xi) || misaligned(phi_n) || misaligned(phi_out) || misaligned(sigma_n) ||
      misaligned(sigma_out))
    return fail(ctx, PX_ERR_INVALID_ARG, "ptim_step: arrays must be 16-byte aligned");
  const StepLayout l = step_layout(cell, prec, n, n_phi, kStepMaxIter);
  st = need_ws(ctx, l.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t ng = ngrid(cell);
  const size_t nel = size_t(n_phi) * ng;
  const double dV = cell->L[0] * cell->L[1] * cell->L[2] / double(ng);
  char* w = ctx->ws;
  auto D = [w](size_t off) { return reinterpret_cast<double*>(w + off); };
  double* C = D(l.ap.C);
  float* C32 = fp32 ? reinterpret_cast<float*>(w + l.ap.C32) : nullptr;
  const void* Cc = fp32 ? static_cast<const void*>(C32) : C;
  float* X32 = reinterpret_cast<float*>(w + l.X32);
  const void* Xc = fp32 ? static_cast<const void*>(X32) : D(l.X);
  int32_t* sts = reinterpret_cast<int32_t*>(w + l.st);
  int ns1 = 0, ns2 = 0;
  px::gemm_xhy_part_elems(n, n_phi, ng, &ns1);
  px::gemm_xhy_part_elems(n_phi, n_phi, ng, &ns2);
  void* pbufs[2] = {w + l.buf0, w + l.buf1};
  double* sbufs[2] = {D(l.sbuf0), D(l.sbuf1)};
  const void* cur_p = phi_n;
  const double* cur_s = sigma_n;
  auto ok = [&](hipError_t e, const char* what) { return hip_check(ctx, e, what); };
  for (int k = 0; k < n_iter; ++k) {
    const bool last = k == n_iter - 1;
    void* nxt_p = last ? phi_out : pbufs[k & 1];
    double* nxt_s = last ? sigma_out : sbufs[k & 1];
    void* mid = w + l.mid;
    // Eq. 4: midpoints
    if ((st = ok(px::launch_midpoint(fp32, nel, phi_n, cur_p, mid, stream), "midpoint")) != PX_OK) return st;
    // Y = V_ACE mid = -xi (dV xi^H mid) (Eq. 14; alpha is folded into dt_alpha)
    if ((st = ok(px::launch_gemm_xhy(fp32, n, n_phi, ng, xi, mid, dV, C, n_phi, D(l.ap.part), ns1, C32,
                                     stream), "C = dV xi^H mid")) != PX_OK) return st;
    if ((st = ok(px::launch_gemm_xc(fp32, n, n_phi, ng, xi, Cc, n_phi, -1.0, w + l.Y, false, stream),
                 "Y = -xi C")) != PX_OK) return st;
    // S = dV mid^H mid (Eq. 5; Hermitian: upper tiles, mirrored).  Eq. 6's
    // Phi^* H Phi with H = V_ACE: dV mid^H Y = -dV mid^H xi C = -C^H C, an
    // n_phi x n_phi product over the rank of xi from the FP64 C already formed
    // (exactly Hermitian; Hermitised anyway so that the commutator keeps sigma
    // Hermitian to the last bit)
    if ((st = ok(px::launch_gemm_xhy_herm(fp32, n_phi, ng, mid, mid, dV, D(l.S), D(l.part2), ns2, stream),
                 "S = dV mid^H mid")) != PX_OK) return st;
    if ((st = ok(px::launch_zgemm_gen(true, n_phi, n_phi, n, C, n_phi, C, n_phi, D(l.Hm), n_phi, -1.0,
                                      stream), "Hm = -C^H C")) != PX_OK) return st;
    if ((st = ok(px::launch_hermitize(D(l.Hm), n_phi, stream), "hermitize Hm")) != PX_OK) return st;
    // X = S^{-1} Hm in FP64: S = L L^H (the Cholesky of -(-S)), U = L^{-H}, X = U (U^H Hm)
    if ((st = ok(px::launch_scale(size_t(2) * n_phi * n_phi, D(l.S), -1.0, D(l.Mneg), stream), "-S")) != PX_OK)
      return st;
    if ((st = ok(px::launch_chol_inv(D(l.Mneg), n_phi, D(l.L), D(l.U), sts + k, D(l.dinv), stream),
                 "cholesky of S")) != PX_OK) return st;
    if ((st = ok(px::launch_zgemm(true, n_phi, D(l.U), D(l.Hm), D(l.T), stream), "U^H Hm")) != PX_OK) return st;
    if ((st = ok(px::launch_zgemm(false, n_phi, D(l.U), D(l.T), D(l.X), stream), "U (U^H Hm)")) != PX_OK)
      return st;
    if (fp32 && (st = ok(px::launch_convert_f64_f32(size_t(2) * n_phi * n_phi, D(l.X), X32, stream),
                         "X to FP32")) != PX_OK) return st;
    // Z = -mid X (the projection P~ Y with its sign), then Phi^(k+1) = Phi_n - i dt_alpha (Y + Z)
    if ((st = ok(px::launch_gemm_xc(fp32, n_phi, n_phi, ng, mid, Xc, n_phi, -1.0, w + l.Z, false, stream),
                 "Z = -mid X")) != PX_OK) return st;
    if ((st = ok(px::launch_ptim_update(fp32, nel, phi_n, w + l.Y, w + l.Z, cur_p, nxt_p, dt_alpha,
                                        D(l.partial), residuals + k, stream), "orbital update")) != PX_OK)
      return st;
    // sigma^(k+1) = sigma_n - i dt_alpha (Hm smid - smid Hm) (Eq. 6)
    if ((st = ok(px::launch_midpoint(false, size_t(n_phi) * n_phi, sigma_n, cur_s, D(l.smid), stream),
                 "sigma midpoint")) != PX_OK) return st;
    if ((st = ok(px::launch_zgemm(false, n_phi, D(l.Hm), D(l.smid), D(l.A1), stream), "Hm smid")) != PX_OK)
      return st;
    if ((st = ok(px::launch_zgemm(false, n_phi, D(l.smid), D(l.Hm), D(l.A2), stream), "smid Hm")) != PX_OK)
      return st;
    if ((st = ok(px::launch_sigma_update(n_phi, sigma_n, D(l.A1), D(l.A2), cur_s, nxt_s, dt_alpha,
                                         residuals + n_iter + k, stream), "sigma update")) != PX_OK)
      return st;
    cur_p = nxt_p;
    cur_s = nxt_s;
  }
  st = ok(px::launch_status_first(sts, n_iter, status, stream), "status");
  if (st == PX_OK)
    ctx->last_status.assign(1, {status, PX_ERR_NOT_POSITIVE_DEFINITE, "ptim_step: the midpoint overlap S"});
  return st;
}

px_status px_set_symmetry(px_context* ctx, int32_t enable) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  ctx->symmetric_ace = enable != 0;
  return PX_OK;
}

px_status px_set_profiling(px_context* ctx, int32_t enable) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  ctx->profiling = enable != 0;
  return PX_OK;
}

px_status px_profile_read(px_context* ctx, double* ms, double* bytes, int64_t* launches,
                          int32_t reset) {
  if (!ctx || !ms || !bytes || !launches) return PX_ERR_INVALID_ARG;
  for (int k = 0; k < 4; ++k) {
    ms[k] = ctx->prof_ms[k];
    bytes[k] = ctx->prof_bytes[k];
    launches[k] = ctx->prof_launches[k];
    if (reset) ctx->prof_ms[k] = ctx->prof_bytes[k] = 0.0, ctx->prof_launches[k] = 0;
  }
  return PX_OK;
}

px_status px_profile_read_ace(px_context* ctx, double* ms, int64_t* calls, int32_t reset) {
  if (!ctx || !ms || !calls) return PX_ERR_INVALID_ARG;
  for (int k = 0; k < 4; ++k) {
    ms[k] = ctx->ace_ms[k];
    if (reset) ctx->ace_ms[k] = 0.0;
  }
  *calls = ctx->ace_calls;
  if (reset) ctx->ace_calls = 0;
  return PX_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batched form
namespace {

struct BatchWave {
  int g[3];         // grid of the wave's instances
  int p2;           // pass-2 configuration of that size
  int first, count; // tasks [first, first + count)
  int max_ic, max_jc, max_pairs, max_slots;  // max_pairs: solved pairs; max_slots: ic * jc
  bool any_v;       // its tasks keep v_ij for pass 4 (a wave holds one block diagonal, so
                    // all of its tasks or none)
};

// The ACE tail of the instances whose last chunk is in wave after_wave: their
// Gram matrices, one grouped factorisation (jobs [first_job, first_job +
// count) of the job table) and their xi, on side stream lane.
struct TailGroup {
  int after_wave, lane, first_job, count, max_n;
};

struct BatchPlan {
  size_t tasks_off = 0, jobs_off = 0, table_end = 0, t_off = 0, g0_off = 0, ex_off = 0;
  std::vector<size_t> S_off, W_off, K32_off;
  // ACE: per instance M (unless the caller's), L (FP32: then U in complex64),
  // U and the diagonal-block inverses; per lane the Gram split partials
  std::vector<size_t> M_off, L_off, U_off, dinv_off, part_off;
  size_t end = 0;
  std::vector<px::ChunkArgs> tasks;
  std::vector<px::CholJob> jobs;   // instance order of the tail groups
  std::vector<int> job_inst;       // instance of each job
  std::vector<BatchWave> waves;
  std::vector<TailGroup> groups;
};

int block_for(const px_context* c, const px_cell* cell, px_precision prec) {
  int ic, jc;
  tuning_for(c, cell, prec, &ic, &jc);
  return ic > jc ? ic : jc;
}
int pass2_cfg_for(const px_context* c, const px_cell* cell, px_precision prec) {
  int ic, jc, p2;
  tuning_for(c, cell, prec, &ic, &jc, &p2);
  return p2;
}

// Plan of one batched call.  Instances are grouped by grid (all three
// lengths); within a grid the block pairs (I, J <= I) of every instance are
// scheduled by block diagonal d = I - J, so that one launch never has two
// chunks writing the same output block (pass 3 writes block I, pass 4 block
// J): d = 0 first (those chunks initialise the output), then d = 1, 2, ...  A
// diagonal's chunks are packed into waves that fit the pair buffer.  In ACE
// mode the instances completed by a wave form a tail group.  ws == nullptr:
// sizes only.
BatchPlan plan_batch(const px_context* c, int n_inst, const px_instance* in, px_precision prec,
                     bool ace, char* ws) {
  BatchPlan P;
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t b = elem_bytes(prec);
  size_t t_bytes = 0, side_pairs = 0;  // sizes of the pair buffer and of the per-plane partials
  // schedule: grids in order of size
  using Grid = std::array<int, 3>;
  auto grid_of = [&](int k) { return Grid{in[k].cell.n[0], in[k].cell.n[1], in[k].cell.n[2]}; };
  std::vector<Grid> grids;
  for (int k = 0; k < n_inst; ++k)
    if (std::find(grids.begin(), grids.end(), grid_of(k)) == grids.end()) grids.push_back(grid_of(k));
  std::sort(grids.begin(), grids.end(), [](const Grid& x, const Grid& y) {
    const size_t nx = size_t(x[0]) * x[1] * x[2], ny = size_t(y[0]) * y[1] * y[2];
    return nx != ny ? nx < ny : x < y;
  });
  struct Chunk { int inst, I, J, B; };
  for (const Grid& gr : grids) {
    // pair-buffer capacity of the grid: batch_cap_bytes, at least its largest chunk
    int max_nb = 0;
    size_t min_pairs = 1;
    for (int k = 0; k < n_inst; ++k)
      if (grid_of(k) == gr) {
        const int B = block_for(c, &in[k].cell, prec);
        max_nb = std::max(max_nb, (int(in[k].n) + B - 1) / B);
        const size_t e = size_t(std::min(B, int(in[k].n)));
        min_pairs = std::max(min_pairs, e * e);
      }
    const size_t ng = size_t(gr[0]) * gr[1] * gr[2];
    const size_t cap = std::max(min_pairs, c->batch_cap_bytes / (ng * b));
    t_bytes = std::max(t_bytes, cap * ng * b);
    // per pair: n2 slab sums (g0) and n1 * XS energy-partial slots
    int p2 = 0;  // the tuning of the grid (every instance of a grid shares it)
    for (int k = 0; k < n_inst; ++k)
      if (grid_of(k) == gr) p2 = pass2_cfg_for(c, &in[k].cell, prec);
    const size_t per_pair = std::max(size_t(gr[1]) * px::pass2_sections_grid(fp32, gr.data(), p2),
                                     size_t(gr[2]));
    side_pairs = std::max(side_pairs, cap * per_pair);
    for (int d = 0; d < max_nb; ++d) {
      std::vector<Chunk> diag;
      for (int k = 0; k < n_inst; ++k) {
        if (grid_of(k) != gr) continue;
        const int B = block_for(c, &in[k].cell, prec);
        const int nb = (int(in[k].n) + B - 1) / B;
        for (int J = 0; J + d < nb; ++J) diag.push_back({k, J + d, J, B});
      }
      size_t used = cap;  // forces a new wave at the first chunk
      for (const Chunk& ch : diag) {
        const int n = in[ch.inst].n;
        const int icc = std::min(ch.B, n - ch.I * ch.B), jcc = std::min(ch.B, n - ch.J * ch.B);
        const size_t pairs = size_t(icc) * jcc;
        if (used + pairs > cap) {
          P.waves.push_back({{gr[0], gr[1], gr[2]}, p2, int(P.tasks.size()), 0, 0, 0, 0, 0, false});
          used = 0;
        }
        BatchWave& w = P.waves.back();
        px::ChunkArgs a{};
        a.i0 = ch.I * ch.B;
        a.ic = icc;
        a.j0 = ch.J * ch.B;
        a.jc = jcc;
        a.first = d == 0;
        a.tri = d == 0 && c->tri_diag && icc == jcc;
        a.store_v = d > 0 || a.tri;
        a.n2 = gr[2];
        a.inv_ng = 1.0 / double(ng);
        a.s_ld = n;
        // pointers are filled below once the layout is known; keep the
        // within-wave pair offset in t (as an integer) until then
        a.t = reinterpret_cast<void*>(used);
        a.psi = a.phi = in[ch.inst].psi;
        a.occ = in[ch.inst].occ;
        a.kern = in[ch.inst].kernel_G;
        a.S = reinterpret_cast<double*>(size_t(ch.inst));  // instance index until layout
        P.tasks.push_back(a);
        w.count++;
        w.max_ic = std::max(w.max_ic, icc);
        w.max_jc = std::max(w.max_jc, jcc);
        // launch grids cover the solved pairs (the lower triangle of a
        // triangular block), not the block's pair slots
        w.max_pairs = std::max(w.max_pairs, px::chunk_pairs(a));
        w.max_slots = std::max(w.max_slots, int(pairs));
        w.any_v = w.any_v || a.store_v;
        used += pairs;
      }
    }
  }
  // ACE tails: an instance's tail may start once the last wave holding one of
  // its chunks has run; the instances completed by one wave form a group
  if (ace) {
    std::vector<int> last(n_inst, -1);
    for (int w = 0; w < int(P.waves.size()); ++w)
      for (int t = P.waves[w].first; t < P.waves[w].first + P.waves[w].count; ++t)
        last[int(reinterpret_cast<size_t>(P.tasks[t].S))] = w;
    for (int w = 0; w < int(P.waves.size()); ++w) {
      TailGroup g{w, int(P.groups.size()) % px_context::kTailLanes, int(P.job_inst.size()), 0, 0};
      for (int k = 0; k < n_inst; ++k)
        if (last[k] == w) {
          P.job_inst.push_back(k);
          g.count++;
          g.max_n = std::max(g.max_n, int(in[k].n));
        }
      if (g.count) P.groups.push_back(g);
    }
    P.jobs.resize(P.job_inst.size());
  }
  // layout
  size_t off = 0;
  P.tasks_off = off;
  off = align_up(off + P.tasks.size() * sizeof(px::ChunkArgs));
  P.jobs_off = off;
  off = align_up(off + P.jobs.size() * sizeof(px::CholJob));
  P.table_end = off;
  P.t_off = off;
  off = align_up(off + t_bytes);
  P.g0_off = off;
  if (fp32) off = align_up(off + side_pairs * sizeof(px::G0Part));
  P.ex_off = off;
  off = align_up(off + side_pairs * 8 * (fp32 ? 3 : 1));
  P.S_off.resize(n_inst);
  P.W_off.resize(n_inst);
  P.K32_off.resize(n_inst);
  for (int k = 0; k < n_inst; ++k) {
    P.S_off[k] = off;
    off = align_up(off + size_t(in[k].n) * in[k].n * 8);
  }
  if (fp32) {
    for (int k = 0; k < n_inst; ++k) {
      P.K32_off[k] = off;
      off = align_up(off + ngrid(&in[k].cell) * sizeof(float));
    }
  }
  if (ace) {
    P.M_off.resize(n_inst);
    P.L_off.resize(n_inst);
    P.U_off.resize(n_inst);
    P.dinv_off.resize(n_inst);
    for (int k = 0; k < n_inst; ++k) {
      const size_t nn = size_t(in[k].n) * in[k].n * 16;
      P.W_off[k] = off;
      off = align_up(off + size_t(in[k].n) * ngrid(&in[k].cell) * b);
      P.M_off[k] = off;
      off = align_up(off + nn);
      P.L_off[k] = off;
      off = align_up(off + nn);
      P.U_off[k] = off;
      off = align_up(off + nn);
      P.dinv_off[k] = off;
      off = align_up(off + px::chol_dinv_bytes(in[k].n));
    }
    size_t part = 0;
    for (int k = 0; k < n_inst; ++k) {
      int ns = 0;
      part = std::max(part, px::gemm_xhy_part_elems(in[k].n, in[k].n, ngrid(&in[k].cell), &ns));
    }
    P.part_off.resize(px_context::kTailLanes);
    for (int l = 0; l < px_context::kTailLanes; ++l) {
      P.part_off[l] = off;
      off = align_up(off + part * 16);
    }
  }
  P.end = off;
  if (ws) {
    for (const BatchWave& w : P.waves) {
      const size_t ng = size_t(w.g[0]) * w.g[1] * w.g[2];
      for (int t = w.first; t < w.first + w.count; ++t) {
        px::ChunkArgs& a = P.tasks[t];
        const size_t pofs = reinterpret_cast<size_t>(a.t);
        const int k = int(reinterpret_cast<size_t>(a.S));
        a.t = ws + P.t_off + pofs * ng * b;
        a.g0 = reinterpret_cast<px::G0Part*>(ws + P.g0_off + pofs * w.g[2] * sizeof(px::G0Part));
        a.expart = reinterpret_cast<double*>(ws + P.ex_off + pofs * w.g[1] *
                                             px::pass2_sections_grid(fp32, w.g, w.p2) * 8 *
                                             (fp32 ? 3 : 1));
        a.S = reinterpret_cast<double*>(ws + P.S_off[k]);
        a.out = ace ? static_cast<void*>(ws + P.W_off[k]) : in[k].out;
        if (fp32) a.kern32 = reinterpret_cast<const float*>(ws + P.K32_off[k]);
      }
    }
    for (size_t q = 0; q < P.jobs.size(); ++q) {
      const int k = P.job_inst[q];
      px::CholJob& j = P.jobs[q];
      j.M = in[k].M ? in[k].M : reinterpret_cast<double*>(ws + P.M_off[k]);
      j.L = reinterpret_cast<double*>(ws + P.L_off[k]);
      j.U = reinterpret_cast<double*>(ws + P.U_off[k]);
      j.dinv = reinterpret_cast<double*>(ws + P.dinv_off[k]);
      j.status = in[k].status;
      j.n = int(in[k].n);
    }
  }
  return P;
}

// The host image of the task and job tables, laid out as in the workspace
// from tasks_off.
void table_image(const BatchPlan& P, std::vector<unsigned char>& img) {
  img.assign(P.table_end - P.tasks_off, 0);
  std::memcpy(img.data(), P.tasks.data(), P.tasks.size() * sizeof(px::ChunkArgs));
  if (!P.jobs.empty())
    std::memcpy(img.data() + (P.jobs_off - P.tasks_off), P.jobs.data(),
                P.jobs.size() * sizeof(px::CholJob));
}

px_status check_instances(px_context* c, int n_inst, const px_instance* in, px_precision prec,
                          bool ace) {
  if (n_inst <= 0 || !in) return fail(c, PX_ERR_INVALID_ARG, "batched: need n_inst > 0 instances");
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(c, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  for (int k = 0; k < n_inst; ++k) {
    const px_instance& x = in[k];
    px_status st = check_grid(c, &x.cell);
    if (st != PX_OK) return fail(c, st, "instance %d: %s", k, c->err.c_str());
    if (x.n <= 0) return fail(c, PX_ERR_INVALID_ARG, "instance %d: n must be > 0", k);
    if (!x.psi || !x.occ || !x.kernel_G || !x.out)
      return fail(c, PX_ERR_INVALID_ARG, "instance %d: null array argument", k);
    if (x.out == x.psi) return fail(c, PX_ERR_INVALID_ARG, "instance %d: out aliases psi", k);
    if (misaligned(x.psi) || misaligned(x.out))
      return fail(c, PX_ERR_INVALID_ARG, "instance %d: orbital blocks must be 16-byte aligned", k);
    if (ace && !x.status)
      return fail(c, PX_ERR_INVALID_ARG, "instance %d: ACE mode needs a status word", k);
  }
  return PX_OK;
}

// The ACE tail of one group on stream ls: Gram matrices (and energies), one
// grouped factorisation, xi.
px_status enqueue_tail(px_context* c, const BatchPlan& P, const TailGroup& g, const px_instance* in,
                       px_precision prec, hipStream_t ls) {
  const bool fp32 = prec == PX_PREC_FP32;
  char* ws = c->ws;
  double* part = reinterpret_cast<double*>(ws + P.part_off[g.lane]);
  px_status st = PX_OK;
  for (int q = g.first_job; q < g.first_job + g.count; ++q) {
    const int k = P.job_inst[q];
    const px_instance& x = in[k];
    const size_t ng = ngrid(&x.cell);
    const double omega = x.cell.L[0] * x.cell.L[1] * x.cell.L[2];
    if (x.e_x) {
      st = hip_check(c, px::launch_energy(reinterpret_cast<const double*>(ws + P.S_off[k]), x.occ,
                                          x.n, -0.5 * omega / (double(ng) * double(ng)), x.e_x, ls),
                     "batched energy");
      if (st != PX_OK) return st;
    }
    int nsplit = 0;
    px::gemm_xhy_part_elems(x.n, x.n, ng, &nsplit);
    st = hip_check(c, px::launch_gemm_xhy_herm(fp32, x.n, ng, x.psi, ws + P.W_off[k],
                                               omega / double(ng), P.jobs[q].M, part, nsplit, ls),
                   "batched M");
    if (st != PX_OK) return st;
  }
  const px::CholJob* dj = reinterpret_cast<const px::CholJob*>(ws + P.jobs_off) + g.first_job;
  st = hip_check(c, px::launch_chol_inv_group(dj, g.count, g.max_n, ls), "batched cholesky");
  if (st != PX_OK) return st;
  for (int q = g.first_job; q < g.first_job + g.count; ++q) {
    const int k = P.job_inst[q];
    const px_instance& x = in[k];
    const size_t ng = ngrid(&x.cell);
    // FP32 form: U rounded to complex64 into L's place (L is not read again)
    const void* Uc = P.jobs[q].U;
    if (fp32) {
      st = hip_check(c, px::launch_convert_f64_f32(size_t(2) * x.n * x.n, P.jobs[q].U,
                                                   reinterpret_cast<float*>(P.jobs[q].L), ls),
                     "batched U to FP32");
      if (st != PX_OK) return st;
      Uc = P.jobs[q].L;
    }
    st = hip_check(c, px::launch_gemm_xc(fp32, x.n, x.n, ng, ws + P.W_off[k], Uc, x.n, 1.0, x.out,
                                         true, ls),
                   "batched xi");
    if (st != PX_OK) return st;
  }
  return PX_OK;
}

// Side streams and events of the ACE tails (created once per context).
px_status ensure_lanes(px_context* c, size_t n_fork) {
  for (int l = 0; l < px_context::kTailLanes; ++l) {
    if (!c->lanes[l] && hipStreamCreateWithFlags(&c->lanes[l], hipStreamNonBlocking) != hipSuccess)
      return fail(c, PX_ERR_DEVICE, "hipStreamCreate (tail lane) failed");
    if (!c->lane_done[l] &&
        hipEventCreateWithFlags(&c->lane_done[l], hipEventDisableTiming) != hipSuccess)
      return fail(c, PX_ERR_DEVICE, "hipEventCreate failed");
  }
  while (c->fork_events.size() < n_fork) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return fail(c, PX_ERR_DEVICE, "hipEventCreate failed");
    c->fork_events.push_back(e);
  }
  return PX_OK;
}

// Everything of one batched call, stream ordered on s: the pair-pipeline
// waves on s; in ACE mode each tail group on its lane once its wave has run,
// and s waits for every lane at the end (also after an error, so that a
// capture is always joined).
px_status enqueue_batch(px_context* c, const BatchPlan& P, int n_inst, const px_instance* in,
                        px_precision prec, bool ace, const void* host_table, hipStream_t s) {
  const bool fp32 = prec == PX_PREC_FP32;
  char* ws = c->ws;
  const px::ChunkArgs* dt = reinterpret_cast<const px::ChunkArgs*>(ws + P.tasks_off);
  px_status st = hip_check(c, hipMemcpyAsync(ws + P.tasks_off, host_table, P.table_end - P.tasks_off,
                                             hipMemcpyHostToDevice, s),
                           "task table upload");
  if (st != PX_OK) return st;
  if (ace && (st = ensure_lanes(c, P.waves.size())) != PX_OK) return st;
  if (fp32) {
    for (int k = 0; k < n_inst; ++k) {
      st = hip_check(c, px::launch_convert_f64_f32(ngrid(&in[k].cell), in[k].kernel_G,
                                                   reinterpret_cast<float*>(ws + P.K32_off[k]), s),
                     "batched kernel to FP32");
      if (st != PX_OK) return st;
    }
  }
  bool used[px_context::kTailLanes] = {false, false};
  size_t gi = 0;
  for (int wi = 0; wi < int(P.waves.size()) && st == PX_OK; ++wi) {
    const BatchWave& w = P.waves[wi];
    const size_t ng = size_t(w.g[0]) * w.g[1] * w.g[2];
    st = hip_check(c, px::launch_chunk_tasks(fp32, w.g, dt + w.first, w.count, w.max_ic,
                                             w.max_pairs, true, w.any_v, w.p2, s),
                   "batched pair pipeline");
    if (st != PX_OK) break;
    if (w.any_v) {
      st = hip_check(c, px::launch_pass4_tasks(fp32, dt + w.first, w.count, w.max_jc, ng, s),
                     "batched transposed accumulation");
      if (st != PX_OK) break;
    }
    st = hip_check(c, px::launch_expart_reduce_tasks(fp32, dt + w.first, w.count, w.max_slots,
                                                     w.g[1] * px::pass2_sections_grid(fp32, w.g, w.p2), w.g[2],
                                                     double(ng), s),
                   "batched energy partials");
    if (st != PX_OK) break;
    if (gi < P.groups.size() && P.groups[gi].after_wave == wi) {
      hipEvent_t e = c->fork_events[wi];
      st = hip_check(c, hipEventRecord(e, s), "fork event");
      while (st == PX_OK && gi < P.groups.size() && P.groups[gi].after_wave == wi) {
        const TailGroup& g = P.groups[gi++];
        st = hip_check(c, hipStreamWaitEvent(c->lanes[g.lane], e, 0), "tail lane wait");
        if (st != PX_OK) break;
        used[g.lane] = true;
        st = enqueue_tail(c, P, g, in, prec, c->lanes[g.lane]);
      }
    }
  }
  for (int l = 0; l < px_context::kTailLanes; ++l) {
    if (!used[l]) continue;
    px_status sj = hip_check(c, hipEventRecord(c->lane_done[l], c->lanes[l]), "lane event");
    if (sj == PX_OK) sj = hip_check(c, hipStreamWaitEvent(s, c->lane_done[l], 0), "lane join");
    if (st == PX_OK) st = sj;
  }
  if (st != PX_OK || ace) return st;
  for (int k = 0; k < n_inst; ++k) {
    const px_instance& x = in[k];
    if (!x.e_x) continue;
    const size_t ng = ngrid(&x.cell);
    const double omega = x.cell.L[0] * x.cell.L[1] * x.cell.L[2];
    st = hip_check(c, px::launch_energy(reinterpret_cast<const double*>(ws + P.S_off[k]), x.occ, x.n,
                                        -0.5 * omega / (double(ng) * double(ng)), x.e_x, s),
                   "batched energy");
    if (st != PX_OK) return st;
  }
  return PX_OK;
}

std::vector<unsigned char> batch_key(const px_context* c, int n_inst, const px_instance* in,
                                     px_precision prec, bool ace) {
  std::vector<unsigned char> key;
  auto put = [&key](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    key.insert(key.end(), b, b + n);
  };
  put(&n_inst, sizeof n_inst);
  put(&prec, sizeof prec);
  put(&ace, sizeof ace);
  put(&c->ws, sizeof c->ws);
  put(&c->ws_bytes, sizeof c->ws_bytes);
  put(&c->batch_cap_bytes, sizeof c->batch_cap_bytes);
  for (int k = 0; k < n_inst; ++k) {
    put(&in[k], sizeof(px_instance));
    const int B = block_for(c, &in[k].cell, prec), p2 = pass2_cfg_for(c, &in[k].cell, prec);
    put(&B, sizeof B);
    put(&p2, sizeof p2);
  }
  return key;
}

}  // namespace

extern "C" {

size_t px_workspace_bytes_batched(const px_context* ctx, int32_t n_inst, const px_instance* inst,
                                  px_precision prec, int32_t ace) {
  if (!ctx || n_inst <= 0 || !inst) return 0;
  for (int k = 0; k < n_inst; ++k)
    if (!cell_ok(&inst[k].cell) || inst[k].n <= 0 ||
        !px::grid_supported(inst[k].cell.n[0], inst[k].cell.n[1], inst[k].cell.n[2]))
      return 0;
  return plan_batch(ctx, n_inst, inst, prec, ace != 0, nullptr).end;
}

px_status px_set_batch_capacity(px_context* ctx, size_t pair_buffer_bytes) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  ctx->batch_cap_bytes = pair_buffer_bytes ? pair_buffer_bytes : (size_t(4) << 30);
  return PX_OK;
}

px_status px_set_graph(px_context* ctx, int32_t enable) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  ctx->use_graph = enable != 0;
  return PX_OK;
}

px_status px_exchange_apply_batched(px_context* ctx, int32_t n_inst, const px_instance* inst,
                                    px_precision prec, int32_t ace, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  px_status st = check_instances(ctx, n_inst, inst, prec, ace != 0);
  if (st != PX_OK) return st;
  BatchPlan P = plan_batch(ctx, n_inst, inst, prec, ace != 0, nullptr);
  st = need_ws(ctx, P.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  P = plan_batch(ctx, n_inst, inst, prec, ace != 0, ctx->ws);
  std::vector<unsigned char> img;
  table_image(P, img);
  const size_t tbytes = img.size();
  if (ace) {
    ctx->last_status.clear();
    for (int k = 0; k < n_inst; ++k)
      ctx->last_status.push_back(
          {inst[k].status, PX_ERR_NOT_POSITIVE_DEFINITE, "ace_build of instance " + std::to_string(k) + ": -M"});
  }
  std::vector<unsigned char> key = batch_key(ctx, n_inst, inst, prec, ace != 0);
  if (ctx->use_graph && ctx->graph_exec && key == ctx->graph_key)
    return hip_check(ctx, hipGraphLaunch(ctx->graph_exec, stream), "hipGraphLaunch");
  // new signature: (re)build the page-locked task table; wait for work that
  // may still read the old one
  if (ctx->pinned_tasks) {
    he = hipStreamSynchronize(stream);
    if (he != hipSuccess) return hip_check(ctx, he, "hipStreamSynchronize");
  }
  if (ctx->pinned_bytes < tbytes) {
    if (ctx->pinned_tasks) (void)hipHostFree(ctx->pinned_tasks);
    ctx->pinned_tasks = nullptr;
    ctx->pinned_bytes = 0;
    he = hipHostMalloc(&ctx->pinned_tasks, tbytes, hipHostMallocDefault);
    if (he != hipSuccess) return hip_check(ctx, he, "hipHostMalloc (task table)");
    ctx->pinned_bytes = tbytes;
  }
  std::memcpy(ctx->pinned_tasks, img.data(), tbytes);
  if (!ctx->use_graph) return enqueue_batch(ctx, P, n_inst, inst, prec, ace != 0, ctx->pinned_tasks, stream);
  if (!ctx->cap_stream) {
    he = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
    if (he != hipSuccess) return hip_check(ctx, he, "hipStreamCreate (capture)");
  }
  if (ctx->graph_exec) {
    (void)hipGraphExecDestroy(ctx->graph_exec);
    ctx->graph_exec = nullptr;
    ctx->graph_key.clear();
  }
  he = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
  if (he != hipSuccess) return hip_check(ctx, he, "hipStreamBeginCapture");
  st = enqueue_batch(ctx, P, n_inst, inst, prec, ace != 0, ctx->pinned_tasks, ctx->cap_stream);
  hipGraph_t g = nullptr;
  he = hipStreamEndCapture(ctx->cap_stream, &g);
  if (st != PX_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (he != hipSuccess) return hip_check(ctx, he, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  he = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (he != hipSuccess) return hip_check(ctx, he, "hipGraphInstantiate");
  ctx->graph_exec = ex;
  ctx->graph_key = key;
  return hip_check(ctx, hipGraphLaunch(ex, stream), "hipGraphLaunch");
}

// Times the symmetric pair pipeline for square blocks B in the candidate list
// on the caller's instance, keeps the fastest as the context's tuning for this
// grid and precision, and appends it to cache_path (JSON lines) when given.
px_status px_autotune(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                      const void* psi, const double* occ, const double* kernel_G, void* out,
                      const char* cache_path, int32_t* best_block, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_grid(ctx, cell);
  if (st != PX_OK) return st;
  if (n <= 0 || !psi || !occ || !kernel_G || !out || out == psi || misaligned(psi) ||
      misaligned(out))
    return fail(ctx, PX_ERR_INVALID_ARG,
                "autotune: need n > 0 and valid, non-aliased, 16-byte aligned arrays");
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  // square pair blocks B (the Hermitian-pair mode's chunks are B x B) and the
  // two compiled pass-2 configurations; candidates whose pair buffer does not
  // fit the attached workspace are skipped
  const int cand[] = {16, 24, 32, 48, 64, 96, 128, 192, 256};
  const auto key = std::make_tuple(cell->n[0], cell->n[1], cell->n[2], int(prec));
  const bool had = ctx->tuning.count(key) != 0;
  const auto saved = had ? ctx->tuning[key] : std::make_tuple(0, 0, 0);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(ctx, PX_ERR_DEVICE, "hipEventCreate failed");
  double best = 1e300;
  int bestB = 0, bestP2 = 0;
  std::string trials;
  bool covered = false;  // a candidate B >= n has been timed (larger ones are the same chunking)
  for (int B : cand) {
    if (covered) break;
    covered = B >= n;
    for (int p2 = 0; p2 < px::pass2_configs(cell->n) && st == PX_OK; ++p2) {
      const ExLayout l = ex_layout(cell, prec, n, n, B, B, false, p2);
      if (ctx->ws == nullptr || ctx->ws_bytes < l.end) continue;
      float ms = 0.f, best_ms = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, stream);
        st = run_exchange(ctx, cell, prec, n, psi, occ, n, psi, kernel_G, out, l, false, B, B, true,
                          stream, p2);
        (void)hipEventRecord(e1, stream);
        if (st != PX_OK) break;
        he = hipEventSynchronize(e1);
        if (he != hipSuccess) {
          st = hip_check(ctx, he, "autotune sync");
          break;
        }
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) best_ms = std::min(best_ms, ms);  // first run warms up
      }
      if (st != PX_OK) break;
      const double us_pair = 1e3 * best_ms / (double(n) * n);
      char buf[64];
      snprintf(buf, sizeof buf, "%s\"%d/%d\": %.4f", trials.empty() ? "" : ", ", B, p2, us_pair);
      trials += buf;
      if (us_pair < best) {
        best = us_pair;
        bestB = B;
        bestP2 = p2;
      }
    }
    if (st != PX_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != PX_OK) return st;
  if (bestB == 0) {
    if (had) ctx->tuning[key] = saved;
    return fail(ctx, PX_ERR_WORKSPACE, "autotune: workspace too small for every candidate block");
  }
  ctx->tuning[key] = {bestB, bestB, bestP2};
  if (best_block) *best_block = bestB;
  if (cache_path && cache_path[0]) {
    FILE* f = fopen(cache_path, "a");
    if (!f) return fail(ctx, PX_ERR_INVALID_ARG, "autotune: cannot open %s", cache_path);
    fprintf(f,
            "{\"arch\": \"gfx950\", \"n\": [%d, %d, %d], \"prec\": \"%s\", \"n_orb\": %d, "
            "\"block\": %d, \"p2\": %d, \"us_per_pair\": %.4f, \"trials_us_per_pair\": {%s}}\n",
            cell->n[0], cell->n[1], cell->n[2], prec == PX_PREC_FP32 ? "fp32" : "fp64", n, bestB,
            bestP2, best, trials.c_str());
    fclose(f);
  }
  return PX_OK;
}

// Reads the JSON lines written by px_autotune; the last entry per (grid,
// precision) wins.  Returns the number of entries applied in *applied.
px_status px_load_tuning(px_context* ctx, const char* cache_path, int32_t* applied) {
  if (!ctx || !cache_path) return PX_ERR_INVALID_ARG;
  FILE* f = fopen(cache_path, "r");
  if (!f) return fail(ctx, PX_ERR_INVALID_ARG, "load_tuning: cannot open %s", cache_path);
  char line[4096];
  int count = 0;
  while (fgets(line, sizeof line, f)) {
    int n0, n1, n2, blk;
    char prec[8] = {0};
    const char* pn = strstr(line, "\"n\": [");
    const char* pp = strstr(line, "\"prec\": \"");
    const char* pb = strstr(line, "\"block\": ");
    if (!pn || !pp || !pb) continue;
    if (sscanf(pn, "\"n\": [%d, %d, %d]", &n0, &n1, &n2) != 3) continue;
    if (sscanf(pp, "\"prec\": \"%4[a-z0-9]\"", prec) != 1) continue;
    if (sscanf(pb, "\"block\": %d", &blk) != 1 || blk <= 0 || blk > 4096) continue;
    const int pr = strcmp(prec, "fp32") == 0 ? int(PX_PREC_FP32) : int(PX_PREC_FP64);
    int p2 = 0;  // pass-2 configuration (absent in older lines: the default)
    const char* pq = strstr(line, "\"p2\": ");
    const int grid[3] = {n0, n1, n2};
    if (pq && (sscanf(pq, "\"p2\": %d", &p2) != 1 || p2 < 0 || p2 >= px::pass2_configs(grid))) p2 = 0;
    ctx->tuning[std::make_tuple(n0, n1, n2, pr)] = {blk, blk, p2};
    ++count;
  }
  fclose(f);
  if (applied) *applied = count;
  return PX_OK;
}

}  // extern "C"

extern "C" {

px_status px_sync(px_context* ctx, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_check(ctx, e, "hipStreamSynchronize");
  for (size_t k = 0; k < ctx->last_status.size(); ++k) {
    int32_t s = 0;
    e = hipMemcpy(&s, ctx->last_status[k].word, sizeof s, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_check(ctx, e, "status readback");
    if (s != 0 && ctx->latched == PX_OK) {
      const px_status kind = ctx->last_status[k].kind;
      const char* what = ctx->last_status[k].what.c_str();
      ctx->latched = kind;
      if (kind == PX_ERR_NOT_POSITIVE_DEFINITE)
        fail(ctx, kind, "%s is not positive definite (Cholesky breakdown at column %d)", what, s);
      else
        fail(ctx, kind, "%s: the Jacobi sweeps of the diagonalisation did not converge (%d sweeps)", what, s);
    }
  }
  ctx->last_status.clear();
  return px_status(ctx->latched);
}

void px_clear_error(px_context* ctx) {
  if (!ctx) return;
  ctx->latched = PX_OK;
  ctx->err.clear();
}

}  // extern "C"


// ------------------------------------------------------------------ ACE application without workspace
// For callers that cannot allocate device memory (code under graph capture,
// tight loops that forbid allocation): the contraction scratch of
// px_ace_apply (the matrix C = dV xi^H phi, its complex64 copy and the split
// partials) lives in a file-scope device array instead of the caller's
// workspace.  Each device holds its own copy of the array, at its own address,
// until the process ends; host code must use that address (taken once per
// device with hipGetSymbolAddress), never the array's name.
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_addr;  // device -> device address of `scratch`

// The device address of `scratch` on the context's (current) device.
px_status scratch_addr(px_context* c, char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(c->device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return PX_OK;
  }
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_check(c, e, "hipGetSymbolAddress (scratch)");
  if (p == nullptr || (reinterpret_cast<uintptr_t>(p) % kAlign) != 0)
    return fail(c, PX_ERR_DEVICE, "scratch array has no usable device address");
  g_scratch_addr[c->device] = static_cast<char*>(p);
  *out = static_cast<char*>(p);
  return PX_OK;
}

}  // namespace

extern "C" px_status px_ace_apply_noalloc(px_context* ctx, const px_cell* cell, px_precision prec,
                                          int32_t n, const void* xi, int32_t n_phi, const void* phi,
                                          void* out, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  px_status st = check_gemm_grid(ctx, cell, prec);
  if (st != PX_OK) return st;
  if (n <= 0 || n_phi <= 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "n and n_phi must be > 0 (got %d, %d)", n, n_phi);
  if (!xi || !phi || !out)
    return fail(ctx, PX_ERR_INVALID_ARG, "ace_apply_noalloc: null array argument");
  if (out == phi || out == xi)
    return fail(ctx, PX_ERR_INVALID_ARG, "ace_apply_noalloc: out must not alias xi or phi");
  if (misaligned(xi) || misaligned(phi) || misaligned(out))
    return fail(ctx, PX_ERR_INVALID_ARG,
                "ace_apply_noalloc: orbital blocks must be 16-byte aligned");
  // scratch: C (complex128), C rounded to complex64, then at least one split of partials
  const size_t nn = size_t(n) * size_t(n_phi);
  const size_t c_off = 0, c32_off = align_up(nn * 16), part_off = align_up(c32_off + nn * 8);
  if (part_off + nn * 16 > kScratchBytes)
    return fail(ctx, PX_ERR_WORKSPACE,
                "ace_apply_noalloc: n * n_phi = %zu exceeds the %zu MiB scratch (at most %zu)", nn,
                kScratchBytes >> 20, (kScratchBytes - 2 * kAlign) / 40);
  const int max_split = int((kScratchBytes - part_off) / (nn * 16));
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  char* sc = nullptr;
  st = scratch_addr(ctx, &sc);
  if (st != PX_OK) return st;
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t ng = ngrid(cell);
  const double dV = cell->L[0] * cell->L[1] * cell->L[2] / double(ng);
  double* C = reinterpret_cast<double*>(sc + c_off);
  float* C32 = fp32 ? reinterpret_cast<float*>(sc + c32_off) : nullptr;
  double* part = reinterpret_cast<double*>(sc + part_off);
  const int nsplit = px::gemm_xhy_splits(n, n_phi, ng, max_split);
  // every element of the partials, C and C32 is written before it is read:
  // nothing in the scratch has to start at zero
  st = hip_check(ctx, px::launch_gemm_xhy(fp32, n, n_phi, ng, xi, phi, dV, C, n_phi, part, nsplit,
                                          C32, stream),
                 "C = dV xi^H phi");
  if (st != PX_OK) return st;
  const void* Cc = fp32 ? static_cast<const void*>(C32) : C;
  return hip_check(ctx, px::launch_gemm_xc(fp32, n, n_phi, ng, xi, Cc, n_phi, -1.0, out, false, stream),
                   "out = -xi C");
}
