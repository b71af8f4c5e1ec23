// Host side of libpx: argument validation, workspace carving and the
// stream-ordered orchestration of the exchange and ACE kernels.  No call here
// allocates device memory or synchronises the host, except px_sync.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/px.h"
#include "px_internal.hpp"

struct px_context {
  int device = 0;
  std::string err = "";
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int32_t* last_status = nullptr;  // device status word of the last ACE build
  int latched = PX_OK;
  std::map<std::tuple<int, int, int, int>, std::pair<int, int>> tuning;  // (n0,n1,n2,prec) -> (ic, jc)
  // measurement mode: HIP events around each pass of each chunk
  bool profiling = false;
  std::vector<hipEvent_t> events;
  double prof_ms[4] = {0, 0, 0, 0};
  double prof_bytes[4] = {0, 0, 0, 0};
  int64_t prof_launches[4] = {0, 0, 0, 0};
  bool symmetric_ace = true;  // ACE build solves only pairs j <= i (block level)
  ~px_context() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
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

void tuning_for(const px_context* c, const px_cell* cell, px_precision prec, int* ic, int* jc) {
  auto it = c->tuning.find({cell->n[0], cell->n[1], cell->n[2], int(prec)});
  if (it != c->tuning.end()) {
    *ic = it->second.first;
    *jc = it->second.second;
  } else {
    default_tuning(cell, prec, ic, jc);
  }
}

// Workspace layout of one exchange application.
struct ExLayout {
  size_t t, g0, expart, S, end;
};

ExLayout ex_layout(const px_cell* cell, px_precision prec, int n_psi, int n_phi, int ic, int jc,
                   bool energy) {
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
    off = align_up(off + pairs * cell->n[1] * 8 * (prec == PX_PREC_FP32 ? 3 : 1));
    l.S = off;
    off = align_up(off + size_t(n_phi) * n_psi * 8);
  }
  l.end = off;
  return l;
}

struct AceLayout {
  ExLayout ex;
  size_t W, M, L, U, dinv, part, end;
};

AceLayout ace_layout(const px_cell* cell, px_precision prec, int n, int ic, int jc,
                     bool symmetric) {
  AceLayout a{};
  if (symmetric) ic = jc = (ic > jc ? ic : jc);
  a.ex = ex_layout(cell, prec, n, n, ic, jc, true);
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
  off = align_up(off + 32 * 32 * 16);
  int nsplit = 0;
  const size_t pe = px::gemm_xhy_part_elems(n, n, ngrid(cell), &nsplit);
  a.part = off;
  off = align_up(off + pe * 16);
  a.end = off;
  return a;
}

struct ApplyLayout {
  size_t C, part, end;
};

ApplyLayout apply_layout(const px_cell* cell, int n, int n_phi) {
  ApplyLayout a{};
  size_t off = 0;
  a.C = off;
  off = align_up(off + size_t(n) * n_phi * 16);
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

px_status check_grid(px_context* c, const px_cell* cell) {
  if (!cell_ok(cell))
    return fail(c, PX_ERR_INVALID_ARG, "cell: edge lengths must be > 0 and grid sizes > 0");
  if (!px::grid_supported(cell->n[0], cell->n[1], cell->n[2]))
    return fail(c, PX_ERR_UNSUPPORTED_GRID,
                "grid %dx%dx%d has no compiled FFT plan (cubic n in {16,24,32,40,48,60,64,72,80,96})",
                cell->n[0], cell->n[1], cell->n[2]);
  return PX_OK;
}

px_status need_ws(px_context* c, size_t bytes) {
  if (c->ws == nullptr || c->ws_bytes < bytes)
    return fail(c, PX_ERR_WORKSPACE, "workspace of %zu bytes attached, %zu needed", c->ws_bytes,
                bytes);
  return PX_OK;
}

// Enqueue the pair pipeline for all (i, j); `out` gets Vx phi.  S, when
// non-null, receives sum_G K |rho_ij(G)|^2 per pair for the energy.
// Enqueue the pair pipeline; `out` gets Vx phi.  With energy, S[i][j]
// receives sum_G K |rho_ij(G)|^2 per pair.  Symmetric mode (phi is psi): the
// orbitals are cut into square blocks of B = max(ic, jc); only blocks J <= I
// are solved, and for J < I pass 3 keeps v_ij so that pass 4 adds the
// transposed contributions to the J block (v_ji = conj(v_ij)).
px_status run_exchange(px_context* c, const px_cell* cell, px_precision prec, int n_psi,
                       const void* psi, const double* occ, int n_phi, const void* phi,
                       const double* kern, void* out, const ExLayout& l, bool energy, int ic,
                       int jc, bool symmetric, hipStream_t s) {
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t ng = ngrid(cell);
  px::ChunkArgs a{};
  a.psi = psi;
  a.phi = phi;
  a.t = c->ws + l.t;
  a.out = out;
  a.occ = occ;
  a.kern = kern;
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
      a.store_v = symmetric && j0 < i0;
      hipEvent_t* ev = c->profiling ? &c->events[5 * nchunks] : nullptr;
      px_status st = hip_check(
          c, px::launch_chunk(fp32, cell->n[0], a, a.ic * a.jc, energy, s, ev), "pair pipeline");
      if (st != PX_OK) return st;
      if (a.store_v) {
        st = hip_check(c, px::launch_pass4(fp32, a, ng, s), "transposed accumulation");
        if (st != PX_OK) return st;
      }
      if (c->profiling) {
        (void)hipEventRecord(c->events[5 * nchunks + 4], s);
        // algorithmic bytes, 2 N_g b per pair in each pass (pass 1: read psi_j,
        // write the pair slab; pass 2: read and rewrite it; pass 3: read it and
        // psi_j); in symmetric mode pass 3 also writes v_ij (1 N_g b) and
        // pass 4 reads v_ij and psi_i (2 N_g b)
        const double np = double(a.ic) * a.jc;
        for (int k = 0; k < 3; ++k) {
          c->prof_bytes[k] += 2.0 * pair_bytes * np + (k == 2 && a.store_v ? pair_bytes * np : 0.0);
          c->prof_launches[k] += 1;
        }
        if (a.store_v) {
          c->prof_bytes[3] += 2.0 * pair_bytes * np;
          c->prof_launches[3] += 1;
        }
        has4.push_back(a.store_v);
      }
      ++nchunks;
      if (energy) {
        st = hip_check(c, px::launch_expart_reduce(a.expart, fp32 ? a.g0 : nullptr, cell->n[1],
                                                   cell->n[2], double(ng), i0, a.ic, j0, a.jc, S,
                                                   n_psi, a.store_v != 0, s),
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
  int ic, jc;
  tuning_for(ctx, cell, prec, &ic, &jc);
  switch (op) {
    case PX_OP_EXCHANGE:
      if (n_phi <= 0) return 0;
      return ex_layout(cell, prec, n_psi, n_phi, ic, jc, true).end;
    case PX_OP_ACE_BUILD:
      return ace_layout(cell, prec, n_psi, ic, jc, ctx->symmetric_ace).end;
    case PX_OP_ACE_APPLY:
      if (n_phi <= 0) return 0;
      return apply_layout(cell, n_psi, n_phi).end;
    case PX_OP_PTIM_LOOP:
      if (n_phi <= 0) return 0;
      return loop_layout(cell, prec, n_psi, n_phi).end;
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
  if (ic == 0 || jc == 0) ctx->tuning.erase(key);
  else ctx->tuning[key] = {ic, jc};
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
  if (e_x && (phi != psi || n_phi != n_psi))
    return fail(ctx, PX_ERR_INVALID_ARG, "exchange_apply: e_x requires phi == psi and n_phi == n_psi");
  int ic, jc;
  tuning_for(ctx, cell, prec, &ic, &jc);
  const ExLayout l = ex_layout(cell, prec, n_psi, n_phi, ic, jc, e_x != nullptr);
  st = need_ws(ctx, l.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  st = run_exchange(ctx, cell, prec, n_psi, psi, occ, n_phi, phi, kernel_G, vx_phi, l,
                    e_x != nullptr, ic, jc, false, stream);
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
  int ic, jc;
  tuning_for(ctx, cell, prec, &ic, &jc);
  const AceLayout l = ace_layout(cell, prec, n, ic, jc, ctx->symmetric_ace);
  st = need_ws(ctx, l.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t ng = ngrid(cell);
  const double omega = cell->L[0] * cell->L[1] * cell->L[2];
  const double dV = omega / double(ng);
  void* W = ctx->ws + l.W;
  double* Mw = M ? M : reinterpret_cast<double*>(ctx->ws + l.M);
  double* L = reinterpret_cast<double*>(ctx->ws + l.L);
  double* U = reinterpret_cast<double*>(ctx->ws + l.U);
  double* part = reinterpret_cast<double*>(ctx->ws + l.part);
  // W = Vx Psi (pair pipeline) and the energy sums
  st = run_exchange(ctx, cell, prec, n, psi, occ, n, psi, kernel_G, W, l.ex, true, ic, jc,
                    ctx->symmetric_ace, stream);
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
  // M = dV Psi^H W, Hermitised; -M = L L^H; U = L^{-H}; xi = W U
  st = hip_check(ctx, px::launch_gemm_xhy(fp32, n, n, ng, psi, W, dV, Mw, n, part, nsplit, stream),
                 "M = dV Psi^H W");
  if (st != PX_OK) return st;
  st = hip_check(ctx, px::launch_hermitize(Mw, n, stream), "hermitize");
  if (st != PX_OK) return st;
  st = hip_check(ctx,
                 px::launch_chol_inv(Mw, n, L, U, status,
                                     reinterpret_cast<double*>(ctx->ws + l.dinv), stream),
                 "cholesky");
  if (st != PX_OK) return st;
  st = hip_check(ctx, px::launch_gemm_xc(fp32, n, n, ng, W, U, n, 1.0, xi, true, stream),
                 "xi = W L^-H");
  if (st != PX_OK) return st;
  ctx->last_status = status;
  return PX_OK;
}

px_status px_ace_apply(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                       const void* xi, int32_t n_phi, const void* phi, void* out,
                       hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  if (!cell_ok(cell))
    return fail(ctx, PX_ERR_INVALID_ARG, "cell: edge lengths must be > 0 and grid sizes > 0");
  if (n <= 0 || n_phi <= 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "n and n_phi must be > 0 (got %d, %d)", n, n_phi);
  if (!xi || !phi || !out) return fail(ctx, PX_ERR_INVALID_ARG, "ace_apply: null array argument");
  if (out == phi || out == xi)
    return fail(ctx, PX_ERR_INVALID_ARG, "ace_apply: out must not alias xi or phi");
  const ApplyLayout l = apply_layout(cell, n, n_phi);
  px_status st = need_ws(ctx, l.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t ng = ngrid(cell);
  const double dV = cell->L[0] * cell->L[1] * cell->L[2] / double(ng);
  double* C = reinterpret_cast<double*>(ctx->ws + l.C);
  double* part = reinterpret_cast<double*>(ctx->ws + l.part);
  int nsplit = 0;
  px::gemm_xhy_part_elems(n, n_phi, ng, &nsplit);
  st = hip_check(ctx, px::launch_gemm_xhy(fp32, n, n_phi, ng, xi, phi, dV, C, n_phi, part, nsplit,
                                          stream),
                 "C = dV xi^H phi");
  if (st != PX_OK) return st;
  return hip_check(ctx, px::launch_gemm_xc(fp32, n, n_phi, ng, xi, C, n_phi, -1.0, out, false, stream),
                   "out = -xi C");
}

px_status px_ptim_exchange_loop(px_context* ctx, const px_cell* cell, px_precision prec, int32_t n,
                                const void* xi, int32_t n_phi, const void* phi_n, int32_t n_iter,
                                double dt_alpha, void* phi_out, double* residuals,
                                hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  if (prec != PX_PREC_FP64 && prec != PX_PREC_FP32)
    return fail(ctx, PX_ERR_INVALID_ARG, "unknown precision %d", int(prec));
  if (!cell_ok(cell))
    return fail(ctx, PX_ERR_INVALID_ARG, "cell: edge lengths must be > 0 and grid sizes > 0");
  if (n <= 0 || n_phi <= 0 || n_iter <= 0)
    return fail(ctx, PX_ERR_INVALID_ARG, "n, n_phi and n_iter must be > 0");
  if (!xi || !phi_n || !phi_out || !residuals)
    return fail(ctx, PX_ERR_INVALID_ARG, "ptim_exchange_loop: null array argument");
  if (phi_out == phi_n || phi_out == xi)
    return fail(ctx, PX_ERR_INVALID_ARG, "ptim_exchange_loop: phi_out must not alias xi or phi_n");
  const LoopLayout l = loop_layout(cell, prec, n, n_phi);
  px_status st = need_ws(ctx, l.end);
  if (st != PX_OK) return st;
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_check(ctx, he, "hipSetDevice");
  const bool fp32 = prec == PX_PREC_FP32;
  const size_t ng = ngrid(cell);
  const size_t nel = size_t(n_phi) * ng;
  const double dV = cell->L[0] * cell->L[1] * cell->L[2] / double(ng);
  double* C = reinterpret_cast<double*>(ctx->ws + l.ap.C);
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
                                            nsplit, stream),
                   "C = dV xi^H mid");
    if (st != PX_OK) return st;
    st = hip_check(ctx, px::launch_gemm_xc(fp32, n, n_phi, ng, xi, C, n_phi, -1.0, y, false, stream),
                   "y = -xi C");
    if (st != PX_OK) return st;
    st = hip_check(ctx, px::launch_ptim_update(fp32, nel, phi_n, y, cur, nxt, dt_alpha, partial,
                                               residuals + k, stream),
                   "update");
    if (st != PX_OK) return st;
    cur = nxt;
  }
  return PX_OK;
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

px_status px_sync(px_context* ctx, hipStream_t stream) {
  if (!ctx) return PX_ERR_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_check(ctx, e, "hipStreamSynchronize");
  if (ctx->last_status) {
    int32_t s = 0;
    e = hipMemcpy(&s, ctx->last_status, sizeof s, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_check(ctx, e, "status readback");
    ctx->last_status = nullptr;
    if (s != 0) {
      ctx->latched = PX_ERR_NOT_POSITIVE_DEFINITE;
      fail(ctx, PX_ERR_NOT_POSITIVE_DEFINITE,
           "ace_build: -M is not positive definite (Cholesky breakdown at column %d)", s);
    }
  }
  return px_status(ctx->latched);
}

void px_clear_error(px_context* ctx) {
  if (!ctx) return;
  ctx->latched = PX_OK;
  ctx->err.clear();
}

}  // extern "C"
