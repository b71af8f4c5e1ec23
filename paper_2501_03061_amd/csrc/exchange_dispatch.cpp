// Size dispatch of the pair pipeline: the cubic grids with compiled plans
// (per-size tuned configurations) and the non-cubic grids (configurations
// from the plans alone).
#include "px_internal.hpp"

namespace px {

template <int N>
hipError_t launch_chunk_n(bool fp32, const ChunkArgs& a, int npairs, bool ex, bool store_v,
                          int p2cfg, hipStream_t s, hipEvent_t* ev, const ChunkArgs* tasks,
                          int ntasks, int max_ic);
template <int N0, int N1, int N2>
hipError_t launch_chunk_shape(bool fp32, const ChunkArgs& a, int npairs, bool ex, bool store_v,
                              hipStream_t s, hipEvent_t* ev, const ChunkArgs* tasks, int ntasks,
                              int max_ic);

#define PX_SIZES(X) X(16) X(24) X(32) X(40) X(48) X(60) X(64) X(72) X(80) X(96)
#define PX_SHAPES(X) X(60, 60, 90) X(60, 90, 120)

bool grid_supported(int n0, int n1, int n2) {
#define PX_SHAPE_CASE(A, B, C) if (n0 == A && n1 == B && n2 == C) return true;
  PX_SHAPES(PX_SHAPE_CASE)
#undef PX_SHAPE_CASE
  if (n0 != n1 || n1 != n2) return false;
#define PX_CASE(N) if (n0 == N) return true;
  PX_SIZES(PX_CASE)
#undef PX_CASE
  return false;
}

bool grid_cubic(int n0, int n1, int n2) { return n0 == n1 && n1 == n2; }

hipError_t launch_chunk(bool fp32, const int* n, const ChunkArgs& a, int npairs, bool ex, int p2cfg,
                        hipStream_t s, hipEvent_t* ev) {
#define PX_SHAPE_CASE(A, B, C)                   \
  if (n[0] == A && n[1] == B && n[2] == C)       \
    return launch_chunk_shape<A, B, C>(fp32, a, npairs, ex, a.store_v != 0, s, ev, nullptr, 1, 0);
  PX_SHAPES(PX_SHAPE_CASE)
#undef PX_SHAPE_CASE
  if (!grid_cubic(n[0], n[1], n[2])) return hipErrorInvalidValue;
#define PX_CASE(N) \
  if (n[0] == N)   \
    return launch_chunk_n<N>(fp32, a, npairs, ex, a.store_v != 0, p2cfg, s, ev, nullptr, 1, 0);
  PX_SIZES(PX_CASE)
#undef PX_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_chunk_tasks(bool fp32, const int* n, const ChunkArgs* tasks, int ntasks, int max_ic,
                              int max_pairs, bool ex, bool store_v, int p2cfg, hipStream_t s) {
  ChunkArgs dummy{};
#define PX_SHAPE_CASE(A, B, C)                                                                    \
  if (n[0] == A && n[1] == B && n[2] == C)                                                        \
    return launch_chunk_shape<A, B, C>(fp32, dummy, max_pairs, ex, store_v, s, nullptr, tasks, ntasks, \
                                       max_ic);
  PX_SHAPES(PX_SHAPE_CASE)
#undef PX_SHAPE_CASE
  if (!grid_cubic(n[0], n[1], n[2])) return hipErrorInvalidValue;
#define PX_CASE(N)                                                                                  \
  if (n[0] == N)                                                                                    \
    return launch_chunk_n<N>(fp32, dummy, max_pairs, ex, store_v, p2cfg, s, nullptr, tasks, ntasks, \
                             max_ic);
  PX_SIZES(PX_CASE)
#undef PX_CASE
  return hipErrorInvalidValue;
}

}  // namespace px
