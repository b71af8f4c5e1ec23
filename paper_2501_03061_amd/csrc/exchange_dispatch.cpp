// Size dispatch of the pair pipeline: the cubic grids with compiled plans.
#include "px_internal.hpp"

namespace px {

template <int N>
hipError_t launch_chunk_n(bool fp32, const ChunkArgs& a, int npairs, bool ex, bool store_v,
                          int p2cfg, hipStream_t s, hipEvent_t* ev, const ChunkArgs* tasks,
                          int ntasks, int max_ic);

#define PX_SIZES(X) X(16) X(24) X(32) X(40) X(48) X(60) X(64) X(72) X(80) X(96)

bool grid_supported(int n0, int n1, int n2) {
  if (n0 != n1 || n1 != n2) return false;
#define PX_CASE(N) if (n0 == N) return true;
  PX_SIZES(PX_CASE)
#undef PX_CASE
  return false;
}

hipError_t launch_chunk(bool fp32, int n, const ChunkArgs& a, int npairs, bool ex, int p2cfg,
                        hipStream_t s, hipEvent_t* ev) {
#define PX_CASE(N) \
  if (n == N)      \
    return launch_chunk_n<N>(fp32, a, npairs, ex, a.store_v != 0, p2cfg, s, ev, nullptr, 1, 0);
  PX_SIZES(PX_CASE)
#undef PX_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_chunk_tasks(bool fp32, int n, const ChunkArgs* tasks, int ntasks, int max_ic,
                              int max_pairs, bool ex, bool store_v, int p2cfg, hipStream_t s) {
  ChunkArgs dummy{};
#define PX_CASE(N)                                                                                  \
  if (n == N)                                                                                       \
    return launch_chunk_n<N>(fp32, dummy, max_pairs, ex, store_v, p2cfg, s, nullptr, tasks, ntasks, \
                             max_ic);
  PX_SIZES(PX_CASE)
#undef PX_CASE
  return hipErrorInvalidValue;
}

}  // namespace px
