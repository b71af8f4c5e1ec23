// One translation unit per grid size: compiled with -DPX_N=<n> so that the
// sizes build in parallel.
#include "exchange_kernels.hpp"

#ifndef PX_N
#error "PX_N (cubic grid size) must be defined"
#endif

namespace px {
template hipError_t launch_chunk_n<PX_N>(bool, const ChunkArgs&, int, bool, bool, int, hipStream_t,
                                         hipEvent_t*, const ChunkArgs*, int, int);
}
