// One translation unit per non-cubic grid: compiled with -DPX_S0=<n0>
// -DPX_S1=<n1> -DPX_S2=<n2>.
#include "exchange_kernels.hpp"

#if !defined(PX_S0) || !defined(PX_S1) || !defined(PX_S2)
#error "PX_S0, PX_S1, PX_S2 (grid lengths) must be defined"
#endif

namespace px {
template hipError_t launch_chunk_shape<PX_S0, PX_S1, PX_S2>(bool, const ChunkArgs&, int, bool, bool,
                                                            hipStream_t, hipEvent_t*,
                                                            const ChunkArgs*, int, int);
}
