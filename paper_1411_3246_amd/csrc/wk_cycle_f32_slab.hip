// Pipelined-cycle kernels for mixed-precision plans in slab geometry.
#include "wk_cycle_impl.h"

namespace wk {
hipError_t launch_cycle_f32_slab(const CycleDesc& c, int warm, int shape, int grid, size_t lds, hipStream_t s,
                              int* occ)
{
    return cycle_impl::launch<float, WK_SLAB>(c, warm, shape, grid, lds, s, occ);
}
}  // namespace wk
