// March kernels for FP64 plans in slab geometry.
#include "wk_march_impl.h"

namespace wk {
hipError_t launch_march_f64_slab(const MarchLaunch& L, int warm, int shape, int grid, size_t lds, hipStream_t s,
                              int* occ)
{
    return march_impl::launch<double, WK_SLAB>(L, warm, shape, grid, lds, s, occ);
}
}  // namespace wk
