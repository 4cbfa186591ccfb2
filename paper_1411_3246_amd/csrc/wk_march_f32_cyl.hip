// March kernels for mixed-precision plans in cylindrical geometry.
#include "wk_march_impl.h"

namespace wk {
hipError_t launch_march_f32_cyl(const MarchLaunch& L, int warm, int shape, int grid, size_t lds, hipStream_t s,
                              int* occ)
{
    return march_impl::launch<float, WK_CYL>(L, warm, shape, grid, lds, s, occ);
}
}  // namespace wk
