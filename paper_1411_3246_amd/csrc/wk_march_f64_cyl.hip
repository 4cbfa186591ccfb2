// March kernels for FP64 plans in cylindrical geometry.
#include "wk_march_impl.h"

namespace wk {
hipError_t launch_march_f64_cyl(const MarchLaunch& L, int warm, int shape, int grid, size_t lds, hipStream_t s,
                              int* occ)
{
    return march_impl::launch<double, WK_CYL>(L, warm, shape, grid, lds, s, occ);
}
}  // namespace wk
