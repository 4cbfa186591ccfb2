// Host side of the march and cycle launches: kernel shapes, LDS sizes and the
// dispatch to the kernels instantiated per precision and geometry
// (wk_march_*.hip, wk_cycle_*.hip).
#include "wk_internal.h"

namespace wk {

hipError_t launch_cycle_f64_cyl(const CycleDesc& c, int warm, int shape, int grid, size_t lds, hipStream_t s, int* occ);
hipError_t launch_cycle_f64_slab(const CycleDesc& c, int warm, int shape, int grid, size_t lds, hipStream_t s, int* occ);
hipError_t launch_cycle_f32_cyl(const CycleDesc& c, int warm, int shape, int grid, size_t lds, hipStream_t s, int* occ);
hipError_t launch_cycle_f32_slab(const CycleDesc& c, int warm, int shape, int grid, size_t lds, hipStream_t s, int* occ);

namespace {
constexpr size_t kMaxLds = 159 * 1024;  // leaves room for static LDS

bool regs_for_constants(const ShapeInfo& S, int prec)
{
    return S.resident && (S.kp <= 4 || (S.kp <= 8 && prec != WK_FP64));
}
}  // namespace

bool march_needs_global_rows(int n_nodes) { return march_lds_bytes(n_nodes, 0) > kMaxLds; }

size_t shape_lds_bytes(int shape, int n_nodes, int prec)
{
    const ShapeInfo& S = kShapes[shape];
    if (S.big) return big_lds_bytes(n_nodes);
    size_t lds = march_lds_bytes(n_nodes, S.threads);
    const size_t rs = prec == WK_FP64 ? sizeof(double) : sizeof(float);
    if (S.resident && !regs_for_constants(S, prec)) lds += 2 * (size_t)S.threads * S.kp * rs;
    return lds;
}

int pick_shape(int64_t np, int threads, int n_nodes, int prec, int group)
{
    if (march_needs_global_rows(n_nodes))
        return (prec != WK_FP64 && np <= (int64_t)kShapes[SH_BIG_512_8].threads * kShapes[SH_BIG_512_8].kp)
                   ? SH_BIG_512_8
                   : SH_BIG_STREAM;
    static const int order[] = {SH_256_4, SH_512_4, SH_512_8, SH_512_16, SH_1024_8};
    for (int sh : order) {
        const ShapeInfo& S = kShapes[sh];
        if (S.threads < threads) continue;
        if (group > 1 && S.kp > 8) continue;
        if (np > (int64_t)S.threads * S.kp) continue;
        if (shape_lds_bytes(sh, n_nodes, prec) > kMaxLds) continue;
        return sh;
    }
    return SH_1024_STREAM;
}

hipError_t launch_march(const MarchLaunch& L, int prec, int geom, int warm, int shape, int grid, int max_nodes,
                        hipStream_t s)
{
    const size_t lds = shape_lds_bytes(shape, max_nodes, prec);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    if (prec == WK_FP64)
        return geom == WK_CYL ? launch_march_f64_cyl(L, warm, shape, grid, lds, s, nullptr)
                              : launch_march_f64_slab(L, warm, shape, grid, lds, s, nullptr);
    return geom == WK_CYL ? launch_march_f32_cyl(L, warm, shape, grid, lds, s, nullptr)
                          : launch_march_f32_slab(L, warm, shape, grid, lds, s, nullptr);
}

int march_occupancy(int prec, int geom, int warm, int shape, int max_nodes)
{
    const size_t lds = shape_lds_bytes(shape, max_nodes, prec);
    if (lds > kMaxLds) return 0;
    MarchLaunch L{};
    int occ = 0;
    hipError_t e;
    if (prec == WK_FP64)
        e = geom == WK_CYL ? launch_march_f64_cyl(L, warm, shape, 0, lds, nullptr, &occ)
                           : launch_march_f64_slab(L, warm, shape, 0, lds, nullptr, &occ);
    else
        e = geom == WK_CYL ? launch_march_f32_cyl(L, warm, shape, 0, lds, nullptr, &occ)
                           : launch_march_f32_slab(L, warm, shape, 0, lds, nullptr, &occ);
    return e == hipSuccess ? occ : 0;
}

size_t cycle_lds_bytes(int shape, int n_nodes, int prec)
{
    const size_t lds = shape_lds_bytes(shape, n_nodes, prec);
    return kShapes[shape].big ? lds : lds + (size_t)kCycleRing * lds_stride(n_nodes) * sizeof(double);
}

hipError_t launch_cycle(const CycleDesc& c, int prec, int shape, int grid, hipStream_t s)
{
    const size_t lds = cycle_lds_bytes(shape, c.base.n_r + 1, prec);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    const int warm = c.base.warm;
    if (prec == WK_FP64)
        return c.base.geom == WK_CYL ? launch_cycle_f64_cyl(c, warm, shape, grid, lds, s, nullptr)
                                     : launch_cycle_f64_slab(c, warm, shape, grid, lds, s, nullptr);
    return c.base.geom == WK_CYL ? launch_cycle_f32_cyl(c, warm, shape, grid, lds, s, nullptr)
                                 : launch_cycle_f32_slab(c, warm, shape, grid, lds, s, nullptr);
}

bool lds_fits(size_t bytes) { return bytes <= kMaxLds; }

int cycle_occupancy(int prec, int geom, int warm, int shape, int n_nodes)
{
    const size_t lds = cycle_lds_bytes(shape, n_nodes, prec);
    if (lds > kMaxLds) return 0;
    CycleDesc c{};
    int occ = 0;
    hipError_t e;
    if (prec == WK_FP64)
        e = geom == WK_CYL ? launch_cycle_f64_cyl(c, warm, shape, 0, lds, nullptr, &occ)
                           : launch_cycle_f64_slab(c, warm, shape, 0, lds, nullptr, &occ);
    else
        e = geom == WK_CYL ? launch_cycle_f32_cyl(c, warm, shape, 0, lds, nullptr, &occ)
                           : launch_cycle_f32_slab(c, warm, shape, 0, lds, nullptr, &occ);
    return e == hipSuccess ? occ : 0;
}

}  // namespace wk
