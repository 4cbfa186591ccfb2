// Plasma response march: one persistent workgroup per instance.
//
// Each workgroup keeps the radial grid of its instance in LDS and marches all
// slices of the xi window without leaving the kernel.  Per slice: two Heun
// stages, each = deposit of the xi-flux S -> psi solve -> gather psi ->
// deposit of the currents and the moments of d_xi J_r -> E_z quadrature ->
// B_theta tridiagonal solve -> gather -> stage derivative (WAKE paper,
// Section II A, Eqs. (1)-(7)).
//
// Particles: each thread owns K consecutive particles of a tile of
// threads * K; when the instance fits in one tile the particles stay in
// registers for the whole march, otherwise tiles stream through registers.
// Deposits: consecutive particles of a thread that hit the same cell are
// summed in registers, then added to double LDS rows with LDS atomics.
// Solves: psi and E_z by one wavefront with DPP prefix scans over rounds of
// 64 nodes (no workgroup barrier), B_theta by parallel cyclic reduction over
// the whole workgroup.  Everything in the solves is double precision;
// reciprocals there are refined to double accuracy.  In the mixed mode the
// per-particle arithmetic uses the hardware float reciprocal and square root.
#include <algorithm>

#include "wk_marcher.h"

namespace wk {
namespace {

using dev::Marcher;

template <typename R, int GEOM, bool WARM, int T, int K, bool RES, bool BIG = false>
__global__ __launch_bounds__(T) void k_march_one(MarchDesc d)
{
    extern __shared__ double smem[];
    Marcher<R, GEOM, WARM, K, RES, BIG, T> m(d, smem, smem + NUM_ROWS * lds_stride(d.n_r + 1));
    m.run();
}

// Persistent batched march: workgroups take instances from a queue (longest
// first).  With RES, an instance whose particles fit T * K registers stays
// resident; larger instances stream their particles in tiles.
template <typename R, int GEOM, bool WARM, int T, int K, bool RES>
__global__ __launch_bounds__(T) void k_march_batch(const MarchDesc* __restrict__ descs, int n,
                                                   unsigned int* next)
{
    extern __shared__ double smem[];
    __shared__ int inst;
    for (;;) {
        if (threadIdx.x == 0) inst = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int i = inst;
        __syncthreads();
        if (i >= n) break;
        const MarchDesc d = descs[i];
        if (RES && d.np <= (int64_t)T * K) {
            Marcher<R, GEOM, WARM, K, true, false, T> m(d, smem, smem + NUM_ROWS * lds_stride(d.n_r + 1));
            m.run();
        } else {
            Marcher<R, GEOM, WARM, K, false, false, T> m(d, smem, smem + NUM_ROWS * lds_stride(d.n_r + 1));
            m.run();
        }
        __syncthreads();
    }
}

// Particles per thread: up to 8192 particles stay in registers at 512 and
// 1024 threads per workgroup.
constexpr int tile_for(int T) { return T >= 1024 ? 8 : 16; }
constexpr size_t kMaxLds = 159 * 1024;  // leaves room for static LDS

// Large grid (node rows beyond LDS): 1024 threads, particles streamed, the
// field and solver rows in the descriptor's global rows.
template <typename R, int GEOM, bool WARM>
hipError_t launch_big(const MarchDesc& d, hipStream_t s)
{
    if (!d.grow) return hipErrorInvalidValue;
    const size_t lds = big_lds_bytes(d.n_r + 1);
    auto kern = k_march_one<R, GEOM, WARM, 1024, tile_for(1024), false, true>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(1), dim3(1024), lds, s, d);
    return hipGetLastError();
}

template <typename R, int GEOM, bool WARM, int T>
hipError_t launch_one_t(const MarchDesc& d, hipStream_t s)
{
    if (march_lds_bytes(d.n_r + 1, T) > kMaxLds) return launch_big<R, GEOM, WARM>(d, s);
    const size_t lds = march_lds_bytes(d.n_r + 1, T);
    constexpr int kK = tile_for(T);
    // resident particles per thread (the kernel's own ceil(np / T))
    const int64_t kr = std::min<int64_t>(kK, (d.np + T - 1) / T);
    const size_t lds_res = lds + 2 * (size_t)T * kr * sizeof(R);
    // the whole instance stays on chip when its D0 and w fit in LDS
    const bool res = d.np <= (int64_t)T * kK && lds_res <= kMaxLds;
    if (res) {
        auto kern = k_march_one<R, GEOM, WARM, T, kK, true>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_res);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(1), dim3(T), lds_res, s, d);
    } else {
        auto kern = k_march_one<R, GEOM, WARM, T, kK, false>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(1), dim3(T), lds, s, d);
    }
    return hipGetLastError();
}

template <typename R, int GEOM, bool WARM, int T>
hipError_t launch_batch_t(const MarchDesc* descs, int n, int max_nodes, bool res, int grid, unsigned int* next,
                          hipStream_t s)
{
    size_t lds = march_lds_bytes(max_nodes, T);
    constexpr int kK = tile_for(T);
    if (res && lds + 2 * (size_t)T * kK * sizeof(R) > kMaxLds) res = false;
    if (res) lds += 2 * (size_t)T * kK * sizeof(R);
    if (res) {
        auto kern = k_march_batch<R, GEOM, WARM, T, kK, true>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(T), lds, s, descs, n, next);
    } else {
        auto kern = k_march_batch<R, GEOM, WARM, T, kK, false>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(T), lds, s, descs, n, next);
    }
    return hipGetLastError();
}

template <typename R, int GEOM, bool WARM>
hipError_t launch_one_w(const MarchDesc& d, int threads, hipStream_t s)
{
    switch (threads) {
    case 256: return launch_one_t<R, GEOM, WARM, 256>(d, s);
    case 512: return launch_one_t<R, GEOM, WARM, 512>(d, s);
    default: return launch_one_t<R, GEOM, WARM, 1024>(d, s);
    }
}

template <typename R, int GEOM, bool WARM>
hipError_t launch_batch_w(const MarchDesc* descs, int n, int max_nodes, int threads, bool res, int grid,
                          unsigned int* next, hipStream_t s)
{
    switch (threads) {
    case 256: return launch_batch_t<R, GEOM, WARM, 256>(descs, n, max_nodes, res, grid, next, s);
    case 512: return launch_batch_t<R, GEOM, WARM, 512>(descs, n, max_nodes, res, grid, next, s);
    default: return launch_batch_t<R, GEOM, WARM, 1024>(descs, n, max_nodes, res, grid, next, s);
    }
}

template <typename R>
hipError_t launch_one_r(const MarchDesc& d, int threads, hipStream_t s)
{
    if (d.geom == WK_CYL)
        return d.warm ? launch_one_w<R, WK_CYL, true>(d, threads, s) : launch_one_w<R, WK_CYL, false>(d, threads, s);
    return d.warm ? launch_one_w<R, WK_SLAB, true>(d, threads, s) : launch_one_w<R, WK_SLAB, false>(d, threads, s);
}

template <typename R>
hipError_t launch_batch_r(const MarchDesc* descs, int n, int max_nodes, int geom, int warm, int threads, bool res,
                          int grid, unsigned int* next, hipStream_t s)
{
    if (geom == WK_CYL)
        return warm ? launch_batch_w<R, WK_CYL, true>(descs, n, max_nodes, threads, res, grid, next, s)
                    : launch_batch_w<R, WK_CYL, false>(descs, n, max_nodes, threads, res, grid, next, s);
    return warm ? launch_batch_w<R, WK_SLAB, true>(descs, n, max_nodes, threads, res, grid, next, s)
                : launch_batch_w<R, WK_SLAB, false>(descs, n, max_nodes, threads, res, grid, next, s);
}

}  // namespace

int march_tile(int threads) { return tile_for(threads); }
bool march_needs_global_rows(int n_nodes) { return march_lds_bytes(n_nodes, 0) > kMaxLds; }

hipError_t launch_march(const MarchDesc& d, int prec, MarchShape shape, hipStream_t stream)
{
    return prec == WK_FP64 ? launch_one_r<double>(d, shape.threads, stream)
                           : launch_one_r<float>(d, shape.threads, stream);
}

hipError_t launch_march_batch(const MarchDesc* d_descs, int n, int max_nodes, int geom, int warm, int prec,
                              MarchShape shape, bool resident, int grid, unsigned int* d_next, hipStream_t stream)
{
    return prec == WK_FP64
               ? launch_batch_r<double>(d_descs, n, max_nodes, geom, warm, shape.threads, resident, grid, d_next, stream)
               : launch_batch_r<float>(d_descs, n, max_nodes, geom, warm, shape.threads, resident, grid, d_next, stream);
}

}  // namespace wk
