// Plasma response march kernel: one response marched by its group of
// workgroups, or a batch of independent responses in one persistent launch
// (workgroups take tickets; a ticket is one workgroup of one instance's
// group).  Instantiated per precision and geometry by wk_march_*.hip.
//
// Per slice: two Heun stages, each = deposit of the xi-flux S -> psi solve ->
// gather psi -> deposit of the currents and the moments of d_xi J_r -> E_z
// quadrature -> B_theta tridiagonal solve -> gather -> stage derivative
// (WAKE paper, Section II A, Eqs. (1)-(7)).  Everything in the solves is
// double precision; in the mixed mode the per-particle arithmetic is float.
#pragma once

#include "wk_marcher.h"

namespace wk {
namespace march_impl {

// This workgroup's share of a response: the particles of cells
// [n_r rank / G, n_r (rank + 1) / G).
template <typename R>
__device__ __forceinline__ MarchDesc member_desc(const MarchDesc& full, int rank)
{
    const int G = full.group;
    const int c0 = (int)((int64_t)full.n_r * rank / G);
    const int c1 = (int)((int64_t)full.n_r * (rank + 1) / G);
    const int64_t p0 = (int64_t)c0 * full.ppc;
    MarchDesc d = full;
    d.p0 = full.p0 + p0;
    d.np = (int64_t)(c1 - c0) * full.ppc;
    d.x = full.x + p0;
    d.px = full.px + p0;
    d.y = full.y ? full.y + p0 : nullptr;
    d.py = full.py ? full.py + p0 : nullptr;
    d.d0 = (const R*)full.d0 + p0;
    d.w = (const R*)full.w + p0;
    return d;
}

template <typename R>
__device__ __forceinline__ dev::Group member_group(const MarchDesc& full, int rank)
{
    dev::Group grp;
    grp.G = full.group;
    grp.g = rank;
    grp.xbuf = full.xbuf;
    grp.ctr = full.gctr;
    grp.abort = full.counters + WK_CNT_PIPELINE_ABORT;
    return grp;
}

// SEL: group exchanges re-read only the partials not yet arrived (the batch,
// whose members take their tickets over time); a single response, whose
// members start together, reloads every partial on each try.
template <typename R, int GEOM, bool WARM, int T, int K, bool RES, bool BIG, int WPS, bool TRAJ = false,
          bool SEL = false>
__global__ __launch_bounds__(T, WPS) void k_march(MarchLaunch L)
{
    extern __shared__ double smem[];
    __shared__ int s_ticket;
    using M = dev::Marcher<R, GEOM, WARM, T, K, RES, BIG, SEL>;
    for (;;) {
        int inst = 0, rank = blockIdx.x;
        if (L.descs) {
            if (threadIdx.x == 0) s_ticket = (int)atomicAdd(L.next, 1u);
            __syncthreads();
            const int t = s_ticket;
            __syncthreads();
            if (t >= L.n_tickets) break;
            inst = L.tickets[2 * t];
            rank = L.tickets[2 * t + 1];
        }
        const MarchDesc full = L.descs ? L.descs[inst] : L.one;
        MarchDesc d = member_desc<R>(full, rank);
        d.grow = BIG ? L.grow + (int64_t)blockIdx.x * BIG_ROWS * L.grow_stride : nullptr;
        void* pconst = BIG ? nullptr : (void*)(smem + NUM_ROWS * lds_stride(full.n_r + 1));
        M m(d, smem, pconst, member_group<R>(full, rank), rank == 0, true);
        if constexpr (TRAJ)
            m.run_traj();
        else
            m.run();
        if (!L.descs) break;
        __syncthreads();
    }
}

template <typename R, int GEOM, bool WARM, int SH>
hipError_t go(const MarchLaunch& L, int grid, size_t lds, hipStream_t s, int* occ)
{
    constexpr ShapeInfo S = kShapes[SH];
    // large-grid resident particles keep D0 and w in registers (float only)
    if constexpr (S.big && S.resident && sizeof(R) == 8) {
        return hipErrorInvalidValue;
    } else {
        auto kern = k_march<R, GEOM, WARM, S.threads, S.kp, S.resident, S.big, S.waves_per_simd>;
        // batches (not the large-grid or single-workgroup shapes, which a
        // batch does not use) with selective re-reads
        if constexpr (!S.big && S.kp <= 8) {
            if (L.descs) kern = k_march<R, GEOM, WARM, S.threads, S.kp, S.resident, S.big, S.waves_per_simd, false, true>;
        }
        if (L.one.traj) {
            // particle radii recorded: an FP64 single response only
            if constexpr (sizeof(R) == 8) {
                if (L.descs || occ) return hipErrorInvalidValue;
                kern = k_march<R, GEOM, WARM, S.threads, S.kp, S.resident, S.big, S.waves_per_simd, true>;
            } else {
                return hipErrorInvalidValue;
            }
        }
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        if (occ) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, S.threads, lds);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(S.threads), lds, s, L);
        return hipGetLastError();
    }
}

template <typename R, int GEOM, bool WARM>
hipError_t go_shape(const MarchLaunch& L, int shape, int grid, size_t lds, hipStream_t s, int* occ)
{
    switch (shape) {
    case SH_256_4: return go<R, GEOM, WARM, SH_256_4>(L, grid, lds, s, occ);
    case SH_512_8: return go<R, GEOM, WARM, SH_512_8>(L, grid, lds, s, occ);
    case SH_512_4: return go<R, GEOM, WARM, SH_512_4>(L, grid, lds, s, occ);
    case SH_512_16: return go<R, GEOM, WARM, SH_512_16>(L, grid, lds, s, occ);
    case SH_1024_8: return go<R, GEOM, WARM, SH_1024_8>(L, grid, lds, s, occ);
    case SH_1024_STREAM: return go<R, GEOM, WARM, SH_1024_STREAM>(L, grid, lds, s, occ);
    case SH_BIG_512_8: return go<R, GEOM, WARM, SH_BIG_512_8>(L, grid, lds, s, occ);
    case SH_BIG_STREAM: return go<R, GEOM, WARM, SH_BIG_STREAM>(L, grid, lds, s, occ);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int GEOM>
hipError_t launch(const MarchLaunch& L, int warm, int shape, int grid, size_t lds, hipStream_t s, int* occ)
{
    return warm ? go_shape<R, GEOM, true>(L, shape, grid, lds, s, occ)
                : go_shape<R, GEOM, false>(L, shape, grid, lds, s, occ);
}

}  // namespace march_impl
}  // namespace wk
