// Internal declarations shared by the HIP translation units of libwake.
// Not part of the public ABI (include/wake.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wake.h"

namespace wk {

constexpr double kPi = 3.14159265358979323846;

// Per-instance description of one plasma response, read by the march kernel.
struct MarchDesc {
    int32_t geom;        // WK_CYL / WK_SLAB
    int32_t warm;        // 1: transverse momenta / p_y present
    int32_t n_r;         // cells; nodes 0..n_r
    int32_t n_xi;        // stored slices
    int64_t np;          // macroparticles in a slice
    double r_max, h, dxi, d_min;
    double* x;
    double* y;
    double* px;
    double* py;
    const void* d0;      // real[np]
    const void* w;       // real[np]
    const double* nion;  // double[n_r+1]
    const double* jb;    // double[n_xi][n_r+1]
    void* fields;        // real[4][n_xi][n_r+1]
    void* fk;            // real[4][np] stage-1 derivative scratch
    unsigned long long* counters;
    int64_t cost;        // np * n_xi (scheduling weight)
};

// LDS rows used by the march kernel (each of `stride` doubles).
enum MarchRow {
    ROW_S = 0, ROW_JR, ROW_JZ, ROW_M1, ROW_M2, ROW_M3, ROW_M4, ROW_M5,
    ROW_PSI, ROW_DPSI, ROW_EZ, ROW_B, ROW_NION,
    ROW_PA, ROW_PB, ROW_PC, ROW_PD,   // tridiagonal buffer 0
    NUM_ROWS
};

inline int lds_stride(int n_nodes) { return (n_nodes + 1) & ~1; }
inline size_t march_lds_bytes(int n_nodes, int threads)
{
    return (size_t)NUM_ROWS * lds_stride(n_nodes) * sizeof(double) + (size_t)(threads / 64 + 2) * sizeof(double);
}

// Launch shapes (chosen by the plan).
struct MarchShape {
    int threads;   // workgroup size
    int tile;      // particles per thread per tile (compile-time variant)
};

hipError_t launch_march(const MarchDesc& d, int prec, MarchShape shape, hipStream_t stream);
hipError_t launch_march_batch(const MarchDesc* d_descs, int n, int max_nodes, int geom, int warm,
                              int prec, MarchShape shape, int grid, unsigned int* d_next,
                              hipStream_t stream);

// Beam / loader kernels (wk_beam.hip)
struct GridDesc {
    int32_t geom, n_r, n_xi;
    double r_max, h, xi_min, dxi;
};

hipError_t launch_init_plasma(const GridDesc& g, int ppc, double u_th, double n0, int prec,
                              const wk_plasma_bufs& b, const double* draws, hipStream_t s);
hipError_t launch_init_beam(const GridDesc& g, const wk_problem& p, const wk_beam_bufs& b,
                            const double* draws, hipStream_t s);
hipError_t launch_beam_current_analytic(const GridDesc& g, const wk_problem& p, double* jb,
                                        hipStream_t s);
hipError_t launch_beam_current(const GridDesc& g, int64_t n_beam, const wk_beam_bufs& b,
                               double* jb, void* ws, unsigned long long* counters,
                               hipStream_t s);
hipError_t launch_beam_push(const GridDesc& g, int64_t n_beam, const wk_beam_bufs& b,
                            const void* fields, int prec, int n_steps, double dt,
                            unsigned long long* counters, hipStream_t s);
hipError_t launch_mean_gain(int64_t n_beam, const wk_beam_bufs& b, int which, double* out,
                            void* ws, hipStream_t s);
hipError_t launch_ez_peak(const GridDesc& g, const void* fields, int prec, double xi_from,
                          double* out, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
hipError_t launch_zero_u32(unsigned int* p, int64_t n, hipStream_t s);

// Workspace layout of the beam binning (bytes, 256-aligned pieces).
size_t beam_ws_bytes(int n_xi, int64_t n_beam);

}  // namespace wk
