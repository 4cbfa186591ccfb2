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
    int64_t np;          // macroparticles in a slice (n_r * ppc)
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
    unsigned long long* counters;
    int64_t cost;        // np * n_xi (scheduling weight)
    double* grow;        // large grids: global node rows, BIG_ROWS x stride doubles per workgroup
    int32_t ppc;         // macroparticles per cell
    int32_t group;       // workgroups that march this response together (1..kMaxGroup)
    double* xbuf;        // group > 1: partial deposit rows, [2][group][kXRows][stride] doubles (zeroed)
    unsigned int* gctr;  // group > 1: arrival counter of the group barrier (own 256-byte line)
    int64_t p0;          // index of this descriptor's first particle in the response
    double* traj;        // optional: radius of every traj_stride-th particle per slice,
    int64_t traj_n;      //   [n_xi][traj_n] doubles, traj_n = ceil(np_response / traj_stride)
    int32_t traj_stride;
};

// Largest number of workgroups marching one response.
constexpr int kMaxGroup = 16;
// Deposit rows exchanged between the workgroups of a group (S, J_r, J_z, M1..M5).
constexpr int kXRows = 8;
// Spacing of the group counters (unsigned ints): one 256-byte line each.
constexpr int kCtrPad = 64;

// LDS rows used by the march kernel (each of `stride` doubles): the deposit
// rows, the field rows of both Heun stages, the ion density and the scratch
// of the tridiagonal solve.
enum MarchRow {
    ROW_S = 0, ROW_JR, ROW_JZ, ROW_M1, ROW_M2, ROW_M3, ROW_M4, ROW_M5,
    ROW_PSI1, ROW_DPSI1, ROW_B1, ROW_PSI2, ROW_DPSI2, ROW_B2, ROW_EZ, ROW_NION,
    ROW_TU, ROW_TV, ROW_TW,
    NUM_ROWS
};

__host__ __device__ inline int lds_stride(int n_nodes) { return (n_nodes + 1) & ~1; }
// Large grids keep the deposit rows ROW_S..ROW_M5 in LDS and the others in
// global memory.
constexpr int BIG_LDS_ROWS = ROW_PSI1;
constexpr int BIG_ROWS = NUM_ROWS - ROW_PSI1;
inline size_t big_lds_bytes(int n_nodes) { return (size_t)BIG_LDS_ROWS * lds_stride(n_nodes) * sizeof(double); }
inline size_t big_rows_bytes(int n_nodes) { return (size_t)BIG_ROWS * lds_stride(n_nodes) * sizeof(double); }
inline size_t march_lds_bytes(int n_nodes, int /*threads*/)
{
    return (size_t)NUM_ROWS * lds_stride(n_nodes) * sizeof(double);
}

// Kernel shapes of the march and of the pipelined cycle: workgroup size,
// particles per thread (resident: held in registers for the whole march;
// streamed: tiles of T * kp particles), and the large-grid variant whose
// field rows live in global memory.
struct ShapeInfo {
    int threads, kp;
    bool resident, big;
    int waves_per_simd;   // occupancy the kernel is compiled for (registers)
};
enum ShapeId {
    SH_256_4 = 0, SH_512_4, SH_512_8, SH_512_16, SH_1024_8, SH_1024_STREAM, SH_BIG_512_8, SH_BIG_STREAM, NUM_SHAPES
};
// The 256-thread shape is compiled for two workgroups per compute unit, so
// that one workgroup's field solves and particle passes run while the other
// waits at a group exchange.
// Large grids use 512 threads: their node rows take most of the LDS, and
// the 256-register budget of 512-thread workgroups keeps their kernels
// free of heavy spilling.
// The 16-particle shape marches single workgroups only (group 1): it is
// compiled without the group exchange, which it could not afford in
// registers.
constexpr ShapeInfo kShapes[NUM_SHAPES] = {
    {256, 4, true, false, 2}, {512, 4, true, false, 2}, {512, 8, true, false, 2}, {512, 16, true, false, 2},
    {1024, 8, true, false, 4}, {1024, 8, false, false, 4}, {512, 8, true, true, 2}, {512, 8, false, true, 2},
};
// LDS bytes of a shape for grids of up to n_nodes nodes (rows, plus the
// resident D0 / w slots when they are not kept in registers).
size_t shape_lds_bytes(int shape, int n_nodes, int prec);
// true when the node rows of a grid exceed LDS (large-grid shapes)
bool march_needs_global_rows(int n_nodes);
// The shape for `np` particles per workgroup on a grid of n_nodes nodes: the
// smallest resident shape of at least `threads` threads that holds them and
// fits LDS (for a group of more than one workgroup, one with the exchange),
// else a streamed one.
int pick_shape(int64_t np, int threads, int n_nodes, int prec, int group);

// One launch of the march kernel: a single response (descs == nullptr; its
// `group` workgroups are the grid) or a batch (workgroups take tickets; each
// ticket is one workgroup of one instance's group).
struct MarchLaunch {
    const MarchDesc* descs;   // batch: device array of instances
    MarchDesc one;            // single response
    const int* tickets;       // batch: [n_tickets][2] = (instance, rank)
    int n_tickets;
    unsigned int* next;       // batch: ticket counter (zeroed)
    double* grow;             // large grids: grid * BIG_ROWS * grow_stride doubles
    int grow_stride;
};
hipError_t launch_march(const MarchLaunch& L, int prec, int geom, int warm, int shape, int grid, int max_nodes,
                        hipStream_t s);
// workgroups of a march shape resident per compute unit (0: does not fit)
int march_occupancy(int prec, int geom, int warm, int shape, int max_nodes);
// per-(precision, geometry) launchers (wk_march_*.hip)
// (occ != nullptr: only report the resident workgroups per compute unit)
hipError_t launch_march_f64_cyl(const MarchLaunch& L, int warm, int shape, int grid, size_t lds, hipStream_t s, int* occ);
hipError_t launch_march_f64_slab(const MarchLaunch& L, int warm, int shape, int grid, size_t lds, hipStream_t s, int* occ);
hipError_t launch_march_f32_cyl(const MarchLaunch& L, int warm, int shape, int grid, size_t lds, hipStream_t s, int* occ);
hipError_t launch_march_f32_slab(const MarchLaunch& L, int warm, int shape, int grid, size_t lds, hipStream_t s, int* occ);

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
hipError_t launch_gain_hist(int64_t n_beam, const wk_beam_bufs& b, int which, int n_bins, double lo, double hi,
                            unsigned long long* hist, hipStream_t s);
hipError_t launch_ez_peak(const GridDesc& g, const void* fields, int prec, double xi_from,
                          double* out, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
hipError_t launch_zero_u32(unsigned int* p, int64_t n, hipStream_t s);

// Workspace layout of the beam binning (bytes, 256-aligned pieces).
size_t beam_ws_bytes(int n_xi, int64_t n_beam);

// Pipelined quasi-static cycle (wk_cycle_impl.h).  The beam is split into
// `group` contiguous subsets; workgroup g of every response handles subset g
// and keeps its own xi bins of it.
struct CycleDesc {
    MarchDesc base;                  // plasma template (loaded), constants, counters, group
    wk_beam_bufs beam;
    GridDesc grid;
    unsigned int* bin_start;         // [2][group][n_xi + 2] per-subset bin starts (slot 0 filled
                                     // by launch_beam_bins_split); bin n_xi: outside the window
    unsigned int* order;             // [2][n_beam] subset-relative indices sorted by bin
    int64_t n_beam;
    unsigned int* progress;          // [n_steps] stored slices per response (zeroed)
    unsigned int* ticket;            // zeroed
    unsigned long long* abort_flag;  // counter slot, zeroed
    double* plasma_ws;               // streamed particles: grid * 4 * (largest subset) doubles
    double* big_rows;                // large grids: grid * BIG_ROWS node rows
    double* xbuf;                    // group > 1: [n_steps][2][group][kXRows][stride] doubles (zeroed)
    unsigned int* gctr;              // group > 1: [n_steps + 1] counters, kCtrPad apart (zeroed)
    void* ring;                      // 2 field slots
    int64_t slot_elems;
    int n_steps;
    double dt;
};
// Rows of beam current the cycle keeps in LDS (grids whose rows fit LDS).
constexpr int kCycleRing = 4;
// LDS bytes of the cycle kernel of a shape (the march rows plus the ring).
size_t cycle_lds_bytes(int shape, int n_nodes, int prec);
// true when `bytes` of dynamic LDS fit one workgroup
bool lds_fits(size_t bytes);
hipError_t launch_cycle(const CycleDesc& c, int prec, int shape, int grid, hipStream_t s);
int cycle_occupancy(int prec, int geom, int warm, int shape, int n_nodes);
// Bin each of `group` contiguous beam subsets by xi cell: bin_start gets
// [group][n_xi + 2] subset-relative starts, order the subset-relative indices.
// count/fill: scratch of group * (n_xi + 1) entries each.
hipError_t launch_beam_bins_split(const GridDesc& g, int64_t n_beam, int group, const wk_beam_bufs& b,
                                  unsigned int* count, unsigned int* bin_start, unsigned int* fill,
                                  unsigned int* order, hipStream_t s);

// Reverse-mode derivative of the witness gain (wk_adjoint.hip).
struct GradDesc {
    MarchDesc march;             // FP64 plasma of the forward (constants d0, w)
    GridDesc grid;
    wk_beam_bufs beam;
    int64_t n_beam, n_drive;
    int n_steps, every, threads;             // threads: workgroup size of the reverse march
    double dt;
    double n_d, sigma_r, sigma_zd, u_th;     // the parameters
    int prec;                    // WK_FP64 or WK_MIXED (float fields and plasma constants)
    const void* fields;          // real[4][n_xi][N1] of the forward
    double* d0_f64;              // mixed: [np] plasma D0 and w as double (scratch)
    double* w_f64;
    const double* tape;
    const double* ckpt;
    const double* hist;          // [n_steps + 1][6][n_beam]
    double* fbar;                // [4][n_xi][N1]
    double* jbbar;               // [n_xi][N1]
    double* scratch;             // adjoint_scratch_doubles
    double* ybar;                // [4][np]
    double* d0bar;               // [np]
    double* wbar;                // [np]
    double* sb0;                 // [6][n_beam]
    double* wbar_beam;           // [n_beam]
    double* wsum;                // 1
    double* partials;            // theta_partials_doubles
    const double* beam_draws;
    const double* plasma_draws;
    const double* gbar;          // 1
    double* grad;                // 5
};
size_t adjoint_lds_bytes(int n_nodes);
size_t adjoint_tape_doubles(int n_xi, int n_nodes);
size_t adjoint_scratch_doubles(int64_t np, int every, int threads);
size_t theta_partials_doubles();
hipError_t launch_march_record(const MarchDesc& d, int prec, int threads, double* tape, double* ckpt, int every,
                               hipStream_t s);
hipError_t launch_push_record(const GridDesc& g, int64_t n, const wk_beam_bufs& b, const void* fields, int prec,
                              int n_steps, double dt, double* hist, unsigned long long* counters, hipStream_t s);
hipError_t launch_gradient_backward(const GradDesc& gd, hipStream_t s);

}  // namespace wk
