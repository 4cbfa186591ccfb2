// Pipelined quasi-static cycle: n_steps plasma responses, each followed by a
// beam advance (WAKE paper, Section II A: plasma response for the frozen
// beam, then the beam advanced in t), run concurrently on many workgroups.
//
// A beam particle at xi only needs the fields of the previous response at its
// own xi, and its xi moves by far less than a slice per step.  So response n
// can march slice k as soon as response n-1 has stored the slices up to k+3:
// workgroup n then advances (step n-1) the beam particles of the xi bins it is
// about to need, deposits their current into a ring of LDS rows, and marches.
// Ordering between workgroups uses one progress counter per response
// (device-scope release after a slice is stored, acquire before use).  The
// arithmetic of every response, deposit and push is the one of the sequential
// cycle (current -> response -> push), so the two give the same result.
//
// Responses are handed out in increasing order by a ticket counter, so a
// workgroup only ever waits for a response that a running workgroup owns;
// each wait is bounded and sets an abort flag when exceeded so that every
// workgroup drains.
#include "wk_beam_dev.h"
#include <algorithm>

#include "wk_marcher.h"

namespace wk {
namespace {

using dev::Marcher;

constexpr int kRing = 4;          // rows of beam current in flight

// true when the node rows and the beam rows exceed LDS (large-grid variant)
__host__ __device__ inline bool cycle_needs_global_rows(int n_nodes)
{
    return (size_t)(NUM_ROWS + kRing) * lds_stride(n_nodes) * sizeof(double) > 159 * 1024;
}
constexpr int kLag = 2;           // slices of response n-1 needed beyond a bin: a particle of
                                  // bin b gathers slices b and b+1
constexpr int kPublish = 1;       // slices between progress publications
constexpr unsigned kSpinLimit = 1u << 26;

struct CycleDescFull {
    MarchDesc base;           // plasma template, constants, counters
    wk_beam_bufs beam;
    GridDesc grid;
    unsigned int* bin_start;         // [2][n_xi + 2]; bin n_xi: outside the window
    unsigned int* order;             // [2][n_beam] beam indices sorted by bin
    unsigned int* progress;          // [n_steps] stored slices per response
    unsigned int* ticket;
    unsigned long long* abort_flag;
    double* plasma_ws;               // per workgroup: x, y, px, py (4 * np doubles)
    double* big_rows;                // large grids, per workgroup: BIG_ROWS node rows + kRing beam rows
    void* ring;                      // 2 field slots, each 4 * n_xi * (n_r + 1) reals
    int64_t slot_elems;
    int64_t n_beam;
    int n_steps;
    double dt;
};

__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Thread 0 waits until progress[n] >= need (bounded); the caller follows
// with a workgroup barrier.  `seen` caches the last value read so that no
// acquire is issued while it already suffices.
__device__ __forceinline__ void wait_progress(const CycleDescFull& c, int n, unsigned need, unsigned& seen)
{
    if (seen >= need) return;
    unsigned spins = 0;
    for (;;) {
        const unsigned v = __hip_atomic_load(c.progress + n, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        seen = v;
        if (v >= need) return;
        if (__hip_atomic_load(c.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
        if (++spins > kSpinLimit) {
            __hip_atomic_store(c.abort_flag, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// Append, in order, the indices of old-bin range [beg, end) that satisfy
// pred to out[pos...]; returns the number appended.  Whole workgroup; uses
// the wave ballots and `wtot` (LDS, one int per wave).
template <class Pred>
__device__ __forceinline__ unsigned compact_append(const unsigned* old_order, unsigned beg, unsigned end, const Pred& pred,
                                   unsigned* out, unsigned pos, int* wtot)
{
    const int T = blockDim.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = T >> 6;
    unsigned total = 0;
    for (unsigned base = beg; base < end; base += T) {
        const unsigned q = base + tid;
        unsigned idx = 0;
        bool f = false;
        if (q < end) {
            idx = old_order[q];
            f = pred(idx);
        }
        const unsigned long long mask = __ballot(f);
        const unsigned rank = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wtot[wid] = __popcll(mask);
        __syncthreads();
        unsigned off = 0, chunk = 0;
        for (int w = 0; w < nw; ++w) {
            const unsigned c = (unsigned)wtot[w];
            if (w < wid) off += c;
            chunk += c;
        }
        if (f) out[pos + total + off + rank] = idx;
        total += chunk;
        __syncthreads();
    }
    return total;
}

template <typename R, class M>
struct CycleHooks : M::NoRecord {
    const CycleDescFull c;
    int n;                 // response index
    int next_bin;          // first bin not yet processed
    const R* prev;         // fields of response n-1 (ring slot)
    double* jb;            // kRing LDS rows
    int st;
    int* wtot;             // LDS scratch of the compaction
    unsigned seen;         // last progress[n-1] read (thread 0)
    unsigned pos;          // next free entry of the new order (uniform)
    // bins of the beam before this response's push (read) and after it (written)
    const unsigned* in_start;
    const unsigned* in_order;
    unsigned* out_start;
    unsigned* out_order;
    unsigned long long out_push, out_dep, bad_bin;

    __device__ __forceinline__ CycleHooks(const CycleDescFull& cd, int resp, double* rows, int stride, int* wt)
        : c(cd), n(resp), next_bin(0), jb(rows), st(stride), wtot(wt), seen(0), pos(0), out_push(0),
          out_dep(0), bad_bin(0)
    {
        prev = n > 0 ? (const R*)c.ring + (int64_t)((n - 1) & 1) * c.slot_elems : nullptr;
        const int nb2 = c.grid.n_xi + 2;
        const int rd = n > 0 ? ((n - 1) & 1) : 0;
        in_start = c.bin_start + (int64_t)rd * nb2;
        in_order = c.order + (int64_t)rd * c.n_beam;
        out_start = c.bin_start + (int64_t)(n & 1) * nb2;
        out_order = c.order + (int64_t)(n & 1) * c.n_beam;
    }

    __device__ __forceinline__ int cell_of(unsigned i) const { return dev::beam_xi_bin(c.grid, c.beam.d_xi[i]); }

    // New bin b of the pushed beam: the particles of old bin b-1 that left it,
    // then the ones of old bin b that stayed (xi only grows, by far less than
    // a slice per step).
    __device__ __forceinline__ void emit_movers(int b)
    {
        if (threadIdx.x == 0) out_start[b] = pos;
        if (b == 0) return;
        const int from = b - 1;
        pos += compact_append(in_order, in_start[from], in_start[from + 1],
                              [&](unsigned i) { return cell_of(i) != from; }, out_order, pos, wtot);
    }

    __device__ __forceinline__ void emit_stayers(int b)
    {
        pos += compact_append(in_order, in_start[b], in_start[b + 1],
                              [&](unsigned i) { return cell_of(i) == b; }, out_order, pos, wtot);
    }

    __device__ __forceinline__ double* jb_ring(int m) const { return jb + (m % kRing) * st; }

    // Advance (step n-1) and deposit the particles of xi bin b into the rows
    // b, b+1, b+2 of the ring; row b is then complete.
    __device__ __forceinline__ void process_bin(M& m, int b)
    {
        const GridDesc& g = c.grid;
        const int nxi = g.n_xi;
        if (n > 0) {
            if (threadIdx.x == 0) {
                const unsigned need = (unsigned)min(b + kLag, nxi);
                wait_progress(c, n - 1, need, seen);
            }
            __syncthreads();
            emit_movers(b);
        }
        const unsigned beg = in_start[b], end = in_start[b + 1];
        for (unsigned q = beg + threadIdx.x; q < end; q += blockDim.x) {
            const unsigned i = in_order[q];
            double x = c.beam.d_x[i], y = c.beam.d_y[i], xi = c.beam.d_xi[i];
            if (n > 0) {
                double px = c.beam.d_px[i], py = c.beam.d_py[i], pz = c.beam.d_pz[i];
                out_push += dev::beam_push_particle<R>(g, prev, x, y, xi, px, py, pz, 1, c.dt);
                c.beam.d_x[i] = x;
                c.beam.d_y[i] = y;
                c.beam.d_xi[i] = xi;
                c.beam.d_px[i] = px;
                c.beam.d_py[i] = py;
                c.beam.d_pz[i] = pz;
            }
            const double r = dev::beam_radius(g, x, y);
            const double xi_max = g.xi_min + nxi * g.dxi;
            if (r > g.r_max || xi < g.xi_min || xi >= xi_max) {
                ++out_dep;
                continue;
            }
            int j;
            double tr;
            dev::grid_hat(g, r, j, tr);
            const double u = (xi - g.xi_min) / g.dxi;
            int k = (int)floor(u);
            if (k > nxi - 1) k = nxi - 1;
            const double tk = u - k;
            if (k < b || k > b + 1) {
                ++bad_bin;     // moved by more than a slice in one step
                continue;
            }
            const double wb = c.beam.d_w[i];
            double* r0 = jb_ring(k);
            atomicAdd(r0 + j, wb * (1.0 - tr) * (1.0 - tk));
            atomicAdd(r0 + j + 1, wb * tr * (1.0 - tk));
            if (k + 1 < nxi) {
                double* r1 = jb_ring(k + 1);
                atomicAdd(r1 + j, wb * (1.0 - tr) * tk);
                atomicAdd(r1 + j + 1, wb * tr * tk);
            }
        }
        if (M::kBig) wait_stores();
        __syncthreads();
        // large grids: the ring rows are in global memory and the deposits
        // were L2 atomics, so drop this CU's L1 copies before reading them
        if (M::kBig) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (n > 0) emit_stayers(b);
        // row b is complete: J_bz = -sum / (V_j dxi)
        double* rb = jb_ring(b);
        for (int j = threadIdx.x; j <= g.n_r; j += blockDim.x)
            rb[j] = -rb[j] / (dev::grid_node_volume(g, j) * g.dxi);
        if (M::kBig) wait_stores();
        __syncthreads();
    }

    // After the march: advance the particles outside the window (no field)
    // and write the outside bin of the pushed beam (leavers of the last bin,
    // then the particles that were outside already).
    __device__ __forceinline__ void finish(int nxi)
    {
        if (n == 0) return;
        if (threadIdx.x == 0) wait_progress(c, n - 1, (unsigned)nxi + 1u, seen);
        __syncthreads();
        const unsigned beg = in_start[nxi], end = in_start[nxi + 1];
        for (unsigned q = beg + threadIdx.x; q < end; q += blockDim.x) {
            const unsigned i = in_order[q];
            double x = c.beam.d_x[i], y = c.beam.d_y[i], xi = c.beam.d_xi[i];
            double px = c.beam.d_px[i], py = c.beam.d_py[i], pz = c.beam.d_pz[i];
            out_push += dev::beam_push_particle<R>(c.grid, prev, x, y, xi, px, py, pz, 1, c.dt);
            c.beam.d_x[i] = x;
            c.beam.d_y[i] = y;
            c.beam.d_xi[i] = xi;
            c.beam.d_px[i] = px;
            c.beam.d_py[i] = py;
            c.beam.d_pz[i] = pz;
        }
        __syncthreads();
        emit_movers(nxi);
        pos += compact_append(in_order, beg, end, [&](unsigned) { return true; }, out_order, pos, wtot);
        if (threadIdx.x == 0) out_start[nxi + 1] = pos;
    }

    __device__ __forceinline__ void before_slice(M& m, int k)
    {
        const int need = min(k + 1, c.grid.n_xi - 1);
        while (next_bin <= need) {
            process_bin(m, next_bin);
            ++next_bin;
        }
    }

    __device__ __forceinline__ const double* jb_row(M&, int k) { return jb_ring(k); }

    __device__ __forceinline__ void after_store(M& m, int k)
    {
        // row k is no longer needed: clear it for row k + kRing
        double* rk = jb_ring(k);
        for (int j = threadIdx.x; j <= c.grid.n_r; j += blockDim.x) rk[j] = 0.0;
        if ((k + 1) % kPublish != 0 && k + 1 != c.grid.n_xi) return;
        wait_stores();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(c.progress + n, (unsigned)(k + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
};

// Advance every particle of bin b by one step with the fields of response
// n_prev (no deposit).
template <typename R>
__device__ __forceinline__ void push_bin_only(const CycleDescFull& c, const unsigned* start, const unsigned* order,
                              const R* fields, int b, unsigned long long& out)
{
    const unsigned beg = start[b], end = start[b + 1];
    for (unsigned q = beg + threadIdx.x; q < end; q += blockDim.x) {
        const unsigned i = order[q];
        double x = c.beam.d_x[i], y = c.beam.d_y[i], xi = c.beam.d_xi[i];
        double px = c.beam.d_px[i], py = c.beam.d_py[i], pz = c.beam.d_pz[i];
        out += dev::beam_push_particle<R>(c.grid, fields, x, y, xi, px, py, pz, 1, c.dt);
        c.beam.d_x[i] = x;
        c.beam.d_y[i] = y;
        c.beam.d_xi[i] = xi;
        c.beam.d_px[i] = px;
        c.beam.d_py[i] = py;
        c.beam.d_pz[i] = pz;
    }
}

template <typename R, int GEOM, bool WARM, int T, int K, bool RES, bool BIG = false>
__global__ __launch_bounds__(T) void k_cycle(CycleDescFull c)
{
    extern __shared__ double smem[];
    __shared__ int s_n;
    __shared__ int wtot[T / 64];
    using M = Marcher<R, GEOM, WARM, K, RES, BIG, T>;
    const int N1 = c.base.n_r + 1;
    const int st = lds_stride(N1);
    double* grow = BIG ? c.big_rows + (int64_t)blockIdx.x * (BIG_ROWS + kRing) * st : nullptr;
    double* jb_rows = BIG ? grow + (int64_t)BIG_ROWS * st : smem + NUM_ROWS * st;
    const int64_t np = c.base.np;
    double* mine = c.plasma_ws + (int64_t)blockIdx.x * 4 * np;
    for (;;) {
        if (threadIdx.x == 0) s_n = (int)atomicAdd(c.ticket, 1u);
        __syncthreads();
        const int n = s_n;
        __syncthreads();
        if (n > c.n_steps) break;
        unsigned long long out_push = 0, out_dep = 0, bad_bin = 0;
        if (n < c.n_steps) {
            // private copy of the unperturbed plasma (each response restarts
            // from the plasma ahead of the beam)
            MarchDesc d = c.base;
            d.x = mine;
            d.y = mine + np;
            d.px = mine + 2 * np;
            d.py = mine + 3 * np;
            d.fields = (R*)c.ring + (int64_t)(n & 1) * c.slot_elems;
            d.grow = grow;
            for (int64_t i = threadIdx.x; i < np; i += blockDim.x) {
                d.x[i] = c.base.x[i];
                d.px[i] = c.base.px[i];
                if (GEOM == WK_CYL && WARM) {
                    d.y[i] = c.base.y[i];
                    d.py[i] = c.base.py[i];
                } else if (WARM) {
                    d.py[i] = c.base.py[i];
                }
            }
            for (int r = 0; r < kRing; ++r)
                for (int j = threadIdx.x; j < N1; j += blockDim.x) jb_rows[r * st + j] = 0.0;
            wait_stores();
            __syncthreads();
            if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __syncthreads();
            M m(d, smem, jb_rows + kRing * st);
            CycleHooks<R, M> hooks(c, n, jb_rows, st, wtot);
            m.run(hooks);
            // particles outside the window see no field; advance them after the
            // previous response has advanced its own (progress n_xi + 1)
            hooks.finish(c.grid.n_xi);
            out_push = hooks.out_push;
            out_dep = hooks.out_dep;
            bad_bin = hooks.bad_bin;
            wait_stores();
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_store(c.progress + n, (unsigned)c.grid.n_xi + 1u, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // the last beam advance, in the fields of the last response
            const R* prev = (const R*)c.ring + (int64_t)((n - 1) & 1) * c.slot_elems;
            const int nb2 = c.grid.n_xi + 2;
            const unsigned* st_in = c.bin_start + (int64_t)((n - 1) & 1) * nb2;
            const unsigned* or_in = c.order + (int64_t)((n - 1) & 1) * c.n_beam;
            unsigned seen = 0;
            for (int b = 0; b <= c.grid.n_xi; ++b) {
                const unsigned need = b < c.grid.n_xi ? (unsigned)min(b + kLag, c.grid.n_xi) : (unsigned)c.grid.n_xi + 1u;
                if (threadIdx.x == 0) wait_progress(c, n - 1, need, seen);
                __syncthreads();
                push_bin_only<R>(c, st_in, or_in, prev, b, out_push);
            }
        }
        if (out_push) atomicAdd(c.base.counters + WK_CNT_BEAM_OUT_PUSH, out_push);
        if (out_dep) atomicAdd(c.base.counters + WK_CNT_BEAM_OUT_DEPOSIT, out_dep);
        if (bad_bin) atomicAdd(c.base.counters + WK_CNT_BEAM_BIN, bad_bin);
        __syncthreads();
    }
}

// Particles per thread of the resident variant: up to 8192 particles stay in
// registers at every workgroup size.
template <int T>
constexpr int cycle_tile() { return T >= 1024 ? 8 : 16; }

// Large grids: 1024 threads, particles streamed, node rows and beam rows in
// global memory.
template <typename R, int GEOM, bool WARM>
hipError_t launch_big(const CycleDescFull& c, int grid, hipStream_t s)
{
    if (!c.big_rows) return hipErrorInvalidValue;
    const size_t lds = big_lds_bytes(c.base.n_r + 1);
    auto kern = k_cycle<R, GEOM, WARM, 1024, cycle_tile<1024>(), false, true>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(1024), lds, s, c);
    return hipGetLastError();
}

template <typename R, int GEOM, bool WARM, int T>
hipError_t launch_t(const CycleDescFull& c, int grid, hipStream_t s)
{
    if (cycle_needs_global_rows(c.base.n_r + 1)) return launch_big<R, GEOM, WARM>(c, grid, s);
    constexpr int K = cycle_tile<T>();
    const size_t lds = march_lds_bytes(c.base.n_r + 1, T) + (size_t)kRing * lds_stride(c.base.n_r + 1) * sizeof(double);
    const int64_t kr = std::min<int64_t>(K, (c.base.np + T - 1) / T);
    const size_t lds_res = lds + 2 * (size_t)T * kr * sizeof(R);
    const bool res = c.base.np <= (int64_t)T * K && lds_res + 1024 <= 160 * 1024;
    if (res) {
        auto kern = k_cycle<R, GEOM, WARM, T, K, true>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_res);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(T), lds_res, s, c);
    } else {
        auto kern = k_cycle<R, GEOM, WARM, T, K, false>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(T), lds, s, c);
    }
    return hipGetLastError();
}

template <typename R, int GEOM, bool WARM>
hipError_t launch_w(const CycleDescFull& c, int threads, int grid, hipStream_t s)
{
    switch (threads) {
    case 256: return launch_t<R, GEOM, WARM, 256>(c, grid, s);
    case 512: return launch_t<R, GEOM, WARM, 512>(c, grid, s);
    default: return launch_t<R, GEOM, WARM, 1024>(c, grid, s);
    }
}

template <typename R>
hipError_t launch_r(const CycleDescFull& c, int threads, int grid, hipStream_t s)
{
    if (c.base.geom == WK_CYL)
        return c.base.warm ? launch_w<R, WK_CYL, true>(c, threads, grid, s) : launch_w<R, WK_CYL, false>(c, threads, grid, s);
    return c.base.warm ? launch_w<R, WK_SLAB, true>(c, threads, grid, s) : launch_w<R, WK_SLAB, false>(c, threads, grid, s);
}

}  // namespace

size_t cycle_lds_bytes(int n_nodes)
{
    if (cycle_needs_global_rows(n_nodes)) return big_lds_bytes(n_nodes);
    return march_lds_bytes(n_nodes, 0) + (size_t)kRing * lds_stride(n_nodes) * sizeof(double);
}
size_t cycle_big_rows_bytes(int n_nodes)
{
    return cycle_needs_global_rows(n_nodes) ? (size_t)(BIG_ROWS + kRing) * lds_stride(n_nodes) * sizeof(double) : 0;
}

hipError_t launch_cycle(const CycleDesc& cd, int prec, int threads, int grid, hipStream_t s)
{
    CycleDescFull c;
    c.base = cd.base;
    c.beam = cd.beam;
    c.grid = cd.grid;
    c.bin_start = cd.bin_start;
    c.order = cd.order;
    c.n_beam = cd.n_beam;
    c.progress = cd.progress;
    c.ticket = cd.ticket;
    c.abort_flag = cd.abort_flag;
    c.plasma_ws = cd.plasma_ws;
    c.big_rows = cd.big_rows;
    c.ring = cd.ring;
    c.slot_elems = cd.slot_elems;
    c.n_steps = cd.n_steps;
    c.dt = cd.dt;
    return prec == WK_FP64 ? launch_r<double>(c, threads, grid, s) : launch_r<float>(c, threads, grid, s);
}

}  // namespace wk
