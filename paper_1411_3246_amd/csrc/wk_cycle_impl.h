// Pipelined quasi-static cycle: n_steps plasma responses, each followed by a
// beam advance (WAKE paper, Section II A: plasma response for the frozen
// beam, then the beam advanced in t), run concurrently on many workgroups.
// Instantiated per precision and geometry by wk_cycle_*.hip.
//
// A beam particle at xi only needs the fields of the previous response at its
// own xi, and its xi moves by far less than a slice per step.  So response n
// can march slice k as soon as response n-1 has stored the slices up to k+2:
// it then advances (step n-1) the beam particles of the xi bins it is about
// to need and deposits their current while it marches.
//
// Each response is marched by a group of G workgroups (ranks g = 0..G-1):
// rank g owns a band of plasma cells and one contiguous subset of the beam,
// with its own xi bins of that subset, double-buffered between successive
// responses.  Rank 0 stores the fields and publishes the response's progress
// (stored slices) after every slice.  Everything another compute unit reads
// during the launch (fields, beam particles, bins, progress) is written and
// read with device-coherent accesses (wk_marcher.h).
//
// Workgroups take tickets in increasing order (ticket t: response t / G,
// rank t % G), so a workgroup only waits for workgroups that have started;
// every wait is bounded and raises the abort counter when exceeded.
#pragma once

#include "wk_beam_dev.h"
#include "wk_march_impl.h"

namespace wk {
namespace cycle_impl {

using dev::ld_dev;
using dev::st_dev;

constexpr int kLag = 2;   // slices of response n-1 needed beyond a bin: a particle of
                          // bin b gathers slices b and b+1
constexpr int kRing = kCycleRing;  // LDS rows of beam current in flight (grids whose rows fit LDS)

// One beam subset (pointers offset to its first particle).
struct BeamSub {
    double *x, *y, *xi, *px, *py, *pz;
    const double* w;
    unsigned n;
};

// Append, in order, the indices of old-bin range [beg, end) that satisfy
// pred to out[pos...]; returns the number appended.  Whole workgroup; uses
// the wave ballots and `wtot` (LDS, one int per wave).
template <int T, class Pred>
__device__ __forceinline__ unsigned compact_append(const unsigned* old_order, unsigned beg, unsigned end,
                                                   const Pred& pred, unsigned* out, unsigned pos, int* wtot)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int nw = T >> 6;
    unsigned total = 0;
    for (unsigned base = beg; base < end; base += T) {
        const unsigned q = base + tid;
        unsigned idx = 0;
        bool f = false;
        if (q < end) {
            idx = ld_dev(old_order + q);
            f = pred(idx);
        }
        const unsigned long long mask = __ballot(f);
        const unsigned rank = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wtot[wid] = __popcll(mask);
        __syncthreads();
        unsigned off = 0, chunk = 0;
#pragma unroll
        for (int w = 0; w < nw; ++w) {
            const unsigned c = (unsigned)wtot[w];
            if (w < wid) off += c;
            chunk += c;
        }
        if (f) st_dev(out + pos + total + off + rank, idx);
        total += chunk;
        dev::wait_vm();
        __syncthreads();
    }
    return total;
}

template <typename R, class M, int K>
struct CycleHooks : M::NoRecord {
    static constexpr int T = M::kT;
    const CycleDesc& c;
    int n, g;              // response index, rank in the group
    int next_bin;          // first bin not yet processed
    const R* prev;         // fields of response n-1 (ring slot)
    BeamSub B;
    int* wtot;             // LDS scratch of the compaction
    double* ring;          // kRing LDS rows of raw beam J_z (row k at k % kRing); null on large grids
    int st;                // stride of the ring rows
    unsigned seen;         // last progress[n-1] read (thread 0)
    unsigned pos;          // next free entry of the new order (uniform)
    // this subset's bins before this response's push (read) and after it (written)
    const unsigned* in_start;
    const unsigned* in_order;
    unsigned* out_start;
    unsigned* out_order;
    unsigned pend;         // movers of the last old bin, written at [pos, pos + pend) of the new order
    unsigned long long out_push, out_dep, bad_bin;

    __device__ __forceinline__ CycleHooks(const CycleDesc& cd, int resp, int rank, int* wt, double* ring_rows,
                                          int stride)
        : c(cd), n(resp), g(rank), next_bin(0), wtot(wt), ring(ring_rows), st(stride), seen(0), pos(0), pend(0),
          out_push(0), out_dep(0), bad_bin(0)
    {
        const int G = c.base.group;
        prev = n > 0 ? (const R*)c.ring + (int64_t)((n - 1) & 1) * c.slot_elems : nullptr;
        const int64_t b0 = c.n_beam * g / G, b1 = c.n_beam * (g + 1) / G;
        B.x = c.beam.d_x + b0;
        B.y = c.beam.d_y + b0;
        B.xi = c.beam.d_xi + b0;
        B.px = c.beam.d_px + b0;
        B.py = c.beam.d_py + b0;
        B.pz = c.beam.d_pz + b0;
        B.w = c.beam.d_w + b0;
        B.n = (unsigned)(b1 - b0);
        const int nb2 = c.grid.n_xi + 2;
        const int rd = n > 0 ? ((n - 1) & 1) : 0;
        in_start = c.bin_start + ((int64_t)rd * G + g) * nb2;
        in_order = c.order + (int64_t)rd * c.n_beam + b0;
        out_start = c.bin_start + ((int64_t)(n & 1) * G + g) * nb2;
        out_order = c.order + (int64_t)(n & 1) * c.n_beam + b0;
    }

    __device__ __forceinline__ int cell_of(unsigned i) const { return dev::beam_xi_bin(c.grid, ld_dev(B.xi + i)); }

    // Thread 0 waits until response n-1 has stored `need` slices, then the
    // workgroup synchronizes.
    __device__ __forceinline__ void wait_prev(unsigned need)
    {
        if (threadIdx.x == 0 && seen < need) {
            dev::wait_at_least(c.progress + (n - 1), need, c.abort_flag);
            seen = ld_dev(c.progress + (n - 1));
        }
        __syncthreads();
    }

    // Chunks (of T particles) of a bin whose movers are kept in registers
    // until the bin's stayers are counted; the movers of later chunks are
    // found again.  One chunk for the 16-particle shape, whose registers are
    // already short (one workgroup per response).
    static constexpr int kMvChunks = K > 8 ? 1 : 4;

    // Advance (step n-1) the particles of this subset's old xi bin b, deposit
    // their current, and write the new order.  New bin b is the particles of
    // old bin b-1 that left it (written when that bin was processed), then the
    // particles of old bin b that stay in it (xi only grows, by far less than a
    // slice per step); the ones that leave old bin b are written after those
    // and open new bin b+1.  Each particle's slot comes from wavefront ballots
    // over the pass that pushes it, so the order is that of the old order.
    __device__ __forceinline__ void process_bin(int b)
    {
        const GridDesc& gr = c.grid;
        const int nxi = gr.n_xi;
        const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
        constexpr int nw = T >> 6;
        if (n > 0) {
            // the last bin also waits for response n-1 to finish reading the
            // order slot that this response writes
            const unsigned need = (b == nxi - 1 && n >= 2) ? (unsigned)nxi + 1u : (unsigned)min(b + kLag, nxi);
            wait_prev(need);
            if (tid == 0) st_dev(out_start + b, pos);
            pos += pend;
            pend = 0;
        }
        const unsigned beg = ld_dev(in_start + b), end = ld_dev(in_start + b + 1);
        const double xi_max = gr.xi_min + nxi * gr.dxi;
        unsigned mv_idx[kMvChunks], mv_rank[kMvChunks];
        unsigned n_stay = 0, n_move = 0;
        unsigned n_move_rec = 0;   // movers of the chunks kept in registers
        int ci = 0;
        for (unsigned base = beg; base < end; base += T, ++ci) {
            if (ci == kMvChunks) n_move_rec = n_move;
            const unsigned q = base + tid;
            unsigned i = 0;
            bool stay = false, move = false;
            if (q < end) {
                i = ld_dev(in_order + q);
                double x = ld_dev(B.x + i), y = ld_dev(B.y + i), xi = ld_dev(B.xi + i);
                if (n > 0) {
                    double px = ld_dev(B.px + i), py = ld_dev(B.py + i), pz = ld_dev(B.pz + i);
                    out_push += dev::beam_push_particle<R, true>(gr, prev, x, y, xi, px, py, pz, 1, c.dt);
                    st_dev(B.x + i, x);
                    st_dev(B.y + i, y);
                    st_dev(B.xi + i, xi);
                    st_dev(B.px + i, px);
                    st_dev(B.py + i, py);
                    st_dev(B.pz + i, pz);
                    const int kk = dev::beam_xi_bin(gr, xi);
                    if (kk != nxi && kk != b && kk != b + 1) ++bad_bin;   // moved by more than a slice
                    stay = kk == b;
                    move = !stay;
                }
                const double r = dev::beam_radius(gr, x, y);
                if (r > gr.r_max || xi < gr.xi_min || xi >= xi_max) ++out_dep;
                else if (ring) ring_deposit(r, xi, B.w[i], b);
            }
            if (n == 0) continue;
            const unsigned long long ms = __ballot(stay), mm = __ballot(move);
            const unsigned long long below = (1ull << lane) - 1ull;
            if (lane == 0) {
                wtot[wid] = __popcll(ms);
                wtot[nw + wid] = __popcll(mm);
            }
            __syncthreads();
            unsigned off_s = 0, off_m = 0, ch_s = 0, ch_m = 0;
#pragma unroll
            for (int w = 0; w < nw; ++w) {
                const unsigned cs = (unsigned)wtot[w], cm = (unsigned)wtot[nw + w];
                if (w < wid) {
                    off_s += cs;
                    off_m += cm;
                }
                ch_s += cs;
                ch_m += cm;
            }
            if (stay) st_dev(out_order + pos + n_stay + off_s + __popcll(ms & below), i);
#pragma unroll
            for (int r = 0; r < kMvChunks; ++r)
                if (r == ci) {
                    mv_idx[r] = move ? i : ~0u;
                    mv_rank[r] = n_move + off_m + __popcll(mm & below);
                }
            n_stay += ch_s;
            n_move += ch_m;
            __syncthreads();   // wtot is reused by the next chunk
        }
        if (n > 0) {
            // the movers after the stayers: those of the first chunks from
            // registers, those of later chunks found again (their new xi was
            // stored by this same thread)
            const unsigned pm = pos + n_stay;
#pragma unroll
            for (int r = 0; r < kMvChunks; ++r)
                if (r < ci && mv_idx[r] != ~0u) st_dev(out_order + pm + mv_rank[r], mv_idx[r]);
            if (ci > kMvChunks)
                compact_append<T>(in_order, beg + (unsigned)kMvChunks * T, end,
                                  [&](unsigned i) { return cell_of(i) != b; }, out_order, pm + n_move_rec, wtot);
            pos = pm;
            pend = n_move;
        }
        dev::wait_vm();
        __syncthreads();
    }

    // End of new bin b (bins up to next_bin - 1 are complete).
    __device__ __forceinline__ unsigned new_end(int b) const
    {
        return b + 1 < next_bin ? ld_dev(out_start + b + 1) : pos;
    }

    // Raw J_z of one beam particle of bin b (just pushed) into the ring rows
    // of slices kk and kk + 1, bilinear in (r, xi) (Section II A: the total
    // current includes the beam's; v_z = c).  A particle of bin b is at
    // kk = b or b + 1; rows b .. b + 2 are free or still accumulating.
    __device__ __forceinline__ void ring_deposit(double r, double xi, double w, int b)
    {
        const GridDesc& gr = c.grid;
        const double u = (xi - gr.xi_min) / gr.dxi;
        int kk = (int)floor(u);
        if (kk > gr.n_xi - 1) kk = gr.n_xi - 1;
        if (kk < b || kk > b + 1) return;   // counted as a bin escape after the push
        const double tk = u - kk;
        int j;
        double tr;
        dev::grid_hat(gr, r, j, tr);
        const double v = -w / gr.dxi;
        double* r0 = ring + (kk % kRing) * st;
        atomicAdd(r0 + j, v * (1.0 - tr) * (1.0 - tk));
        atomicAdd(r0 + j + 1, v * tr * (1.0 - tk));
        if (kk + 1 < gr.n_xi) {
            double* r1 = ring + ((kk + 1) % kRing) * st;
            atomicAdd(r1 + j, v * (1.0 - tr) * tk);
            atomicAdd(r1 + j + 1, v * tr * tk);
        }
    }

    // Raw J_z of the beam particles of this subset at slice k, added to the
    // J_z deposit row (divided by the node volumes with the plasma deposits):
    // the ring row of slice k, or on large grids the particles of new bins
    // k-1 and k, bilinear in (r, xi).
    __device__ __forceinline__ void deposit_beam(M& m, int k)
    {
        if (ring) {
            double* jz = m.row(ROW_JZ);
            const double* rk = ring + (k % kRing) * st;
            for (int j = threadIdx.x; j <= c.grid.n_r; j += T) atomicAdd(jz + j, rk[j]);
            return;
        }
        if (B.n == 0) return;
        const GridDesc& gr = c.grid;
        const unsigned* S = n > 0 ? out_start : in_start;
        const unsigned* O = n > 0 ? out_order : in_order;
        const unsigned beg = ld_dev(S + (k > 0 ? k - 1 : 0));
        const unsigned end = n > 0 ? new_end(k) : ld_dev(in_start + k + 1);
        const double xi_max = gr.xi_min + gr.n_xi * gr.dxi;
        const double idxi = 1.0 / gr.dxi;
        double* jz = m.row(ROW_JZ);
        for (unsigned q = beg + threadIdx.x; q < end; q += T) {
            const unsigned i = ld_dev(O + q);
            const double x = ld_dev(B.x + i), y = ld_dev(B.y + i), xi = ld_dev(B.xi + i);
            const double r = dev::beam_radius(gr, x, y);
            if (r > gr.r_max || xi < gr.xi_min || xi >= xi_max) continue;
            const double u = (xi - gr.xi_min) / gr.dxi;
            int kk = (int)floor(u);
            if (kk > gr.n_xi - 1) kk = gr.n_xi - 1;
            const double tk = u - kk;
            double wk;
            if (kk == k) wk = 1.0 - tk;
            else if (kk == k - 1) wk = tk;
            else continue;
            int j;
            double tr;
            dev::grid_hat(gr, r, j, tr);
            const double v = -B.w[i] * wk * idxi;
            atomicAdd(jz + j, v * (1.0 - tr));
            atomicAdd(jz + j + 1, v * tr);
        }
    }

    // After the march: advance the particles outside the window (they see no
    // field) and write the outside bin of the pushed beam (leavers of the last
    // bin, then the particles that were outside already).  A particle ahead of
    // the window that has drifted into it stays in the outside bin here and is
    // counted in WK_CNT_BEAM_BIN.
    __device__ __forceinline__ void finish()
    {
        if (n == 0) return;
        const int nxi = c.grid.n_xi;
        wait_prev((unsigned)nxi + 1u);
        const unsigned beg = ld_dev(in_start + nxi), end = ld_dev(in_start + nxi + 1);
        for (unsigned q = beg + threadIdx.x; q < end; q += T) {
            const unsigned i = ld_dev(in_order + q);
            double x = ld_dev(B.x + i), y = ld_dev(B.y + i), xi = ld_dev(B.xi + i);
            double px = ld_dev(B.px + i), py = ld_dev(B.py + i), pz = ld_dev(B.pz + i);
            out_push += dev::beam_push_particle<R, true>(c.grid, prev, x, y, xi, px, py, pz, 1, c.dt);
            st_dev(B.x + i, x);
            st_dev(B.y + i, y);
            st_dev(B.xi + i, xi);
            st_dev(B.px + i, px);
            st_dev(B.py + i, py);
            st_dev(B.pz + i, pz);
            if (dev::beam_xi_bin(c.grid, xi) != nxi) ++bad_bin;
        }
        dev::wait_vm();
        __syncthreads();
        // the new outside bin: the movers of the last old bin (written when it
        // was processed), then the particles that were outside already
        if (threadIdx.x == 0) st_dev(out_start + nxi, pos);
        pos += pend;
        pend = 0;
        pos += compact_append<T>(in_order, beg, end, [&](unsigned) { return true; }, out_order, pos, wtot);
        if (threadIdx.x == 0) {
            st_dev(out_start + nxi + 1, pos);
            if (pos != B.n) atomicAdd(c.base.counters + WK_CNT_BEAM_ORDER, 1ull);
        }
    }

    __device__ __forceinline__ void before_slice(M&, int k)
    {
        const int need = min(k + 1, c.grid.n_xi - 1);
        while (next_bin <= need) {
            process_bin(next_bin);
            ++next_bin;
        }
    }

    __device__ __forceinline__ const double* jb_row(M&, int) { return nullptr; }

    __device__ __forceinline__ void after_store(M&, int k)
    {
        // ring row k is used up: cleared for slice k + kRing
        if (ring) {
            double* rk = ring + (k % kRing) * st;
            for (int j = threadIdx.x; j <= c.grid.n_r; j += T) rk[j] = 0.0;
        }
        if (g != 0) return;
        dev::wait_vm();
        __syncthreads();
        if (threadIdx.x == 0) st_dev(c.progress + n, (unsigned)(k + 1));
    }
};

// Advance every particle of bin b of one subset by one step with the fields
// of the last response (no deposit).
template <typename R, int T>
__device__ __forceinline__ void push_bin_only(const CycleDesc& c, const BeamSub& B, const unsigned* start,
                                              const unsigned* order, const R* fields, int b, unsigned long long& out)
{
    const unsigned beg = ld_dev(start + b), end = ld_dev(start + b + 1);
    for (unsigned q = beg + threadIdx.x; q < end; q += T) {
        const unsigned i = ld_dev(order + q);
        double x = ld_dev(B.x + i), y = ld_dev(B.y + i), xi = ld_dev(B.xi + i);
        double px = ld_dev(B.px + i), py = ld_dev(B.py + i), pz = ld_dev(B.pz + i);
        out += dev::beam_push_particle<R, true>(c.grid, fields, x, y, xi, px, py, pz, 1, c.dt);
        st_dev(B.x + i, x);
        st_dev(B.y + i, y);
        st_dev(B.xi + i, xi);
        st_dev(B.px + i, px);
        st_dev(B.py + i, py);
        st_dev(B.pz + i, pz);
    }
}

template <typename R, int GEOM, bool WARM, int T, int K, bool RES, bool BIG, int WPS>
__global__ __launch_bounds__(T, WPS) void k_cycle(CycleDesc c)
{
    extern __shared__ double smem[];
    __shared__ int s_ticket;
    __shared__ int wtot[2 * (T / 64)];
    using M = dev::Marcher<R, GEOM, WARM, T, K, RES, BIG>;
    const int G = c.base.group;
    const int N1 = c.base.n_r + 1;
    const int st = lds_stride(N1);
    double* grow = BIG ? c.big_rows + (int64_t)blockIdx.x * BIG_ROWS * st : nullptr;
    const int64_t np_max = (int64_t)((c.base.n_r + G - 1) / G) * c.base.ppc;
    double* mine = c.plasma_ws ? c.plasma_ws + (int64_t)blockIdx.x * 4 * np_max : nullptr;
    const int nb2 = c.grid.n_xi + 2;
    for (;;) {
        if (threadIdx.x == 0) s_ticket = (int)atomicAdd(c.ticket, 1u);
        __syncthreads();
        const int t = s_ticket;
        __syncthreads();
        const int n = t / G, g = t % G;
        if (n > c.n_steps) break;
        unsigned long long out_push = 0, out_dep = 0, bad_bin = 0;
        if (n < c.n_steps) {
            MarchDesc d = march_impl::member_desc<R>(c.base, g);
            if (!RES) {
                // streamed particles are stored back every slice: a private
                // copy of the unperturbed plasma (each response restarts from
                // the plasma ahead of the beam)
                for (int64_t i = threadIdx.x; i < d.np; i += T) {
                    mine[i] = d.x[i];
                    mine[2 * np_max + i] = d.px[i];
                    if (GEOM == WK_CYL && WARM) {
                        mine[np_max + i] = d.y[i];
                        mine[3 * np_max + i] = d.py[i];
                    } else if (WARM) {
                        mine[3 * np_max + i] = d.py[i];
                    }
                }
                d.x = mine;
                d.y = mine + np_max;
                d.px = mine + 2 * np_max;
                d.py = mine + 3 * np_max;
                __syncthreads();
            }
            d.fields = (R*)c.ring + (int64_t)(n & 1) * c.slot_elems;
            d.grow = grow;
            dev::Group grp;
            grp.G = G;
            grp.g = g;
            grp.xbuf = c.xbuf ? c.xbuf + (int64_t)n * 2 * G * kXRows * st : nullptr;
            grp.ctr = c.gctr ? c.gctr + (int64_t)n * kCtrPad : nullptr;
            grp.abort = c.abort_flag;
            double* ring = BIG ? nullptr : smem + NUM_ROWS * st;
            void* pconst = BIG ? nullptr : (void*)(smem + (NUM_ROWS + kRing) * st);
            if (ring) {
                for (int q = threadIdx.x; q < kRing * st; q += T) ring[q] = 0.0;
                __syncthreads();
            }
            // resident particles are loaded from the template and not stored back
            M m(d, smem, pconst, grp, g == 0, false);
            CycleHooks<R, M, K> hooks(c, n, g, wtot, ring, st);
            m.run(hooks);
            hooks.finish();
            out_push = hooks.out_push;
            out_dep = hooks.out_dep;
            bad_bin = hooks.bad_bin;
            // every rank has finished its beam subset: response n is complete
            if (G > 1) dev::group_barrier(m.grp);
            dev::wait_vm();
            __syncthreads();
            if (g == 0 && threadIdx.x == 0) st_dev(c.progress + n, (unsigned)c.grid.n_xi + 1u);
        } else {
            // the last beam advance, in the fields of the last response
            const R* prev = (const R*)c.ring + (int64_t)((n - 1) & 1) * c.slot_elems;
            const int64_t b0 = c.n_beam * g / G, b1 = c.n_beam * (g + 1) / G;
            BeamSub B{c.beam.d_x + b0, c.beam.d_y + b0, c.beam.d_xi + b0, c.beam.d_px + b0,
                      c.beam.d_py + b0, c.beam.d_pz + b0, c.beam.d_w + b0, (unsigned)(b1 - b0)};
            const unsigned* st_in = c.bin_start + ((int64_t)((n - 1) & 1) * G + g) * nb2;
            const unsigned* or_in = c.order + (int64_t)((n - 1) & 1) * c.n_beam + b0;
            unsigned seen = 0;
            for (int b = 0; b <= c.grid.n_xi; ++b) {
                const unsigned need = b < c.grid.n_xi ? (unsigned)min(b + kLag, c.grid.n_xi) : (unsigned)c.grid.n_xi + 1u;
                if (threadIdx.x == 0 && seen < need) {
                    dev::wait_at_least(c.progress + (n - 1), need, c.abort_flag);
                    seen = ld_dev(c.progress + (n - 1));
                }
                __syncthreads();
                push_bin_only<R, T>(c, B, st_in, or_in, prev, b, out_push);
            }
        }
        if (out_push) atomicAdd(c.base.counters + WK_CNT_BEAM_OUT_PUSH, out_push);
        if (out_dep) atomicAdd(c.base.counters + WK_CNT_BEAM_OUT_DEPOSIT, out_dep);
        if (bad_bin) atomicAdd(c.base.counters + WK_CNT_BEAM_BIN, bad_bin);
        __syncthreads();
    }
}

template <typename R, int GEOM, bool WARM, int SH>
hipError_t go(const CycleDesc& c, int grid, size_t lds, hipStream_t s, int* occ)
{
    constexpr ShapeInfo S = kShapes[SH];
    if constexpr (S.big && S.resident && sizeof(R) == 8) {
        return hipErrorInvalidValue;
    } else {
        auto kern = k_cycle<R, GEOM, WARM, S.threads, S.kp, S.resident, S.big, S.waves_per_simd>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        if (occ) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, S.threads, lds);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(S.threads), lds, s, c);
        return hipGetLastError();
    }
}

template <typename R, int GEOM, bool WARM>
hipError_t go_shape(const CycleDesc& c, int shape, int grid, size_t lds, hipStream_t s, int* occ)
{
    switch (shape) {
    case SH_256_4: return go<R, GEOM, WARM, SH_256_4>(c, grid, lds, s, occ);
    case SH_512_8: return go<R, GEOM, WARM, SH_512_8>(c, grid, lds, s, occ);
    case SH_512_4: return go<R, GEOM, WARM, SH_512_4>(c, grid, lds, s, occ);
    case SH_512_16: return go<R, GEOM, WARM, SH_512_16>(c, grid, lds, s, occ);
    case SH_1024_8: return go<R, GEOM, WARM, SH_1024_8>(c, grid, lds, s, occ);
    case SH_1024_STREAM: return go<R, GEOM, WARM, SH_1024_STREAM>(c, grid, lds, s, occ);
    case SH_BIG_512_8: return go<R, GEOM, WARM, SH_BIG_512_8>(c, grid, lds, s, occ);
    case SH_BIG_STREAM: return go<R, GEOM, WARM, SH_BIG_STREAM>(c, grid, lds, s, occ);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int GEOM>
hipError_t launch(const CycleDesc& c, int warm, int shape, int grid, size_t lds, hipStream_t s, int* occ)
{
    return warm ? go_shape<R, GEOM, true>(c, shape, grid, lds, s, occ)
                : go_shape<R, GEOM, false>(c, shape, grid, lds, s, occ);
}

}  // namespace cycle_impl
}  // namespace wk
