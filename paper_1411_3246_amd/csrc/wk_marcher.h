// Device-side march of one plasma response (shared by the single, batched and
// pipelined launches and by the recording forward of the adjoint).  Internal
// header of libwake.
//
// A response may be marched by a group of G workgroups: workgroup g owns the
// plasma macroparticles of a contiguous band of cells, deposits them into its
// own LDS rows, and the G partial rows are summed between the workgroups in a
// fixed order through device memory (four exchanges per slice).  Every
// workgroup then solves the radial field equations itself on the identical
// sums, so all of them gather the same fields.
#pragma once

#include "wk_internal.h"

namespace wk {
namespace dev {

// --------------------------------------------------------------------------
// Reciprocals and square roots
// --------------------------------------------------------------------------
// Double reciprocal: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

template <typename R> __device__ __forceinline__ R frcp(R x);
template <> __device__ __forceinline__ float frcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double frcp<double>(double x) { return 1.0 / x; }
template <typename R> __device__ __forceinline__ R fsqrt(R x);
template <> __device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double fsqrt<double>(double x) { return sqrt(x); }

// --------------------------------------------------------------------------
// Device-coherent accesses.  Data that another compute unit reads during the
// same launch (partial deposit rows, stored fields of the pipelined cycle,
// beam particles and their bins) is written and read with agent-scope
// atomic accesses, which bypass the caches that are not coherent across
// compute units and accelerator dies.  A writer waits for its stores to be
// acknowledged (wait_vm) before it signals, so a reader that has seen the
// signal reads the new values.  No cache-wide writeback or invalidation is
// needed.
// --------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ V ld_dev(const V* p)
{
    return __hip_atomic_load(const_cast<V*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V>
__device__ __forceinline__ void st_dev(V* p, V v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Workgroup barrier that orders LDS accesses only: unlike __syncthreads it
// does not wait for this thread's global stores to be acknowledged.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Bounded waits: a wait gives up after kWaitTicks of the constant-rate
// device clock (wall_clock64, 100 MHz) and raises the abort counter, so a
// launch whose workgroups cannot all run at once ends with an error instead
// of hanging.
constexpr unsigned long long kWaitTicks = 2000000000ull;   // 20 s at 100 MHz

// Thread 0 only: spin until *p >= need or the abort flag is set.
__device__ __forceinline__ void wait_at_least(const unsigned* p, unsigned need, unsigned long long* abort_flag)
{
    if (ld_dev(p) >= need) return;
    const unsigned long long t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        if (ld_dev(p) >= need) return;
        if (ld_dev(abort_flag)) return;
        if (wall_clock64() - t0 > kWaitTicks) {
            st_dev(abort_flag, 1ull);
            return;
        }
    }
}

// The workgroups that march one response together.
struct Group {
    int G = 1;                           // workgroups in the group
    int g = 0;                           // this workgroup's rank
    double* xbuf = nullptr;              // [2][G][kXRows][stride] partial rows (two slots)
    unsigned* ctr = nullptr;             // arrival counter
    unsigned long long* abort = nullptr;
    unsigned epoch = 0;                  // exchanges done
    unsigned bars = 0;                   // counter barriers passed
};

// All threads: every thread's device-coherent stores are complete; arrive at
// the group barrier and wait for the other workgroups of the group.
__device__ __forceinline__ void group_barrier(Group& grp)
{
    wait_vm();
    __syncthreads();
    ++grp.bars;
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(grp.ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_at_least(grp.ctr, grp.bars * (unsigned)grp.G, grp.abort);
    }
    __syncthreads();
}

// --------------------------------------------------------------------------
// Wave-level prefix sums with DPP row shifts and row broadcasts
// --------------------------------------------------------------------------
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ double wave_prefix(double v)
{
    v += dpp_move<0x111, 0xf>(v);   // row_shr:1
    v += dpp_move<0x112, 0xf>(v);   // row_shr:2
    v += dpp_move<0x114, 0xf>(v);   // row_shr:4
    v += dpp_move<0x118, 0xf>(v);   // row_shr:8
    v += dpp_move<0x142, 0xa>(v);   // row_bcast:15
    v += dpp_move<0x143, 0xc>(v);   // row_bcast:31
    return v;
}

// LDS scratch of the block-wide scans: two buffers of per-wave totals (at
// most 16 waves each).
__device__ __forceinline__ double* scan_scratch()
{
    __shared__ double s[32];
    return s;
}

// Barrier of the march.  Its node rows are in LDS, so the barrier orders LDS
// accesses only and does not wait for outstanding global stores (fields,
// exchange rows).  The large-grid variant keeps node rows in global memory,
// so there a barrier also waits for this thread's stores.
template <bool GLOBAL_ROWS>
__device__ __forceinline__ void block_sync()
{
    if (GLOBAL_ROWS) {
        wait_vm();
        __syncthreads();
    } else {
        lds_barrier();
    }
}

// Double value of lane `src` of the wavefront (two 32-bit permutes).
__device__ __forceinline__ double lane_value(double v, int src)
{
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Parallel cyclic reduction by the whole workgroup of the tridiagonal system
// with rows (a, b, c, d) in buffer 0 (a[0] and c[n-1] ignored); buffer 1 is
// scratch.  Solution in x.  Reduction steps with strides 1, 2, 4, ... run in
// memory with one barrier each until the rows of equal index modulo the
// stride s form independent systems of at most 64 rows; each wavefront then
// finishes its systems in registers (lane l holds row c + l s) with lane
// permutes and no barrier.  Every step computes the same expressions as a
// step in memory would.
template <bool GLOBAL_ROWS = false>
__device__ __forceinline__ void block_pcr(double* a0, double* b0, double* c0, double* d0, double* a1, double* b1,
                                          double* c1, double* d1, double* x, int n)
{
    const int T = blockDim.x, tid = threadIdx.x;
    int s = 1;
    for (; (n + s - 1) / s > 64; s <<= 1) {
        for (int i = tid; i < n; i += T) {
            double na = 0.0, nb = b0[i], nc = 0.0, nd = d0[i];
            if (i - s >= 0) {
                const double k1 = a0[i] * rcp64(b0[i - s]);
                na = -a0[i - s] * k1;
                nb -= c0[i - s] * k1;
                nd -= d0[i - s] * k1;
            }
            if (i + s < n) {
                const double k2 = c0[i] * rcp64(b0[i + s]);
                nc = -c0[i + s] * k2;
                nb -= a0[i + s] * k2;
                nd -= d0[i + s] * k2;
            }
            a1[i] = na;
            b1[i] = nb;
            c1[i] = nc;
            d1[i] = nd;
        }
        block_sync<GLOBAL_ROWS>();
        double* t;
        t = a0; a0 = a1; a1 = t;
        t = b0; b0 = b1; b1 = t;
        t = c0; c0 = c1; c1 = t;
        t = d0; d0 = d1; d1 = t;
    }
    const int lane = tid & 63;
    for (int c = tid >> 6; c < s; c += T >> 6) {
        const int m = (n - c + s - 1) / s;   // rows of system c
        const int i = c + lane * s;
        const bool on = lane < m;
        double a = on ? a0[i] : 0.0, b = on ? b0[i] : 1.0, cc = on ? c0[i] : 0.0, d = on ? d0[i] : 0.0;
        for (int t = 1; t < m; t <<= 1) {
            const int lo = lane - t >= 0 ? lane - t : lane;
            const int hi = lane + t < 64 ? lane + t : lane;
            const double am = lane_value(a, lo), bm = lane_value(b, lo), cm = lane_value(cc, lo),
                         dm = lane_value(d, lo);
            const double ap = lane_value(a, hi), bp = lane_value(b, hi), cp = lane_value(cc, hi),
                         dp = lane_value(d, hi);
            double na = 0.0, nb = b, nc = 0.0, nd = d;
            if (lane - t >= 0) {
                const double k1 = a * rcp64(bm);
                na = -am * k1;
                nb -= cm * k1;
                nd -= dm * k1;
            }
            if (lane + t < m) {
                const double k2 = cc * rcp64(bp);
                nc = -cp * k2;
                nb -= ap * k2;
                nd -= dp * k2;
            }
            a = na;
            b = nb;
            cc = nc;
            d = nd;
        }
        if (on) x[i] = d * rcp64(b);
    }
}

// --------------------------------------------------------------------------
// Per-particle geometry
// --------------------------------------------------------------------------
template <typename R>
struct Rad {
    int j;      // hat cell
    R t;        // hat weight of node j+1
    R rho;      // radius used for deposit/gather (folded at the wall)
    R sw;       // -1 beyond the wall
    R sg;       // parity of radial vectors (slab: sign(x) * sw)
    R r;        // unfolded radius
};

template <typename R, int GEOM, bool WARM>
__device__ __forceinline__ Rad<R> radial(double xd, double yd, R rmax, R h, R inv_h, int N)
{
    Rad<R> q;
    const R x = (R)xd;
    R r;
    if (GEOM == WK_CYL && WARM) {
        const R y = (R)yd;
        r = fsqrt(x * x + y * y);
    } else {
        r = fabs(x);
    }
    q.r = r;
    R rho = r, sw = (R)1;
    if (r > rmax) {
        sw = (R)-1;
        rho = (R)2 * rmax - r;
        if (rho < (R)0) rho = (R)0;
    }
    q.rho = rho;
    q.sw = sw;
    q.sg = (GEOM == WK_SLAB) ? ((x < (R)0) ? -sw : sw) : sw;
    // the double path divides like the oracle; the float path multiplies
    const R u = sizeof(R) == 8 ? rho / h : rho * inv_h;
    int j = (int)floor(u);
    j = j < 0 ? 0 : (j > N - 1 ? N - 1 : j);
    q.j = j;
    q.t = u - (R)j;
    return q;
}

template <typename R>
__device__ __forceinline__ R gather(const double* row, const Rad<R>& q)
{
    return ((R)1 - q.t) * (R)row[q.j] + q.t * (R)row[q.j + 1];
}

template <typename R>
struct Part {
    double x, y, px, py;
    R d0, w;
};

// Stage derivative d(x, y, px, py)/dxi of one particle, in the precision of
// the per-particle arithmetic.
template <typename R>
struct Deriv {
    R fx, fy, fpx, fpy;
};

// Register accumulator of NR deposit rows for the current cell of a thread.
// The per-particle terms are formed in the particle precision R and summed in
// double.
template <typename R, int NR>
struct Acc {
    int j;
    double lo[NR], hi[NR];
    __device__ __forceinline__ void reset(int jj)
    {
        j = jj;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            lo[r] = 0.0;
            hi[r] = 0.0;
        }
    }
    __device__ __forceinline__ void add(int r, const Rad<R>& q, R v)
    {
        lo[r] += (double)(v * ((R)1 - q.t));
        hi[r] += (double)(v * q.t);
    }
    // Add the sums to NR consecutive LDS rows starting at `first` (row r at
    // first + r * stride); row `skip` is left out.
    __device__ __forceinline__ void flush(double* first, int stride, int skip = -1) const
    {
        if (j < 0) return;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r != skip) {
                atomicAdd(first + r * stride + j, lo[r]);
                atomicAdd(first + r * stride + j + 1, hi[r]);
            }
        }
    }
};

// T: workgroup size.  K: particles per thread (resident) or per tile
// (streamed).  RES: the particles stay in registers for the whole march.
// BIG: the large-grid variant.  Only the deposit rows (S, J_r, J_z, M1..M5)
// are in LDS; the field, ion and solver rows are in the descriptor's
// per-workgroup global rows (d.grow), and every barrier first waits for the
// thread's stores.
//
// The descriptor a Marcher gets is its own workgroup's share of the response:
// the particle pointers and count are those of its band of cells, the grid
// and field pointers those of the whole response.
// SEL: a group exchange re-reads only the partials that have not yet arrived
// (the batched and single-response march, whose members often wait for
// partners that start later); otherwise every try reloads all of them (the
// pipelined cycle, whose members run in step).
template <typename R, int GEOM, bool WARM, int T, int K, bool RES, bool BIG = false, bool SEL = false>
struct Marcher {
    static constexpr bool kBig = BIG;
    static constexpr int kT = T;
    // With few resident particles per thread, D0 and w live in registers
    // (else in LDS slots); with at most four, the stage-1 derivative is also
    // kept in registers between the three passes that use it (else
    // recomputed: caching it for eight float particles costs more in spilled
    // registers than the recomputation).
    static constexpr bool kRegConst = RES && (K <= 4 || (K <= 8 && sizeof(R) == 4));
    static constexpr bool kCacheF = RES && K <= 4;
    MarchDesc d;
    double* sm;
    int st, N, N1, tid, lane, wid, blk;
    int kr;   // resident particles per thread: ceil(np / T), at most K
    double h;
    R hR, ihR, rmaxR, dminR;
    unsigned long long clamps, walls;
    Group grp;
    bool stores;        // this workgroup writes the fields
    bool keep_state;    // write the final resident state back to d.x ... d.py
    // resident state: positions and momenta in registers
    double X[RES ? K : 1], Y[RES ? K : 1], PX[RES ? K : 1], PY[RES ? K : 1];
    R D0r[kRegConst ? K : 1], Wr[kRegConst ? K : 1];
    R FX[kCacheF ? K : 1], FY[kCacheF ? K : 1], FPX[kCacheF ? K : 1], FPY[kCacheF ? K : 1];
    R* cd0;
    R* cw;

    // pconst: LDS for the resident D0 and w when they are not in registers
    // (2 * T * K reals)
    __device__ __forceinline__ Marcher(const MarchDesc& desc, double* smem, void* pconst = nullptr,
                                       const Group& group = Group(), bool store_fields = true,
                                       bool keep = true)
        : d(desc), sm(smem), clamps(0), walls(0), grp(group), stores(store_fields), keep_state(keep)
    {
        N = d.n_r;
        N1 = N + 1;
        st = (N1 + 1) & ~1;
        kr = RES ? (int)min((int64_t)K, (d.np + T - 1) / T) : K;
        // D0 in slots [0, T kr), w in [T kr, 2 T kr) (the launch sizes LDS so)
        cd0 = (R*)pconst;
        cw = cd0 ? cd0 + (int64_t)T * kr : nullptr;
        tid = threadIdx.x;
        lane = tid & 63;
        wid = tid >> 6;
        h = d.h;
        hR = (R)d.h;
        ihR = (R)(1.0 / d.h);
        rmaxR = (R)d.r_max;
        dminR = (R)d.d_min;
    }

    __device__ __forceinline__ double* row(int r) const
    {
        return (BIG && r >= ROW_PSI1) ? d.grow + (int64_t)(r - ROW_PSI1) * st : sm + r * st;
    }
    __device__ __forceinline__ void sync() const { block_sync<BIG>(); }

    __device__ __forceinline__ Part<R> load(int64_t i) const
    {
        Part<R> p;
        p.x = d.x[i];
        p.px = d.px[i];
        p.y = (GEOM == WK_CYL && WARM) ? d.y[i] : 0.0;
        p.py = WARM ? d.py[i] : 0.0;
        p.d0 = ((const R*)d.d0)[i];
        p.w = ((const R*)d.w)[i];
        return p;
    }

    __device__ __forceinline__ void store_state(int64_t i, const Part<R>& p) const
    {
        d.x[i] = p.x;
        d.px[i] = p.px;
        if (GEOM == WK_CYL && WARM) {
            d.y[i] = p.y;
            d.py[i] = p.py;
        }
    }

    __device__ __forceinline__ static Part<R> advance(const Part<R>& p, const Deriv<R>& g, double dt)
    {
        Part<R> q = p;
        q.x = p.x + dt * (double)g.fx;
        q.px = p.px + dt * (double)g.fpx;
        if (GEOM == WK_CYL && WARM) {
            q.y = p.y + dt * (double)g.fy;
            q.py = p.py + dt * (double)g.fpy;
        }
        return q;
    }

    // Eqs. (4)-(5) in the transverse Cartesian frame, with the field rows of
    // one stage (psi, psi', B_theta).
    __device__ __forceinline__ Deriv<R> derivative(const Part<R>& p, const double* psi, const double* dpsi,
                                                   const double* bt) const
    {
        const Rad<R> q = radial<R, GEOM, WARM>(p.x, p.y, rmaxR, hR, ihR, N);
        R D = p.d0 + gather(psi, q);
        if (D < dminR) D = dminR;
        const R px = (R)p.px;
        const R py = WARM ? (R)p.py : (R)0;
        const R p2 = px * px + py * py;
        const R iD = frcp(D);
        const R gam = ((R)1 + p2 + D * D) * ((R)0.5 * iD);
        const R F = (gam * iD) * gather(dpsi, q) - gather(bt, q);
        Deriv<R> g;
        g.fx = px * iD;
        if (GEOM == WK_CYL) {
            g.fy = WARM ? py * iD : (R)0;
            if (q.r > (R)0) {
                const R fr = q.sw * F * frcp(q.r);
                g.fpx = fr * (R)p.x;
                g.fpy = WARM ? fr * (R)p.y : (R)0;
            } else {
                g.fpx = (R)0;
                g.fpy = (R)0;
            }
        } else {
            g.fy = (R)0;
            g.fpx = q.sg * F;
            g.fpy = (R)0;
        }
        return g;
    }

    __device__ __forceinline__ void reflect(Part<R>& p)
    {
        const double rmax = d.r_max;
        if (GEOM == WK_CYL) {
            // r > r_max implies r^2 > r_max^2 (1 - 1e-12): the square root is
            // taken only for particles that may have crossed
            const double r2 = p.x * p.x + (WARM ? p.y * p.y : 0.0);
            if (r2 <= rmax * rmax * (1.0 - 1e-12)) return;
            const double r = WARM ? sqrt(r2) : fabs(p.x);
            if (r > rmax) {
                double rn = 2.0 * rmax - r;
                if (rn < 0.0) rn = 0.0;
                const double ux = p.x / r, uy = WARM ? p.y / r : 0.0;
                const double pr = ux * p.px + uy * p.py;
                p.x = rn * ux;
                p.px -= 2.0 * pr * ux;
                if (WARM) {
                    p.y = rn * uy;
                    p.py -= 2.0 * pr * uy;
                }
                ++walls;
            }
        } else {
            const double ax = fabs(p.x);
            if (ax > rmax) {
                double xn = 2.0 * rmax - ax;
                if (xn < 0.0) xn = 0.0;
                p.x = p.x < 0.0 ? -xn : xn;
                p.px = -p.px;
                ++walls;
            }
        }
    }

    // ---- deposits ------------------------------------------------------------
    __device__ __forceinline__ void dep_S(Acc<R, 1>& a, const Part<R>& p)
    {
        const Rad<R> q = radial<R, GEOM, WARM>(p.x, p.y, rmaxR, hR, ihR, N);
        if (q.j != a.j) {
            a.flush(row(ROW_S), st);
            a.reset(q.j);
        }
        a.add(0, q, p.w);
    }

    // Eqs. (1)-(3): D = D0 + psi, gamma, p_z; currents and moments of d_xi J_r.
    __device__ __forceinline__ void dep_moments(Acc<R, 7>& a, const Part<R>& p)
    {
        const Rad<R> q = radial<R, GEOM, WARM>(p.x, p.y, rmaxR, hR, ihR, N);
        R D = p.d0 + gather(row(ROW_PSI2), q);
        if (D < dminR) {
            D = dminR;
            ++clamps;
        }
        const R px = (R)p.px;
        const R py = WARM ? (R)p.py : (R)0;
        const R p2 = px * px + py * py;
        const R iD = frcp(D);
        const R h2D = (R)0.5 * iD;
        const R gam = ((R)1 + p2 + D * D) * h2D;
        const R pz = ((R)1 + p2 - D * D) * h2D;
        R pr;
        if (GEOM == WK_CYL) {
            const R x = (R)p.x;
            if (WARM) {
                const R y = (R)p.y;
                pr = q.r > (R)0 ? q.sw * (x * px + y * py) * frcp(q.r) : (R)0;
            } else {
                pr = q.r > (R)0 ? q.sw * (x * px) * frcp(q.r) : (R)0;
            }
        } else {
            pr = q.sg * px;
        }
        if (q.j != a.j) {
            flush_moments(a);
            a.reset(q.j);
        }
        const R w = p.w;
        const R wiD = w * iD;
        const R wiD2 = wiD * iD;
        a.add(0, q, -wiD * pr);
        a.add(1, q, -wiD * pz);
        a.add(2, q, wiD);
        a.add(3, q, wiD2 * (gam - pr * pr * iD));
        if (GEOM == WK_CYL && WARM) {
            if (q.rho > (R)0) {
                const R l = (R)p.x * py - (R)p.y * px;
                const R ir = frcp(q.rho);
                a.add(4, q, wiD2 * (l * l) * (ir * ir * ir));
            }
        }
        a.add(5, q, wiD2 * pr);
        a.add(6, q, wiD2 * pr * pr);
    }

    // rows JR, JZ, M1, M2, M3, M4, M5 are consecutive; M3 only for warm
    // cylindrical plasma
    __device__ __forceinline__ void flush_moments(const Acc<R, 7>& a)
    {
        a.flush(row(ROW_JR), st, (GEOM == WK_CYL && WARM) ? -1 : ROW_M3 - ROW_JR);
    }

    // ---- exchange between the workgroups of a group -------------------------
    // Sum the NR LDS rows ROWS (deposit rows, always in LDS) over the G
    // workgroups, in rank order, into every workgroup's LDS rows.  Every
    // thread calls it; the caller synchronizes afterwards.
    //
    // Exchange e (e = 1, 2, ... counted by every workgroup alike) writes the
    // partial rows into buffer slot e % 2 with the two lowest mantissa bits of
    // every value replaced by e % 4.  A reader loads the G partials of its
    // items until every tag matches, so that no separate barrier or store
    // acknowledgement is needed: a value carries its own epoch.  A workgroup
    // can only write exchange e + 2 into a slot after it has read every
    // partial of exchange e + 1, which each workgroup writes only after it has
    // read exchange e, so a slot is never overwritten while it is read.  The
    // slots start zeroed (tag 0) for every launch.  Clearing the two bits
    // changes a partial by at most 2^-51 of itself, identically for every
    // workgroup, so the group still sums identical values.
    // ROWS: the LDS row numbers, 4 bits each (row q in bits 4q..4q+3), so that
    // a row number is register arithmetic rather than a table lookup.
    template <int NR, unsigned ROWS>
    __device__ __forceinline__ static int xrow(int q)
    {
        return (int)((ROWS >> (4 * q)) & 15u);
    }

    template <int NR, unsigned ROWS>
    __device__ __forceinline__ void exchange()
    {
        // the 16-particle shape marches single workgroups only
        if (K > 8 || grp.G <= 1) return;
        const unsigned e = ++grp.epoch;
        const int64_t part = (int64_t)kXRows * st;
        double* slot = grp.xbuf + (int64_t)(e & 1u) * grp.G * part;
        double* mine = slot + (int64_t)grp.g * part;
        lds_barrier();                         // this workgroup's deposits are complete
        const int items = NR * N1;
        for (int it = tid; it < items; it += T) {
            const int q = it / N1, j = it - q * N1;
            st_dev(mine + (int64_t)q * st + j, with_tag(sm[xrow<NR, ROWS>(q) * st + j], e));
        }
        lds_barrier();                         // every row read before the sums overwrite it
        if (grp.G <= 4) sum_partials<4, 4, NR, ROWS>(slot, part, e);
        else if (grp.G <= 8) sum_partials<8, 2, NR, ROWS>(slot, part, e);
        else sum_partials<kMaxGroup, 1, NR, ROWS>(slot, part, e);
    }

    __device__ __forceinline__ static double with_tag(double v, unsigned e)
    {
        return __longlong_as_double((long long)(((unsigned long long)__double_as_longlong(v) & ~3ull) | (e & 3u)));
    }
    __device__ __forceinline__ static unsigned tag_of(double v)
    {
        return (unsigned)((unsigned long long)__double_as_longlong(v) & 3ull);
    }
    __device__ __forceinline__ static double untagged(double v)
    {
        return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(v) & ~3ull));
    }

    // The sums of exchange(): each thread takes items (row, node) tid + m T
    // in batches of B, loads the partials of a batch (MAXG >= G per item)
    // until all carry this exchange's tag, and adds them in rank order.
    template <int MAXG, int B, int NR, unsigned ROWS>
    __device__ __forceinline__ void sum_partials(const double* slot, int64_t part, unsigned e)
    {
        const int G = grp.G;
        const int items = NR * N1;
        const unsigned want = e & 3u;
        static_assert(B * MAXG <= 32, "arrival bits of a batch fit one word");
        for (int base = tid; base < items; base += B * T) {
            double v[B][MAXG];
            // bit c * MAXG + h: partial h of item c still to be read (SEL)
            unsigned missing = 0;
#pragma unroll
            for (int c = 0; c < B; ++c)
#pragma unroll
                for (int h = 0; h < MAXG; ++h) {
                    v[c][h] = 0.0;
                    if (SEL && base + c * T < items && h < G) missing |= 1u << (c * MAXG + h);
                }
            unsigned long long t0 = 0;
            unsigned tries = 0;
            for (;;) {
                // every value of the batch (SEL: every value not yet arrived),
                // all loads in flight at once
                bool ok = true;
#pragma unroll
                for (int c = 0; c < B; ++c) {
                    const int it = base + c * T;
                    const int q = it / N1, j = it - q * N1;
                    const double* src = slot + (int64_t)q * st + j;
                    if constexpr (SEL) {
#pragma unroll
                        for (int h = 0; h < MAXG; ++h)
                            if (missing & (1u << (c * MAXG + h))) v[c][h] = ld_dev(src + h * part);
#pragma unroll
                        for (int h = 0; h < MAXG; ++h) {
                            const unsigned bit = 1u << (c * MAXG + h);
                            if ((missing & bit) && tag_of(v[c][h]) == want) missing &= ~bit;
                        }
                    } else {
#pragma unroll
                        for (int h = 0; h < MAXG; ++h) {
                            const bool use = it < items && h < G;
                            v[c][h] = use ? ld_dev(src + h * part) : 0.0;
                            ok = ok && (!use || tag_of(v[c][h]) == want);
                        }
                    }
                }
                if constexpr (SEL) ok = missing == 0;
                if (ok) break;
                if (++tries > 64) {
                    // a long wait (a partner not yet started, as when a batch
                    // hands out a group's tickets over time): about 1 us
                    // between tries, so that waiting workgroups do not flood
                    // memory with reads; the abort flag and the clock are
                    // looked at every 64 tries
                    __builtin_amdgcn_s_sleep(32);
                    if ((tries & 63u) == 0) {
                        if (t0 == 0) {
                            t0 = wall_clock64();
                        } else if (wall_clock64() - t0 > kWaitTicks) {
                            st_dev(grp.abort, 1ull);
                            break;
                        }
                        if (ld_dev(grp.abort)) break;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < B; ++c) {
                const int it = base + c * T;
                if (it < items) {
                    const int q = it / N1, j = it - q * N1;
                    double s = untagged(v[c][0]);
#pragma unroll
                    for (int h = 1; h < MAXG; ++h)
                        if (h < G) s += untagged(v[c][h]);
                    sm[xrow<NR, ROWS>(q) * st + j] = s;
                }
            }
        }
    }

    // ---- solves ----------------------------------------------------------------
    // 1 / V_j of the hat volumes.
    __device__ __forceinline__ double inv_volume(int j) const
    {
        if (GEOM == WK_CYL) {
            if (j == 0) return 3.0 * rcp64(kPi * h * h);
            if (j == N) return rcp64(kPi * h * h * ((double)N - 1.0 / 3.0));
            return rcp64(2.0 * kPi * (double)j * h * h);
        }
        return (j == 0 || j == N) ? 2.0 * rcp64(h) : rcp64(h);
    }

    // Items [j0, j1) of n owned by this thread in the blocked layout of the
    // block-wide scans (q = ceil(n / T) consecutive items per thread).
    __device__ __forceinline__ void owned(int n, int& j0, int& j1) const
    {
        const int q = (n + T - 1) / T;
        j0 = min(tid * q, n);
        j1 = min(j0 + q, n);
    }

    // Exclusive prefix in thread order of one value s per thread, and the
    // workgroup total; wt holds the per-wave totals.  Contains a barrier, so
    // every thread calls it.
    __device__ __forceinline__ double block_excl(double s, double* wt, double& total) const
    {
        const double incl = wave_prefix(s);
        if (lane == 63) wt[wid] = incl;
        sync();
        constexpr int W = T >> 6;
        double before = 0.0, tot = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const double v = wt[w];
            if (w < wid) before += v;
            tot += v;
        }
        total = tot;
        return before + incl - s;
    }

    // All threads: S -> psi.  Gauss fluxes F_{j+1/2} (prefix sums over the
    // control volumes), u_j = -h F_{j+1/2} / r_{j+1/2}^a, psi_j = sum_{m >= j}
    // u_m (psi_N = 0), as two block-wide scans.  psi' follows in
    // finalize_moments.
    __device__ __forceinline__ void solve_psi(double* psi)
    {
        const double* S = row(ROW_S);
        const double* nion = row(ROW_NION);
        const double c0 = GEOM == WK_CYL ? h * h / 8.0 : 0.5 * h;
        const auto flux = [&](int j) {
            const double s = S[j] * inv_volume(j);
            return j == 0 ? (s - nion[0]) * c0 : (s - nion[j]) * (GEOM == WK_CYL ? (double)j * h : 1.0) * h;
        };
        const auto u_of = [&](int j, double F) {
            const double irph = GEOM == WK_CYL ? rcp64(((double)j + 0.5) * h) : 1.0;
            return -h * F * irph;
        };
        double* wt = scan_scratch();
        int j0, j1;
        owned(N, j0, j1);
        double s1 = 0.0;
        for (int j = j0; j < j1; ++j) s1 += flux(j);
        double ftot, utot;
        const double off1 = block_excl(s1, wt, ftot);
        double F = off1, s2 = 0.0;
        for (int j = j0; j < j1; ++j) {
            F += flux(j);
            s2 += u_of(j, F);
        }
        double U = block_excl(s2, wt + 16, utot);
        F = off1;
        for (int j = j0; j < j1; ++j) {
            F += flux(j);
            psi[j] = utot - U;
            U += u_of(j, F);
        }
        if (tid == 0) psi[N] = 0.0;
    }

    // All threads: divide the deposits by the node volumes, add the beam
    // current (when given as a row); and the node derivative psi' of this
    // stage's psi.
    __device__ __forceinline__ void finalize_moments(const double* jb_row)
    {
        const double* psi = row(ROW_PSI2);
        double* dpsi = row(ROW_DPSI2);
        const double ih = rcp64(h);
        for (int j = tid; j < N1; j += T) {
            const double iv = inv_volume(j);
            for (int r = ROW_JR; r <= ROW_M5; ++r) row(r)[j] = row(r)[j] * iv;
            if (jb_row) row(ROW_JZ)[j] += jb_row[j];
            double v;
            if (j == 0) v = 0.0;
            else if (j == N) v = (psi[N] - psi[N - 1]) * ih;
            else v = (psi[j + 1] - psi[j - 1]) * (0.5 * ih);
            dpsi[j] = v;
        }
    }

    // All threads, two passes with a barrier between: this workgroup's deposits
    // divided by the node volumes (rank 0 adds the beam current row when given;
    // psi' of this stage's psi), then the right-hand side of the B_theta
    // equation without its E_z term,
    //   Q_j = d_r J_z - M2 psi' - a M3 + r^-a d_r(r^a M5)   (rows 1..N-1),
    //   Q_N = (J_z,N + J_z,N-1) / 2                          (Eq. (6) at the wall),
    // written over row M2.  Q is linear in the deposits, so the sums over a
    // group of J_r, M1, M4 and Q are all the B_theta solve needs.
    __device__ __forceinline__ void fold_moments(const double* jb_row)
    {
        finalize_moments(grp.g == 0 ? jb_row : nullptr);
        sync();
        const double a = GEOM == WK_CYL ? 1.0 : 0.0;
        const double ih = rcp64(h);
        const double* jz = row(ROW_JZ);
        const double* m3 = row(ROW_M3);
        const double* m5 = row(ROW_M5);
        const double* dpsi = row(ROW_DPSI2);
        double* q = row(ROW_M2);
        for (int j = tid + 1; j <= N; j += T) {
            double v;
            if (j < N) {
                const double irj = GEOM == WK_CYL ? rcp64((double)j * h) : 1.0;
                const double rp = GEOM == WK_CYL ? (double)(j + 1) * h : 1.0;
                const double rm = GEOM == WK_CYL ? (double)(j - 1) * h : 1.0;
                const double m5flux = GEOM == WK_CYL ? (rp * m5[j + 1] - rm * m5[j - 1]) * (0.5 * ih) * irj
                                                     : (m5[j + 1] - m5[j - 1]) * (0.5 * ih);
                v = (jz[j + 1] - jz[j - 1]) * (0.5 * ih) - q[j] * dpsi[j] - a * m3[j] + m5flux;
            } else {
                v = 0.5 * (jz[N] + jz[N - 1]);
            }
            q[j] = v;
        }
    }

    // All threads: E_z = -int_r^{r_max} J_r dr' (Eq. (7), trapezoid rule), a
    // block-wide scan.
    __device__ __forceinline__ void solve_ez(double* ez)
    {
        const double* jr = row(ROW_JR);
        const auto w = [&](int j) { return -(0.5 * h * (jr[j] + jr[j + 1])); };
        int j0, j1;
        owned(N, j0, j1);
        double s = 0.0;
        for (int j = j0; j < j1; ++j) s += w(j);
        double tot;
        double run = block_excl(s, scan_scratch(), tot);
        for (int j = j0; j < j1; ++j) {
            ez[j] = tot - run;
            run += w(j);
        }
        if (tid == 0) ez[N] = 0.0;
    }

    // All threads: B_theta from the Helmholtz form of Eq. (6) (rows 1..N-1) and
    // Eq. (6) at the wall (row N), by parallel cyclic reduction; then zero the
    // deposit rows for the next stage.  Needs a barrier before (E_z ready).
    // FOLDED: the right-hand side without its M4 E_z term is in row M2
    // (fold_moments); otherwise it is formed here from the moment rows.
    template <bool FOLDED = false>
    __device__ __forceinline__ void solve_b(const double* dpsi, const double* ez, double* bt)
    {
        const double a = GEOM == WK_CYL ? 1.0 : 0.0;
        const double ih = rcp64(h);
        const double ih2 = ih * ih;
        const double* jz = row(ROW_JZ);
        const double* m1 = row(ROW_M1);
        const double* m2 = row(ROW_M2);
        const double* m3 = row(ROW_M3);
        const double* m4 = row(ROW_M4);
        const double* m5 = row(ROW_M5);
        double* A = row(ROW_TU);
        double* B = row(ROW_TV);
        double* C = row(ROW_TW);
        double* D = row(ROW_S);
        for (int i = tid; i < N; i += T) {
            const int j = i + 1;
            if (j < N) {
                const double irj = GEOM == WK_CYL ? rcp64((double)j * h) : 1.0;
                const double rp = GEOM == WK_CYL ? (double)(j + 1) * h : 1.0;
                const double rm = GEOM == WK_CYL ? (double)(j - 1) * h : 1.0;
                A[i] = ih2 - a * (0.5 * ih) * irj;
                B[i] = -2.0 * ih2 - a * irj * irj - m1[j];
                C[i] = ih2 + a * (0.5 * ih) * irj;
                if (FOLDED) {
                    D[i] = m2[j] + m4[j] * ez[j];
                } else {
                    const double m5flux = (rp * m5[j + 1] - rm * m5[j - 1]) * (0.5 * ih) * irj;
                    D[i] = (jz[j + 1] - jz[j - 1]) * (0.5 * ih) - m2[j] * dpsi[j] - (GEOM == WK_CYL ? m3[j] : 0.0)
                           + m4[j] * ez[j] + (GEOM == WK_CYL ? m5flux : (m5[j + 1] - m5[j - 1]) * (0.5 * ih));
                }
            } else {
                const double irh = GEOM == WK_CYL ? rcp64(((double)N - 0.5) * h) : 1.0;
                const double rNm = GEOM == WK_CYL ? (double)(N - 1) * h : 1.0;
                const double rN = GEOM == WK_CYL ? (double)N * h : 1.0;
                A[i] = -rNm * ih * irh;
                B[i] = rN * ih * irh;
                C[i] = 0.0;
                D[i] = FOLDED ? m2[N] : 0.5 * (jz[N] + jz[N - 1]);
            }
        }
        sync();
        block_pcr<BIG>(A, B, C, D, row(ROW_M2), row(ROW_M3), row(ROW_M4), row(ROW_M5), bt + 1, N);
        if (tid == 0) bt[0] = 0.0;
        sync();
        for (int j = tid; j < N1; j += T)
            for (int r = ROW_S; r <= ROW_M5; ++r) row(r)[j] = 0.0;
    }

    // The fields of slice k (one workgroup of a group writes them, with
    // device-coherent stores so that other compute units may read them during
    // the launch).
    __device__ __forceinline__ void store_fields(int k, const double* psi, const double* ez, const double* bt,
                                                 const double* dpsi)
    {
        if (!stores) return;
        R* f = (R*)d.fields;
        const int64_t plane = (int64_t)d.n_xi * N1;
        unsigned long long bad = 0;
        for (int j = tid; j < N1; j += T) {
            const double v0 = psi[j], v1 = ez[j], v2 = bt[j], v3 = -dpsi[j];
            const int64_t o = (int64_t)k * N1 + j;
            st_dev(f + o, (R)v0);
            st_dev(f + plane + o, (R)v1);
            st_dev(f + 2 * plane + o, (R)v2);
            st_dev(f + 3 * plane + o, (R)v3);
            bad += !isfinite(v0) + !isfinite(v1) + !isfinite(v2) + !isfinite(v3);
        }
        if (bad) atomicAdd(d.counters + WK_CNT_NONFINITE, bad);
    }

    // ---- particle passes ----------------------------------------------------
    // Block of K particles owned by this thread within a tile.  When whole
    // blocks tile the cells (K divides ppc and the waves cover the blocks of a
    // cell evenly), consecutive lanes take consecutive cells so that their
    // deposits land on different LDS banks.
    __device__ __forceinline__ int block_of(int t) const
    {
        const int ppc = d.ppc;
        if (kr > 0 && ppc % kr == 0) {
            const int hpc = ppc / kr;
            constexpr int W = T >> 6;
            if (hpc > 1 && W % hpc == 0) {
                const int l = t & 63, w = t >> 6;
                return l * hpc + (w % hpc) + (w / hpc) * 64 * hpc;
            }
        }
        return t;
    }

    // Resident particle m of this thread (registers; D0 and w in registers or
    // LDS slots).
    __device__ __forceinline__ Part<R> resident(int m) const
    {
        Part<R> p;
        p.x = X[m];
        p.y = Y[m];
        p.px = PX[m];
        p.py = PY[m];
        if (kRegConst) {
            p.d0 = D0r[m];
            p.w = Wr[m];
        } else {
            p.d0 = cd0[m * T + tid];
            p.w = cw[m * T + tid];
        }
        return p;
    }

    // Run fn(m, part) over this thread's particles (m: resident slot, or -1
    // when streamed); with STORE the (possibly modified) state is kept.
    template <bool STORE, typename Fn>
    __device__ __forceinline__ void for_parts(Fn fn)
    {
        if (RES) {
            const int64_t i0 = (int64_t)blk * kr;
#pragma unroll
            for (int m = 0; m < K; ++m) {
                if (m < kr && i0 + m < d.np) {
                    Part<R> p = resident(m);
                    fn(m, p);
                    if (STORE) {
                        X[m] = p.x;
                        Y[m] = p.y;
                        PX[m] = p.px;
                        PY[m] = p.py;
                    }
                }
            }
        } else {
            const int64_t per_tile = (int64_t)T * K;
            for (int64_t base = 0; base < d.np; base += per_tile) {
                const int64_t i0 = base + (int64_t)blk * K;
#pragma unroll
                for (int m = 0; m < K; ++m) {
                    const int64_t i = i0 + m;
                    if (i < d.np) {
                        Part<R> p = load(i);
                        fn(-1, p);
                        if (STORE) store_state(i, p);
                    }
                }
            }
        }
    }

    // Hooks called with the field rows of each stage: before_b(k, stage) with
    // psi, psi', E_z and the current/moment rows ready (B not yet solved),
    // after_b(k, stage, B) with B_theta solved.  No-ops by default.
    struct NoRecord {
        // true: the moment rows J_z, M1..M5 are kept (for before_b) instead of
        // being folded into the right-hand side of the B_theta equation
        static constexpr bool kKeepMoments = false;
        // true: the radii of every traj_stride-th particle are stored per slice
        static constexpr bool kTraj = false;
        __device__ __forceinline__ void before_b(Marcher&, int, int) {}
        __device__ __forceinline__ void after_b(Marcher&, int, int, const double*) {}
        // extra raw J_z deposits (before the exchange) at slice k
        __device__ __forceinline__ void deposit_beam(Marcher&, int) {}
    };

    // Run fn(i, part) over this thread's particles (read only), i the
    // particle index.
    template <typename Fn>
    __device__ __forceinline__ void for_idx(Fn fn)
    {
        if (RES) {
            const int64_t i0 = (int64_t)blk * kr;
#pragma unroll
            for (int m = 0; m < K; ++m)
                if (m < kr && i0 + m < d.np) fn(i0 + m, resident(m));
        } else {
            const int64_t per_tile = (int64_t)T * K;
            for (int64_t base = 0; base < d.np; base += per_tile) {
                const int64_t i0 = base + (int64_t)blk * K;
#pragma unroll
                for (int m = 0; m < K; ++m) {
                    const int64_t i = i0 + m;
                    if (i < d.np) fn(i, load(i));
                }
            }
        }
    }

    // Default hooks: beam current rows read from the descriptor's jb array.
    struct GlobalJb : NoRecord {
        __device__ __forceinline__ void before_slice(Marcher&, int) {}
        __device__ __forceinline__ const double* jb_row(Marcher& m, int k) { return m.d.jb + (int64_t)k * m.N1; }
        __device__ __forceinline__ void after_store(Marcher&, int) {}
    };

    __device__ __forceinline__ void run()
    {
        GlobalJb hooks;
        run(hooks);
    }

    // The march with the particle radii recorded (diagnostic variant).
    struct TrajJb : GlobalJb {
        static constexpr bool kTraj = true;
    };
    __device__ __forceinline__ void run_traj()
    {
        TrajJb hooks;
        run(hooks);
    }

    // The stage-1 derivative f_k of a particle: cached in registers for
    // resident particles (computed once per slice), else recomputed.
    template <bool FILL>
    __device__ __forceinline__ Deriv<R> fk(int m, const Part<R>& p, const double* psi1, const double* dpsi1,
                                           const double* b1)
    {
        if (kCacheF && m >= 0) {
            if (FILL) {
                const Deriv<R> g = derivative(p, psi1, dpsi1, b1);
#pragma unroll
                for (int q = 0; q < K; ++q)
                    if (q == m) {
                        FX[q] = g.fx;
                        FY[q] = g.fy;
                        FPX[q] = g.fpx;
                        FPY[q] = g.fpy;
                    }
                return g;
            }
            Deriv<R> g;
            g.fx = FX[m];
            g.fy = FY[m];
            g.fpx = FPX[m];
            g.fpy = FPY[m];
            return g;
        }
        return derivative(p, psi1, dpsi1, b1);
    }

    static constexpr unsigned kRowS = ROW_S;
    static constexpr unsigned kRowsAll = ROW_JR | ROW_JZ << 4 | ROW_M1 << 8 | ROW_M2 << 12 | ROW_M3 << 16 |
                                         ROW_M4 << 20 | ROW_M5 << 24;
    static constexpr unsigned kRowsFold = ROW_JR | ROW_M1 << 4 | ROW_M2 << 8 | ROW_M4 << 12;

    // The deposits of a stage -> the node rows the field solves use (all
    // threads; ends with a barrier).  KEEP: every moment row is kept (a single
    // workgroup); otherwise the moments are folded into J_r, M1, M4 and the
    // right-hand side Q, and those four rows are summed over the group.
    template <bool KEEP>
    __device__ __forceinline__ void moments_to_rows(const double* jb_row)
    {
        if (KEEP) {
            exchange<7, kRowsAll>();
            sync();
            finalize_moments(jb_row);
        } else {
            sync();
            fold_moments(jb_row);
            exchange<4, kRowsFold>();
        }
        sync();
    }

    // Radius of every traj_stride-th particle of the response at slice k
    // (the state Y_k the slice's fields are computed from).
    __device__ __forceinline__ void record_radii(int k)
    {
        for_idx([&](int64_t i, const Part<R>& p) {
            const int64_t gi = d.p0 + i;
            if (gi % d.traj_stride == 0) {
                const double r = (GEOM == WK_CYL && WARM) ? sqrt(p.x * p.x + p.y * p.y) : fabs(p.x);
                d.traj[(int64_t)k * d.traj_n + gi / d.traj_stride] = r;
            }
        });
    }

    template <class Hooks>
    __device__ __forceinline__ void run(Hooks& hooks)
    {
        const double dxi = d.dxi;
        const double hd = 0.5 * dxi;
        double* psi1 = row(ROW_PSI1);
        double* dpsi1 = row(ROW_DPSI1);
        double* b1 = row(ROW_B1);
        double* psi2 = row(ROW_PSI2);
        double* dpsi2 = row(ROW_DPSI2);
        double* b2 = row(ROW_B2);
        double* ez = row(ROW_EZ);
        for (int j = tid; j < N1; j += T) {
            row(ROW_NION)[j] = d.nion[j];
            for (int r = ROW_S; r <= ROW_M5; ++r) row(r)[j] = 0.0;
        }
        blk = block_of(tid);
        if (RES) {
            const int64_t i0 = (int64_t)blk * kr;
#pragma unroll
            for (int m = 0; m < K; ++m) {
                Part<R> p = Part<R>{0.0, 0.0, 0.0, 0.0, (R)1, (R)0};
                if (m < kr && i0 + m < d.np) p = load(i0 + m);
                X[m] = p.x;
                Y[m] = p.y;
                PX[m] = p.px;
                PY[m] = p.py;
                if (kRegConst) {
                    D0r[m] = p.d0;
                    Wr[m] = p.w;
                } else if (m < kr) {
                    cd0[m * T + tid] = p.d0;
                    cw[m * T + tid] = p.w;
                }
            }
        }
        sync();
        {
            Acc<R, 1> a;
            a.reset(-1);
            for_parts<false>([&](int, Part<R>& p) { dep_S(a, p); });
            a.flush(row(ROW_S), st);
        }
        exchange<1, kRowS>();
        for (int k = 0; k < d.n_xi; ++k) {
            if constexpr (Hooks::kTraj) record_radii(k);
            hooks.before_slice(*this, k);
            const double* jb0 = hooks.jb_row(*this, k);
            // ---- stage 1 at (Y_k, xi_k): psi -> moments -> E_z, B ----
            sync();
            solve_psi(psi2);
            sync();
            {
                Acc<R, 7> a;
                a.reset(-1);
                for_parts<false>([&](int, Part<R>& p) { dep_moments(a, p); });
                flush_moments(a);
            }
            hooks.deposit_beam(*this, k);
            moments_to_rows<Hooks::kKeepMoments>(jb0);
            solve_ez(ez);
            sync();
            hooks.before_b(*this, k, 0);
            solve_b<!Hooks::kKeepMoments>(dpsi2, ez, b1);
            hooks.after_b(*this, k, 0, b1);
            // keep the stage-1 psi, psi' for the derivative
            sync();
            for (int j = tid; j < N1; j += T) {
                psi1[j] = psi2[j];
                dpsi1[j] = dpsi2[j];
            }
            store_fields(k, psi2, ez, b1, dpsi2);
            hooks.after_store(*this, k);
            if (k == d.n_xi - 1) break;
            sync();
            // ---- stage 2 at (Y*, xi_{k+1}), Y* = Y_k + dxi f_k ----
            {
                Acc<R, 1> a;
                a.reset(-1);
                for_parts<false>([&](int m, Part<R>& p) {
                    dep_S(a, advance(p, fk<true>(m, p, psi1, dpsi1, b1), dxi));
                });
                a.flush(row(ROW_S), st);
            }
            exchange<1, kRowS>();
            sync();
            solve_psi(psi2);
            sync();
            {
                Acc<R, 7> a;
                a.reset(-1);
                for_parts<false>([&](int m, Part<R>& p) {
                    dep_moments(a, advance(p, fk<false>(m, p, psi1, dpsi1, b1), dxi));
                });
                flush_moments(a);
            }
            hooks.deposit_beam(*this, k + 1);
            moments_to_rows<Hooks::kKeepMoments>(hooks.jb_row(*this, k + 1));
            solve_ez(ez);
            sync();
            hooks.before_b(*this, k, 1);
            solve_b<!Hooks::kKeepMoments>(dpsi2, ez, b2);
            hooks.after_b(*this, k, 1, b2);
            sync();
            // ---- corrector Y_{k+1} = Y_k + dxi/2 (f_k + f*), deposit S(Y_{k+1}) ----
            {
                Acc<R, 1> a;
                a.reset(-1);
                for_parts<true>([&](int m, Part<R>& p) {
                    const Deriv<R> g0 = fk<false>(m, p, psi1, dpsi1, b1);
                    const Deriv<R> g1 = derivative(advance(p, g0, dxi), psi2, dpsi2, b2);
                    p.x = p.x + hd * ((double)g0.fx + (double)g1.fx);
                    p.px = p.px + hd * ((double)g0.fpx + (double)g1.fpx);
                    if (GEOM == WK_CYL && WARM) {
                        p.y = p.y + hd * ((double)g0.fy + (double)g1.fy);
                        p.py = p.py + hd * ((double)g0.fpy + (double)g1.fpy);
                    }
                    reflect(p);
                    dep_S(a, p);
                });
                a.flush(row(ROW_S), st);
            }
            exchange<1, kRowS>();
        }
        if (RES && keep_state) {
            const int64_t i0 = (int64_t)blk * kr;
#pragma unroll
            for (int m = 0; m < K; ++m)
                if (m < kr && i0 + m < d.np) store_state(i0 + m, resident(m));
        }
        if (clamps) atomicAdd(d.counters + WK_CNT_D_CLAMP, clamps);
        if (walls) atomicAdd(d.counters + WK_CNT_WALL, walls);
    }
};

}  // namespace dev
}  // namespace wk
