// Reverse-mode derivative of the witness energy gain after one plasma
// response and n beam steps in its frozen fields, with respect to the drive
// peak density, the common sigma_r, the drive sigma_z, the witness
// separation and the plasma thermal spread (Section II A model; Eq. (12)
// beam; thermal loading of the plasma).  Node rows, states and adjoints are
// double; a mixed plan does its per-particle arithmetic in float.
//
// Forward (recording): the usual march, by the group of workgroups of a
// plain response, which also writes per slice and Heun stage the node rows
// the derivative needs (psi, psi', E_z, B_theta, J_r, J_z, M1..M5: the
// "tape") and the particle state every `every` slices (checkpoints); the
// beam push keeps the state of every step.
//
// Backward: the beam push in reverse (Jacobians of each Boris step by
// forward-mode dual numbers), which gives the adjoint of the stored fields;
// then a group of workgroups, each with a share of the particles, walks the
// slices backwards.  For each segment between
// checkpoints it first recomputes the particle states of the segment from
// the checkpoint and the taped rows (particle motion needs no deposits), then
// reverses each slice: the Heun corrector and the wall reflection, the two
// stage derivatives, and each stage's field solves (transposed tridiagonal
// solve for B_theta, transposed scans for E_z and psi) and deposits (hat
// gathers of the node adjoints).  The beam-current adjoint and the loaders'
// chain rules then reduce everything to the five parameters.
#include <algorithm>

#include "wk_adjoint_dev.h"
#include "wk_marcher.h"

namespace wk {
namespace {


constexpr int kTapeRows = 11;
enum TapeRow { TP_PSI = 0, TP_DPSI, TP_EZ, TP_B, TP_JR, TP_JZ, TP_M1, TP_M2, TP_M3, TP_M4, TP_M5 };

__device__ __forceinline__ const double* tape_rows(const double* tape, int k, int stage, int N1)
{
    return tape + ((int64_t)k * 2 + stage) * kTapeRows * N1;
}

// ---------------------------------------------------------------------------
// Recording forward march
// ---------------------------------------------------------------------------
template <class M>
struct RecordHooks : M::NoRecord {
    static constexpr bool kKeepMoments = true;   // the tape holds the moment rows
    double* tape;
    double* ckpt;
    int every;
    int64_t np, p0;   // particles of the response; this member's first one
    bool writer;      // the member that writes the tape (the rows are the group's sums)
    __device__ __forceinline__ RecordHooks(double* t, double* c, int e, int64_t n, int64_t first, bool w)
        : tape(t), ckpt(c), every(e), np(n), p0(first), writer(w)
    {
    }
    __device__ __forceinline__ void before_slice(M& m, int k)
    {
        if (k % every != 0) return;
        double* c = ckpt + (int64_t)(k / every) * 4 * np + p0;
        m.for_idx([&](int64_t i, const auto& p) {
            c[i] = p.x;
            c[np + i] = p.y;
            c[2 * np + i] = p.px;
            c[3 * np + i] = p.py;
        });
    }
    __device__ __forceinline__ const double* jb_row(M& m, int k) { return m.d.jb + (int64_t)k * m.N1; }
    __device__ __forceinline__ void after_store(M&, int) {}
    __device__ __forceinline__ void before_b(M& m, int k, int stage)
    {
        if (!writer) return;
        const int N1 = m.N1;
        double* t = tape + ((int64_t)k * 2 + stage) * kTapeRows * N1;
        for (int j = m.tid; j < N1; j += M::kT) {
            t[TP_PSI * N1 + j] = m.row(ROW_PSI2)[j];
            t[TP_DPSI * N1 + j] = m.row(ROW_DPSI2)[j];
            t[TP_EZ * N1 + j] = m.row(ROW_EZ)[j];
            t[TP_JR * N1 + j] = m.row(ROW_JR)[j];
            t[TP_JZ * N1 + j] = m.row(ROW_JZ)[j];
            t[TP_M1 * N1 + j] = m.row(ROW_M1)[j];
            t[TP_M2 * N1 + j] = m.row(ROW_M2)[j];
            t[TP_M3 * N1 + j] = m.row(ROW_M3)[j];
            t[TP_M4 * N1 + j] = m.row(ROW_M4)[j];
            t[TP_M5 * N1 + j] = m.row(ROW_M5)[j];
        }
    }
    __device__ __forceinline__ void after_b(M& m, int k, int stage, const double* bt)
    {
        if (!writer) return;
        const int N1 = m.N1;
        double* t = tape + ((int64_t)k * 2 + stage) * kTapeRows * N1;
        for (int j = m.tid; j < N1; j += M::kT) t[TP_B * N1 + j] = bt[j];
    }
};

constexpr int kRecK = 8;

// The recording march of one response by a group of full.group workgroups:
// member `rank` holds the particles of cells [n_r rank / G, n_r (rank + 1) / G)
// (the split of the plain march); rank 0 stores the fields and the tape.
template <typename R, int GEOM, bool WARM, int T, bool RES>
__global__ __launch_bounds__(T) void k_march_record(MarchDesc full, double* tape, double* ckpt, int every)
{
    extern __shared__ double smem[];
    using M = dev::Marcher<R, GEOM, WARM, T, kRecK, RES, false>;
    const int rank = blockIdx.x, G = full.group;
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
    dev::Group grp;
    grp.G = G;
    grp.g = rank;
    grp.xbuf = full.xbuf;
    grp.ctr = full.gctr;
    grp.abort = full.counters + WK_CNT_PIPELINE_ABORT;
    M m(d, smem, smem + NUM_ROWS * lds_stride(full.n_r + 1), grp, rank == 0, true);
    RecordHooks<M> hooks(tape, ckpt, every, full.np, p0, rank == 0);
    m.run(hooks);
}

// ---------------------------------------------------------------------------
// Reverse march (a group of workgroups)
// ---------------------------------------------------------------------------
struct AdjDesc {
    int32_t n_r, n_xi, every, kp;   // kp: particle slots per thread of one member
    int64_t np;
    int32_t group;        // workgroups that march the reverse together
    int64_t np_m;         // particles per member (the last one may hold fewer)
    int64_t member_doubles;   // scratch doubles of one member
    double r_max, h, dxi, d_min;
    const double* d0;     // [np]
    const double* w;      // [np]
    const double* tape;
    const double* ckpt;   // [n_ckpt][4][np]
    const double* fbar;   // [4][n_xi][N1] adjoint of the stored fields
    double* jbbar;        // [n_xi][N1] adjoint of the beam current (written)
    double* scratch;      // thread-major per-particle arrays (see below)
    double* ybar_out;     // [4][np] adjoint of the loaded state
    double* d0bar_out;    // [np]
    double* wbar_out;     // [np]
    double* xbuf;         // [2][group][kRevXRows][kRevXStride] exchange slots, zeroed per launch
    unsigned long long* abort;   // set when a wait between members gives up
};

// LDS rows of the reverse march: the taped rows of the two stages of a
// slice, the node adjoints and the scratch of the transposed solve (which
// overlays the gathered-term rows G0..G6 and SB).
enum AdjRow {
    K_PSI = 0, K_DPSI, K_EZ, K_B, K_M1, K_M2, K_M4,
    S_PSI, S_DPSI, S_EZ, S_B, S_M1, S_M2, S_M4,
    A_PSI, A_DPSI, A_B, A_EZ, A_LAM, A_G0, A_G1, A_G2, A_G3, A_G4, A_G5, A_G6, A_S,
    NUM_ADJ_ROWS
};
constexpr int kSetRows = 7;   // per stage: psi, psi', E_z, B, M1, M2, M4

// The reverse march of one response runs on a group of up to kRevMaxGroup
// workgroups ("members"), each holding a contiguous share of the particles.
// The node work (transposed solves and scans) is repeated by every member;
// the node adjoints that particles deposit are summed over the group through
// device memory, four times a slice.  Without an explicit plan group a
// member holds about one particle per thread (256 x 2048 cells at 16 ppc,
// 512 threads: 8 members, reverse march 2.8x faster than one workgroup).
constexpr int kRevMaxGroup = 8;
constexpr int kRevXRows = 3;          // rows of the largest exchange
constexpr int kRevXStride = 768;      // >= n_r + 1 for every n_r whose rows fit in LDS
constexpr int kRevPerThread = 1;

// P: the type of the per-particle arithmetic of the vector-Jacobian
// products (double, or float for mixed plans, as in their forward march);
// states, rows and adjoint accumulators stay double.
template <int GEOM, bool WARM, int kAdjT, typename P>
struct Reverse {
    const AdjDesc& a;
    double* sm;
    int N, N1, st, tid, lane, wid;
    int rank, ng;           // member rank and group size
    unsigned epoch = 0;     // exchanges done
    int64_t p0, npl;        // first particle and particle count of this member
    int64_t slots;
    adj::Grid G;
    double h, ih;
    // scratch layout (thread-major; slot = m * T + tid)
    double* seg;      // [every][4][slots]
    double* yb;       // [4][slots] running state adjoint
    double* ysb;      // [4][slots] adjoint of the predictor state
    double* ys;       // [4][slots] predictor state Y*
    double* fkb;      // [4][slots] adjoint of the stage-1 derivative
    double* d0t;      // [slots]
    double* wt;       // [slots]
    double* d0b;      // [slots]
    double* wb;       // [slots]

    __device__ __forceinline__ Reverse(const AdjDesc& desc, double* smem) : a(desc), sm(smem)
    {
        N = a.n_r;
        N1 = N + 1;
        st = lds_stride(N1);
        tid = threadIdx.x;
        lane = tid & 63;
        wid = tid >> 6;
        slots = (int64_t)a.kp * kAdjT;
        rank = blockIdx.x;
        ng = a.group;
        p0 = (int64_t)rank * a.np_m;
        npl = p0 < a.np ? min(a.np_m, a.np - p0) : 0;
        G.N = N;
        G.h = a.h;
        G.rmax = a.r_max;
        G.dmin = a.d_min;
        h = a.h;
        ih = 1.0 / a.h;
        double* p = a.scratch + (int64_t)rank * a.member_doubles;
        seg = p;
        p += (int64_t)a.every * 4 * slots;
        yb = p;
        p += 4 * slots;
        ysb = p;
        p += 4 * slots;
        ys = p;
        p += 4 * slots;
        fkb = p;
        p += 4 * slots;
        d0t = p;
        p += slots;
        wt = p;
        p += slots;
        d0b = p;
        p += slots;
        wb = p;
    }

    __device__ __forceinline__ double* row(int r) const { return sm + r * st; }
    // global index of this thread's particle m, and whether it exists
    __device__ __forceinline__ int64_t pidx(int m) const { return p0 + (int64_t)tid * a.kp + m; }
    __device__ __forceinline__ bool live(int m) const { return (int64_t)tid * a.kp + m < npl; }
    __device__ __forceinline__ int64_t slot(int m) const { return (int64_t)m * kAdjT + tid; }

    // Items [j0, j1) of n owned by this thread in the blocked layout of the
    // block-wide scans (ceil(n / kAdjT) consecutive items per thread).
    __device__ __forceinline__ void owned(int n, int& j0, int& j1) const
    {
        const int q = (n + kAdjT - 1) / kAdjT;
        j0 = min(tid * q, n);
        j1 = min(j0 + q, n);
    }

    // Exclusive prefix in thread order of one value per thread and the
    // workgroup total; wt holds the per-wave totals.  Contains a barrier.
    __device__ __forceinline__ double block_excl(double s, double* wt, double& total) const
    {
        const double incl = dev::wave_prefix(s);
        if (lane == 63) wt[wid] = incl;
        __syncthreads();
        double before = 0.0, tot = 0.0;
        for (int w = 0; w < kAdjT / 64; ++w) {
            const double v = wt[w];
            if (w < wid) before += v;
            tot += v;
        }
        total = tot;
        return before + incl - s;
    }

    __device__ __forceinline__ adj::St get(const double* arr, int64_t s) const
    {
        return adj::St{arr[s], arr[slots + s], arr[2 * slots + s], arr[3 * slots + s]};
    }
    __device__ __forceinline__ void put(double* arr, int64_t s, const adj::St& v) const
    {
        arr[s] = v.x;
        arr[slots + s] = v.y;
        arr[2 * slots + s] = v.px;
        arr[3 * slots + s] = v.py;
    }

    __device__ __forceinline__ double inv_volume(int j) const
    {
        if (GEOM == WK_CYL) {
            if (j == 0) return 3.0 / (kPi * h * h);
            if (j == N) return 1.0 / (kPi * h * h * ((double)N - 1.0 / 3.0));
            return 1.0 / (2.0 * kPi * (double)j * h * h);
        }
        return (j == 0 || j == N) ? 2.0 / h : 1.0 / h;
    }

    __device__ __forceinline__ void deposit(int r, int j, double t, double v)
    {
        if (v == 0.0) return;
        atomicAdd(row(r) + j, v * (1.0 - t));
        atomicAdd(row(r) + j + 1, v * t);
    }

    // ---- sum of deposited rows over the group -------------------------------
    // Rows r0 .. r0 + NR - 1 of every member are summed in rank order into
    // every member's LDS rows (bit-identical in all members).  Exchange e
    // writes this member's rows into slot e % 2 with the two lowest mantissa
    // bits replaced by e % 4; a reader loads the partials until each carries
    // that tag.  A member writes slot e % 2 again only at exchange e + 2,
    // after it has read every partial of exchange e + 1, which no member
    // writes before it has read exchange e.  Loads and stores of one thread
    // complete in order, so a partial of exchange e + 1 that a reader has
    // seen implies that the same member's stores of exchange e are visible.
    // Every thread calls it; the caller synchronizes afterwards.
    __device__ __forceinline__ static double tagged(double v, unsigned e)
    {
        return __longlong_as_double((long long)(((unsigned long long)__double_as_longlong(v) & ~3ull) | (e & 3u)));
    }
    __device__ __forceinline__ static unsigned tag(double v)
    {
        return (unsigned)((unsigned long long)__double_as_longlong(v) & 3ull);
    }
    __device__ __forceinline__ static double untag(double v)
    {
        return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(v) & ~3ull));
    }

    template <int NR>
    __device__ __forceinline__ void group_sum(int r0)
    {
        static_assert(NR <= kRevXRows, "exchange rows");
        if (ng <= 1) return;
        constexpr int B = 2;   // items per batch: B * kRevMaxGroup loads in flight
        const unsigned e = ++epoch, want = e & 3u;
        const int64_t part = (int64_t)kRevXRows * kRevXStride;
        double* slot = a.xbuf + (int64_t)(e & 1u) * ng * part;
        double* mine = slot + (int64_t)rank * part;
        const int items = NR * N1;
        dev::lds_barrier();   // this member's deposits are complete
        for (int it = tid; it < items; it += kAdjT) {
            const int q = it / N1, j = it - q * N1;
            dev::st_dev(mine + (int64_t)q * kRevXStride + j, tagged(row(r0 + q)[j], e));
        }
        dev::lds_barrier();   // every row read before the sums overwrite it
        for (int base = tid; base < items; base += B * kAdjT) {
            double v[B][kRevMaxGroup];
            unsigned long long t0 = 0;
            unsigned tries = 0;
            for (;;) {
                bool ok = true;
#pragma unroll
                for (int c = 0; c < B; ++c) {
                    const int it = base + c * kAdjT;
                    const int q = it / N1, j = it - q * N1;
                    const double* src = slot + (int64_t)q * kRevXStride + j;
#pragma unroll
                    for (int g = 0; g < kRevMaxGroup; ++g) {
                        const bool use = it < items && g < ng;
                        v[c][g] = use ? dev::ld_dev(src + g * part) : 0.0;
                        ok = ok && (!use || tag(v[c][g]) == want);
                    }
                }
                if (ok) break;
                if (++tries > 64) {
                    // a partner that is late: about 1 us between tries; give
                    // up (and raise the abort flag) after kWaitTicks
                    __builtin_amdgcn_s_sleep(32);
                    if ((tries & 63u) == 0) {
                        if (t0 == 0) {
                            t0 = wall_clock64();
                        } else if (wall_clock64() - t0 > dev::kWaitTicks) {
                            dev::st_dev(a.abort, 1ull);
                            break;
                        }
                        if (dev::ld_dev(a.abort)) break;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < B; ++c) {
                const int it = base + c * kAdjT;
                if (it < items) {
                    const int q = it / N1, j = it - q * N1;
                    double sum = untag(v[c][0]);
#pragma unroll
                    for (int g = 1; g < kRevMaxGroup; ++g)
                        if (g < ng) sum += untag(v[c][g]);
                    row(r0 + q)[j] = sum;
                }
            }
        }
    }

    // ---- state recompute of a segment: Y_k for k = k0 .. k1 into seg ----
    __device__ __forceinline__ void recompute_segment(int k0, int k1)
    {
        const double dxi = a.dxi, hd = 0.5 * a.dxi;
        const int64_t np = a.np;
        const double* ck = a.ckpt + (int64_t)(k0 / a.every) * 4 * np;
        for (int m = 0; m < a.kp; ++m) {
            const int64_t i = pidx(m);
            if (!live(m)) continue;
            const int64_t s = slot(m);
            adj::St y{ck[i], ck[np + i], ck[2 * np + i], ck[3 * np + i]};
            const double d0 = d0t[s];
            for (int k = k0; k <= k1; ++k) {
                put(seg + (int64_t)(k - k0) * 4 * slots, s, y);
                if (k == k1) break;
                const double* t0 = tape_rows(a.tape, k, 0, N1);
                const double* t1 = tape_rows(a.tape, k, 1, N1);
                const adj::Der g0 = adj::derivative<GEOM, WARM, P>(y, d0, t0 + TP_PSI * N1, t0 + TP_DPSI * N1,
                                                                t0 + TP_B * N1, G);
                adj::St yst = y;
                yst.x = y.x + dxi * g0.fx;
                yst.px = y.px + dxi * g0.fpx;
                if (GEOM == WK_CYL && WARM) {
                    yst.y = y.y + dxi * g0.fy;
                    yst.py = y.py + dxi * g0.fpy;
                }
                const adj::Der g1 = adj::derivative<GEOM, WARM, P>(yst, d0, t1 + TP_PSI * N1, t1 + TP_DPSI * N1,
                                                                t1 + TP_B * N1, G);
                y.x = y.x + hd * (g0.fx + g1.fx);
                y.px = y.px + hd * (g0.fpx + g1.fpx);
                if (GEOM == WK_CYL && WARM) {
                    y.y = y.y + hd * (g0.fy + g1.fy);
                    y.py = y.py + hd * (g0.fpy + g1.fpy);
                }
                adj::reflect<GEOM, WARM>(y, a.r_max);
            }
        }
    }

    __device__ __forceinline__ void load_set(int base, int k, int stage)
    {
        const double* t = tape_rows(a.tape, k, stage, N1);
        for (int j = tid; j < N1; j += kAdjT) {
            row(base + 0)[j] = t[TP_PSI * N1 + j];
            row(base + 1)[j] = t[TP_DPSI * N1 + j];
            row(base + 2)[j] = t[TP_EZ * N1 + j];
            row(base + 3)[j] = t[TP_B * N1 + j];
            row(base + 4)[j] = t[TP_M1 * N1 + j];
            row(base + 5)[j] = t[TP_M2 * N1 + j];
            row(base + 6)[j] = t[TP_M4 * N1 + j];
        }
    }

    __device__ __forceinline__ void zero_seeds()
    {
        for (int j = tid; j < N1; j += kAdjT) {
            row(A_PSI)[j] = 0.0;
            row(A_DPSI)[j] = 0.0;
            row(A_B)[j] = 0.0;
            row(A_EZ)[j] = 0.0;
        }
    }

    // adjoint of the stored fields of slice k: psi, E_z, B, W = -psi'
    __device__ __forceinline__ void seed_fields(int k)
    {
        const int64_t plane = (int64_t)a.n_xi * N1;
        const double* f = a.fbar + (int64_t)k * N1;
        for (int j = tid; j < N1; j += kAdjT) {
            row(A_PSI)[j] += f[j];
            row(A_EZ)[j] += f[plane + j];
            row(A_B)[j] += f[2 * plane + j];
            row(A_DPSI)[j] -= f[3 * plane + j];
        }
    }

    // forward coefficients of row i (node i + 1) of the B_theta system
    __device__ __forceinline__ void b_coef(const double* m1, int i, double& A, double& B, double& C) const
    {
        const double al = GEOM == WK_CYL ? 1.0 : 0.0;
        const double ih2 = ih * ih;
        const int j = i + 1;
        if (j < N) {
            const double irj = GEOM == WK_CYL ? 1.0 / ((double)j * h) : 1.0;
            A = ih2 - al * (0.5 * ih) * irj;
            B = -2.0 * ih2 - al * irj * irj - m1[j];
            C = ih2 + al * (0.5 * ih) * irj;
        } else {
            const double irh = GEOM == WK_CYL ? 1.0 / (((double)N - 0.5) * h) : 1.0;
            const double rNm = GEOM == WK_CYL ? (double)(N - 1) * h : 1.0;
            const double rN = GEOM == WK_CYL ? (double)N * h : 1.0;
            A = -rNm * ih * irh;
            B = rN * ih * irh;
            C = 0.0;
        }
    }

    // Node part of a stage's reverse: B adjoint -> lambda (transposed solve)
    // -> adjoints of J_z, M1..M5, psi', E_z; E_z adjoint -> J_r adjoint.
    // Leaves the gathered-term rows G0..G6 (divided by the node volumes);
    // adds the J_z adjoint to the beam-current adjoint of slice kj.
    // Every member computes the same node adjoints; rank 0 alone adds the
    // beam-current adjoint.  The other members clear their psi adjoint row,
    // into which the particle pass after this one deposits: the exchange
    // that follows adds rank 0's (already summed) row to the group's
    // deposits.
    __device__ __forceinline__ void node_reverse(int base, int kj)
    {
        if (rank != 0)
            for (int j = tid; j < N1; j += kAdjT) row(A_PSI)[j] = 0.0;
        const double* m1 = row(base + 4);
        // transposed system in the scratch rows
        double* ta = row(A_G0);
        double* tb = row(A_G1);
        double* tc = row(A_G2);
        double* td = row(A_G3);
        for (int i = tid; i < N; i += kAdjT) {
            double A, B, C, Am, Bm, Cm, Ap, Bp, Cp;
            b_coef(m1, i, A, B, C);
            ta[i] = 0.0;
            tc[i] = 0.0;
            if (i >= 1) {
                b_coef(m1, i - 1, Am, Bm, Cm);
                ta[i] = Cm;
            }
            if (i + 1 <= N - 1) {
                b_coef(m1, i + 1, Ap, Bp, Cp);
                tc[i] = Ap;
            }
            tb[i] = B;
            td[i] = row(A_B)[i + 1];
        }
        __syncthreads();
        dev::block_pcr(ta, tb, tc, td, row(A_G4), row(A_G5), row(A_G6), row(A_S), row(A_LAM), N);
        __syncthreads();
        const double* psd = row(base + 1);
        const double* ez = row(base + 2);
        const double* bt = row(base + 3);
        const double* m2 = row(base + 5);
        const double* m4 = row(base + 6);
        const double* lam = row(A_LAM);
        auto L = [&](int j) { return (j >= 1 && j <= N) ? lam[j - 1] : 0.0; };
        double* jbb = a.jbbar + (int64_t)kj * N1;
        for (int j = tid; j < N1; j += kAdjT) {
            const double iv = inv_volume(j);
            const bool in = j >= 1 && j <= N - 1;
            double ajz = 0.0;
            if (j - 1 >= 1 && j - 1 <= N - 1) ajz += L(j - 1) * (0.5 * ih);
            if (j + 1 >= 1 && j + 1 <= N - 1) ajz -= L(j + 1) * (0.5 * ih);
            if (j == N || j == N - 1) ajz += 0.5 * L(N);
            double am5 = 0.0;
            if (j - 1 >= 1 && j - 1 <= N - 1)
                am5 += L(j - 1) * (GEOM == WK_CYL ? (double)j / (double)(j - 1) : 1.0) * (0.5 * ih);
            if (j + 1 >= 1 && j + 1 <= N - 1)
                am5 -= L(j + 1) * (GEOM == WK_CYL ? (double)j / (double)(j + 1) : 1.0) * (0.5 * ih);
            const double lj = in ? L(j) : 0.0;
            if (rank == 0) jbb[j] += ajz;
            row(A_G1)[j] = ajz * iv;
            row(A_G2)[j] = lj * bt[j] * iv;
            row(A_G3)[j] = -lj * psd[j] * iv;
            row(A_G4)[j] = (GEOM == WK_CYL ? -lj : 0.0) * iv;
            row(A_G5)[j] = lj * ez[j] * iv;
            row(A_G6)[j] = am5 * iv;
            row(A_DPSI)[j] -= lj * m2[j];
            row(A_EZ)[j] += lj * m4[j];
        }
        __syncthreads();
        // E_z = -int_r^{r_max} J_r (trapezoid): J_r adjoint from prefix sums
        // (a block-wide scan)
        {
            double* pre = row(A_LAM);
            const double* ezb = row(A_EZ);
            int j0, j1;
            owned(N, j0, j1);
            double s = 0.0;
            for (int j = j0; j < j1; ++j) s += ezb[j];
            double tot;
            double run = block_excl(s, dev::scan_scratch(), tot);
            for (int j = j0; j < j1; ++j) {
                run += ezb[j];
                pre[j] = run;
            }
            __syncthreads();
            for (int m = tid; m < N1; m += kAdjT) {
                const double pm = m <= N - 1 ? pre[m] : 0.0;
                const double pm1 = m >= 1 ? pre[m - 1] : 0.0;
                row(A_G0)[m] = -(0.5 * h) * (pm + pm1) * inv_volume(m);
            }
        }
        __syncthreads();
    }

    // psi' adjoint -> psi adjoint; psi adjoint -> S adjoint (transposed scans,
    // block-wide).
    __device__ __forceinline__ void psi_reverse()
    {
        for (int t = tid; t < N1; t += kAdjT) {
            const double* dp = row(A_DPSI);
            double v = 0.0;
            if (t - 1 >= 1 && t - 1 <= N - 1) v += dp[t - 1] * (0.5 * ih);
            if (t + 1 >= 1 && t + 1 <= N - 1) v -= dp[t + 1] * (0.5 * ih);
            if (t == N) v += dp[N] * ih;
            if (t == N - 1) v -= dp[N] * ih;
            row(A_LAM)[t] = v;
        }
        __syncthreads();
        for (int t = tid; t < N1; t += kAdjT) row(A_PSI)[t] += row(A_LAM)[t];
        __syncthreads();
        {
            // F_j = -h / r_{j+1/2} * sum_{m <= j} psibar_m; Sbar_m from the
            // suffix sums of F
            const double* pb = row(A_PSI);
            double* S = row(A_S);
            double* wt = dev::scan_scratch();
            const auto f_of = [&](int j, double incl) {
                const double irph = GEOM == WK_CYL ? 1.0 / (((double)j + 0.5) * h) : 1.0;
                return -h * irph * incl;
            };
            int j0, j1;
            owned(N, j0, j1);
            double s1 = 0.0;
            for (int j = j0; j < j1; ++j) s1 += pb[j];
            double t1, tot;
            const double off1 = block_excl(s1, wt, t1);
            double run = off1, s2 = 0.0;
            for (int j = j0; j < j1; ++j) {
                run += pb[j];
                s2 += f_of(j, run);
            }
            double e = block_excl(s2, wt + 16, tot);
            const double c0 = GEOM == WK_CYL ? h * h / 8.0 : 0.5 * h;
            run = off1;
            for (int j = j0; j < j1; ++j) {
                run += pb[j];
                const double coef = j == 0 ? c0 : (GEOM == WK_CYL ? (double)j * h : 1.0) * h;
                S[j] = (tot - e) * coef * inv_volume(j);
                e += f_of(j, run);
            }
            if (tid == 0) S[N] = 0.0;
        }
        __syncthreads();
    }

    // particle pass: adjoint of the deposited currents and moments at the
    // states `st` (thread-major) with the psi row of `base`; accumulates the
    // state adjoint into `acc`
    __device__ __forceinline__ void moments_pass(int base, const double* stt, double* acc)
    {
        const double* psi = row(base + 0);
        for (int m = 0; m < a.kp; ++m) {
            if (!live(m)) continue;
            const int64_t s = slot(m);
            const adj::St y = get(stt, s);
            const adj::GeoT<P> g = adj::geo_of<GEOM, WARM, P>(y, G);
            double gr[7], dr[7];
#pragma unroll
            for (int r = 0; r < 7; ++r) {
                const double* R = row(A_G0 + r);
                const double v0 = R[g.j], v1 = R[g.j + 1];
                gr[r] = (1.0 - g.t) * v0 + g.t * v1;
                dr[r] = v1 - v0;
            }
            adj::St sb = get(acc, s);
            double d0bar = d0b[s], wbar = wb[s];
            const adj::DerAdj o =
                adj::moment_terms_vjp<GEOM, WARM, P>(y, d0t[s], wt[s], psi, G, gr, dr, sb, d0bar, wbar);
            deposit(A_PSI, o.j, o.t, o.gpsi);
            put(acc, s, sb);
            d0b[s] = d0bar;
            wb[s] = wbar;
        }
    }

    // particle pass: adjoint of the S deposit at the states `stt`
    __device__ __forceinline__ void s_pass(const double* stt, double* acc)
    {
        for (int m = 0; m < a.kp; ++m) {
            if (!live(m)) continue;
            const int64_t s = slot(m);
            const adj::St y = get(stt, s);
            adj::St sb = get(acc, s);
            double wbar = wb[s];
            adj::s_term_vjp<GEOM, WARM, P>(y, wt[s], G, row(A_S), sb, wbar);
            put(acc, s, sb);
            wb[s] = wbar;
        }
    }

    __device__ __forceinline__ void run()
    {
        const int64_t np = a.np;
        const int nx = a.n_xi;
        const double dxi = a.dxi, hd = 0.5 * a.dxi;
        for (int m = 0; m < a.kp; ++m) {
            const int64_t i = pidx(m), s = slot(m);
            const bool ok = live(m);
            d0t[s] = ok ? a.d0[i] : 1.0;
            wt[s] = ok ? a.w[i] : 0.0;
            d0b[s] = 0.0;
            wb[s] = 0.0;
            put(yb, s, adj::St{0.0, 0.0, 0.0, 0.0});
        }
        // (same thread-to-node mapping as the accumulation in node_reverse)
        if (rank == 0)
            for (int k = 0; k < nx; ++k)
                for (int j = tid; j < N1; j += kAdjT) a.jbbar[(int64_t)k * N1 + j] = 0.0;
        const int nseg = (nx - 1) / a.every + 1;
        for (int sgi = nseg - 1; sgi >= 0; --sgi) {
            const int k0 = sgi * a.every;
            const int k1 = min(k0 + a.every - 1, nx - 1);
            recompute_segment(k0, k1);
            for (int k = k1; k >= k0; --k) {
                const double* yk = seg + (int64_t)(k - k0) * 4 * slots;
                __syncthreads();
                load_set(0, k, 0);
                zero_seeds();
                if (k < nx - 1) {
                    load_set(kSetRows, k, 1);
                    __syncthreads();
                    // corrector, reflection and the stage-2 derivative
                    for (int m = 0; m < a.kp; ++m) {
                        if (!live(m)) continue;
                        const int64_t s = slot(m);
                        const adj::St y = get(yk, s);
                        const double d0 = d0t[s];
                        const adj::Der g0 =
                            adj::derivative<GEOM, WARM, P>(y, d0, row(K_PSI), row(K_DPSI), row(K_B), G);
                        adj::St yst = y;
                        yst.x = y.x + dxi * g0.fx;
                        yst.px = y.px + dxi * g0.fpx;
                        if (GEOM == WK_CYL && WARM) {
                            yst.y = y.y + dxi * g0.fy;
                            yst.py = y.py + dxi * g0.fpy;
                        }
                        const adj::Der g1 =
                            adj::derivative<GEOM, WARM, P>(yst, d0, row(S_PSI), row(S_DPSI), row(S_B), G);
                        adj::St yt = y;
                        yt.x = y.x + hd * (g0.fx + g1.fx);
                        yt.px = y.px + hd * (g0.fpx + g1.fpx);
                        if (GEOM == WK_CYL && WARM) {
                            yt.y = y.y + hd * (g0.fy + g1.fy);
                            yt.py = y.py + hd * (g0.fpy + g1.fpy);
                        }
                        adj::St probe = yt;
                        adj::St b = get(yb, s);
                        if (adj::reflect<GEOM, WARM>(probe, a.r_max)) adj::reflect_vjp<GEOM, WARM>(yt, a.r_max, b);
                        // Y_{k+1} = Y_k + dxi/2 (f_k + f*)
                        const adj::Der fb{hd * b.x, hd * b.y, hd * b.px, hd * b.py};
                        adj::St sb{0.0, 0.0, 0.0, 0.0};
                        double d0bar = d0b[s];
                        const adj::DerAdj o = adj::derivative_vjp<GEOM, WARM, P>(yst, d0, row(S_PSI), row(S_DPSI),
                                                                              row(S_B), G, fb, sb, d0bar);
                        deposit(A_PSI, o.j, o.t, o.gpsi);
                        deposit(A_DPSI, o.j, o.t, o.gdpsi);
                        deposit(A_B, o.j, o.t, o.gb);
                        put(yb, s, b);
                        put(ysb, s, sb);
                        put(ys, s, yst);
                        put(fkb, s, adj::St{fb.fx, fb.fy, fb.fpx, fb.fpy});
                        d0b[s] = d0bar;
                    }
                    group_sum<3>(A_PSI);
                    __syncthreads();
                    // stage 2 at (Y*, xi_{k+1})
                    node_reverse(kSetRows, k + 1);
                    moments_pass(kSetRows, ys, ysb);
                    group_sum<1>(A_PSI);
                    __syncthreads();
                    psi_reverse();
                    zero_seeds();
                    __syncthreads();
                    // S adjoint at Y*, then Y* = Y_k + dxi f_k and the stage-1 derivative
                    for (int m = 0; m < a.kp; ++m) {
                        if (!live(m)) continue;
                        const int64_t s = slot(m);
                        const adj::St yst = get(ys, s);
                        adj::St sb = get(ysb, s);
                        double wbar = wb[s];
                        adj::s_term_vjp<GEOM, WARM, P>(yst, wt[s], G, row(A_S), sb, wbar);
                        wb[s] = wbar;
                        adj::St b = get(yb, s);
                        b.x += sb.x;
                        b.y += sb.y;
                        b.px += sb.px;
                        b.py += sb.py;
                        const adj::St f0 = get(fkb, s);
                        const adj::Der fb{f0.x + dxi * sb.x, f0.y + dxi * sb.y, f0.px + dxi * sb.px,
                                          f0.py + dxi * sb.py};
                        const adj::St y = get(yk, s);
                        double d0bar = d0b[s];
                        const adj::DerAdj o = adj::derivative_vjp<GEOM, WARM, P>(y, d0t[s], row(K_PSI), row(K_DPSI),
                                                                              row(K_B), G, fb, b, d0bar);
                        deposit(A_PSI, o.j, o.t, o.gpsi);
                        deposit(A_DPSI, o.j, o.t, o.gdpsi);
                        deposit(A_B, o.j, o.t, o.gb);
                        put(yb, s, b);
                        d0b[s] = d0bar;
                    }
                    group_sum<3>(A_PSI);
                }
                __syncthreads();
                // stage 1 at (Y_k, xi_k), seeded by the stored fields of slice k
                seed_fields(k);
                __syncthreads();
                node_reverse(0, k);
                moments_pass(0, yk, yb);
                group_sum<1>(A_PSI);
                __syncthreads();
                psi_reverse();
                s_pass(yk, yb);
            }
        }
        for (int m = 0; m < a.kp; ++m) {
            const int64_t i = pidx(m), s = slot(m);
            if (!live(m)) continue;
            const adj::St b = get(yb, s);
            a.ybar_out[i] = b.x;
            a.ybar_out[np + i] = b.y;
            a.ybar_out[2 * np + i] = b.px;
            a.ybar_out[3 * np + i] = b.py;
            a.d0bar_out[i] = d0b[s];
            a.wbar_out[i] = wb[s];
        }
    }
};

template <int GEOM, bool WARM, int T, typename P>
__global__ __launch_bounds__(T) void k_adjoint_march(AdjDesc a)
{
    extern __shared__ double smem[];
    Reverse<GEOM, WARM, T, P> r(a, smem);
    r.run();
}

// ---------------------------------------------------------------------------
// Beam: recorded push, push adjoint, current adjoint
// ---------------------------------------------------------------------------
constexpr int kBlk = 256;

struct BeamGeom {
    int geom, n_r, n_xi;
    double r_max, h, xi_min, dxi;
};

// history: [n_steps + 1][6][n] (x, y, xi, px, py, pz)
template <typename FT>
__global__ __launch_bounds__(kBlk) void k_push_record(BeamGeom g, int64_t n, wk_beam_bufs b, const FT* fields,
                                                      int n_steps, double dt, double* hist,
                                                      unsigned long long* counters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t plane = (int64_t)g.n_xi * (g.n_r + 1);
    double x = b.d_x[i], y = b.d_y[i], xi = b.d_xi[i], px = b.d_px[i], py = b.d_py[i], pz = b.d_pz[i];
    unsigned long long out = 0;
    for (int s = 0; s <= n_steps; ++s) {
        double* H = hist + (int64_t)s * 6 * n;
        H[i] = x;
        H[n + i] = y;
        H[2 * n + i] = xi;
        H[3 * n + i] = px;
        H[4 * n + i] = py;
        H[5 * n + i] = pz;
        if (s == n_steps) break;
        const adj::BeamCell c = adj::boris_step<double, FT>(g.geom, g.n_r, g.n_xi, g.r_max, g.h, g.xi_min, g.dxi,
                                                        fields + plane, fields + 2 * plane, fields + 3 * plane, x,
                                                        y, xi, px, py, pz, dt, false);
        out += c.inside ? 0 : 1;
    }
    b.d_x[i] = x;
    b.d_y[i] = y;
    b.d_xi[i] = xi;
    b.d_px[i] = px;
    b.d_py[i] = py;
    b.d_pz[i] = pz;
    if (out) atomicAdd(counters + WK_CNT_BEAM_OUT_PUSH, out);
}

// sum of the witness weights (deterministic: one block)
__global__ __launch_bounds__(1024) void k_witness_weight(int64_t n, wk_beam_bufs b, double* out)
{
    __shared__ double sw[1024];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        if (b.d_tag[i] == 1) v += b.d_w[i];
    sw[threadIdx.x] = v;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sw[threadIdx.x] += sw[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sw[0];
}

// Reverse of the recorded push: state adjoint at the end from the gain
// (witness: W / sum W * p / gamma), then back through each Boris step;
// the adjoint of the gathered fields goes to fbar ([4][n_xi][N1], planes
// E_z, B, W) with the bilinear weights.  sb0: [6][n] adjoint of the state
// before the push.
template <typename FT>
__global__ __launch_bounds__(kBlk) void k_push_adjoint(BeamGeom g, int64_t n, wk_beam_bufs b, const FT* fields,
                                                       int n_steps, double dt, const double* hist,
                                                       const double* wsum, double* fbar, double* sb0)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int N1 = g.n_r + 1;
    const int64_t plane = (int64_t)g.n_xi * N1;
    double sb[6] = {0, 0, 0, 0, 0, 0};
    if (b.d_tag[i] == 1 && wsum[0] > 0.0) {
        const double* H = hist + (int64_t)n_steps * 6 * n;
        const double px = H[3 * n + i], py = H[4 * n + i], pz = H[5 * n + i];
        const double gam = sqrt(1.0 + px * px + py * py + pz * pz);
        const double c = b.d_w[i] / wsum[0] / gam;
        sb[3] = c * px;
        sb[4] = c * py;
        sb[5] = c * pz;
    }
    for (int s = n_steps - 1; s >= 0; --s) {
        const double* H = hist + (int64_t)s * 6 * n;
        adj::Dual v[6];
        for (int q = 0; q < 6; ++q) {
            v[q] = adj::Dual(H[(int64_t)q * n + i]);
            v[q].d[q] = 1.0;
        }
        const adj::BeamCell c =
            adj::boris_step<adj::Dual, FT>(g.geom, g.n_r, g.n_xi, g.r_max, g.h, g.xi_min, g.dxi, fields + plane,
                                       fields + 2 * plane, fields + 3 * plane, v[0], v[1], v[2], v[3], v[4], v[5],
                                       dt, true);
        double nb[6], fb[3];
        for (int q = 0; q < 6; ++q) {
            double acc = 0.0;
            for (int o = 0; o < 6; ++o) acc += sb[o] * v[o].d[q];
            nb[q] = acc;
        }
        for (int f = 0; f < 3; ++f) {
            double acc = 0.0;
            for (int o = 0; o < 6; ++o) acc += sb[o] * v[o].d[6 + f];
            fb[f] = acc;
        }
        if (c.inside) {
            const double x = H[i], y = H[n + i], xi = H[2 * n + i];
            const double r = g.geom == WK_CYL ? sqrt(x * x + y * y) : fabs(x);
            const double tr = r / g.h - (double)c.j;
            const double u = (xi - g.xi_min) / g.dxi;
            const double tk = u - (double)c.k;
            const double tk1 = c.k + 1 < g.n_xi ? tk : 0.0;
            const double w00 = (1.0 - tr) * (1.0 - tk1), w01 = tr * (1.0 - tk1);
            const double w10 = (1.0 - tr) * tk1, w11 = tr * tk1;
            const int64_t o0 = (int64_t)c.k * N1 + c.j, o1 = (int64_t)c.k1 * N1 + c.j;
            for (int f = 0; f < 3; ++f) {
                if (fb[f] == 0.0) continue;
                double* F = fbar + (int64_t)(f + 1) * plane;
                atomicAdd(F + o0, fb[f] * w00);
                atomicAdd(F + o0 + 1, fb[f] * w01);
                atomicAdd(F + o1, fb[f] * w10);
                atomicAdd(F + o1 + 1, fb[f] * w11);
            }
        }
        for (int q = 0; q < 6; ++q) sb[q] = nb[q];
    }
    for (int q = 0; q < 6; ++q) sb0[(int64_t)q * n + i] = sb[q];
}

__device__ __forceinline__ double node_volume(const BeamGeom& g, int j)
{
    const int N = g.n_r;
    const double h = g.h;
    if (g.geom == WK_CYL) {
        if (j == 0) return kPi * h * h / 3.0;
        if (j == N) return kPi * h * h * ((double)N - 1.0 / 3.0);
        return 2.0 * kPi * (double)j * h * h;
    }
    return (j == 0 || j == N) ? 0.5 * h : h;
}

// Adjoint of J_bz = -sum W hat_j(r) hat_k(xi) / (V_j dxi) at the loaded beam
// (hist step 0): adds to the position/xi adjoints in sb0 and writes the
// weight adjoint wb.
__global__ __launch_bounds__(kBlk) void k_current_adjoint(BeamGeom g, int64_t n, wk_beam_bufs b, const double* hist,
                                                          const double* jbbar, double* sb0, double* wbar)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int N1 = g.n_r + 1;
    const double x = hist[i], y = hist[n + i], xi = hist[2 * n + i];
    const double W = b.d_w[i];
    const double r = g.geom == WK_CYL ? sqrt(x * x + y * y) : fabs(x);
    const double xi_max = g.xi_min + g.n_xi * g.dxi;
    double wb = 0.0;
    if (!(r > g.r_max || xi < g.xi_min || xi >= xi_max)) {
        const double ur = r / g.h;
        int j = (int)floor(ur);
        j = j < 0 ? 0 : (j > g.n_r - 1 ? g.n_r - 1 : j);
        const double tr = ur - (double)j;
        const double u = (xi - g.xi_min) / g.dxi;
        int k = (int)floor(u);
        if (k > g.n_xi - 1) k = g.n_xi - 1;
        const double tk = u - (double)k;
        auto A = [&](int kk, int jj) { return -jbbar[(int64_t)kk * N1 + jj] / (node_volume(g, jj) * g.dxi); };
        const double a00 = A(k, j), a01 = A(k, j + 1);
        const bool two = k + 1 < g.n_xi;
        const double a10 = two ? A(k + 1, j) : 0.0, a11 = two ? A(k + 1, j + 1) : 0.0;
        wb = (1.0 - tr) * (1.0 - tk) * a00 + tr * (1.0 - tk) * a01 + (1.0 - tr) * tk * a10 + tr * tk * a11;
        const double trb = W * ((1.0 - tk) * (a01 - a00) + tk * (a11 - a10));
        const double tkb = W * ((1.0 - tr) * (a10 - a00) + tr * (a11 - a01));
        const double rb = trb / g.h;
        sb0[2 * n + i] += tkb / g.dxi;
        if (g.geom == WK_CYL) {
            if (r > 0.0) {
                sb0[i] += rb * x / r;
                sb0[n + i] += rb * y / r;
            }
        } else {
            sb0[i] += rb * (x < 0.0 ? -1.0 : (x > 0.0 ? 1.0 : 0.0));
        }
    }
    wbar[i] = wb;
}

// ---------------------------------------------------------------------------
// Loader chain rules, reduced to the five parameters
// ---------------------------------------------------------------------------
struct ThetaArgs {
    int geom;
    int64_t n_beam, n_drive, np;
    double n_d, sigma_r, sigma_zd, u_th;
    const double* beam_draws;    // [n_beam][4]
    const double* sb0;           // [6][n_beam]
    const double* wbar_beam;     // [n_beam]
    const double* beam_w;        // [n_beam]
    const double* plasma_draws;  // [np/2][3] (warm)
    const double* ybar;          // [4][np]
    const double* d0bar;         // [np]
    const double* wbar;          // [np]
    const double* pw;            // [np] plasma weights
    const double* pd0;           // [np] plasma D0
};

constexpr int kThetaBlocks = 256;

__global__ __launch_bounds__(kBlk) void k_theta_partial(ThetaArgs t, double* part)
{
    __shared__ double red[5][kBlk];
    double acc[5] = {0, 0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const double rexp = t.geom == WK_CYL ? 2.0 : 1.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < t.n_beam; i += stride) {
        const double* e = t.beam_draws + 4 * i;
        const double xb = t.sb0[i], yb = t.sb0[t.n_beam + i], xib = t.sb0[2 * t.n_beam + i];
        const double W = t.beam_w[i], Wb = t.wbar_beam[i];
        acc[1] += xb * e[0] + (t.geom == WK_CYL ? yb * e[1] : 0.0) + Wb * W * rexp / t.sigma_r;
        if (i < t.n_drive) {
            acc[0] += Wb * W / t.n_d;
            acc[2] += xib * e[2] + Wb * W / t.sigma_zd;
        } else {
            acc[3] += xib;
        }
    }
    if (t.u_th > 0.0) {
        const double u = t.u_th;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < t.np; i += stride) {
            const int64_t q = i / 2;
            const double sg = (i % 2 == 0) ? 1.0 : -1.0;
            const double* e = t.plasma_draws + 3 * q;
            const double e2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
            const double g0 = sqrt(1.0 + u * u * e2);
            const double dg0 = u * e2 / g0;
            const double D0 = t.pd0[i];
            const double dD0 = dg0 - sg * e[2];
            const double half = t.pw[i] * g0 / D0;
            const double dw = half * (dD0 * g0 - D0 * dg0) / (g0 * g0);
            acc[4] += t.ybar[2 * t.np + i] * sg * e[0] + t.ybar[3 * t.np + i] * sg * e[1] + t.d0bar[i] * dD0 +
                      t.wbar[i] * dw;
        }
    }
    for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 5; ++c) part[(int64_t)blockIdx.x * 5 + c] = red[c][0];
}

// A reverse march whose members gave up waiting for each other has no
// gradient: NaN.
__global__ void k_theta_final(const double* part, int nb, const double* gbar, const unsigned long long* abort,
                              double* grad)
{
    if (blockIdx.x != 0 || threadIdx.x >= 5) return;
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += part[(int64_t)i * 5 + threadIdx.x];
    grad[threadIdx.x] = *abort ? __builtin_nan("") : gbar[0] * s;
}

__global__ void k_zero_f64(double* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

int64_t blocks_for(int64_t n, int b) { return (n + b - 1) / b; }

template <typename R, int GEOM, bool WARM>
hipError_t launch_record_t(const MarchDesc& d, int threads, double* tape, double* ckpt, int every, hipStream_t s)
{
    const size_t lds = march_lds_bytes(d.n_r + 1, threads);
    auto go = [&](auto kern, size_t bytes) -> hipError_t {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(d.group), dim3(threads), bytes, s, d, tape, ckpt, every);
        return hipGetLastError();
    };
    // the largest member's particles
    const int64_t np = (int64_t)((d.n_r + d.group - 1) / d.group) * d.ppc;
    const size_t extra = 2 * (size_t)threads * std::min<int64_t>(kRecK, (np + threads - 1) / threads) * sizeof(double);
    const bool res = np <= (int64_t)threads * kRecK && lds + extra <= 159 * 1024;
    switch (threads) {
    case 256:
        return res ? go(k_march_record<R, GEOM, WARM, 256, true>, lds + extra)
                   : go(k_march_record<R, GEOM, WARM, 256, false>, lds);
    case 512:
        return res ? go(k_march_record<R, GEOM, WARM, 512, true>, lds + extra)
                   : go(k_march_record<R, GEOM, WARM, 512, false>, lds);
    case 1024:
        return res ? go(k_march_record<R, GEOM, WARM, 1024, true>, lds + extra)
                   : go(k_march_record<R, GEOM, WARM, 1024, false>, lds);
    default:
        return hipErrorInvalidValue;
    }
}

template <int GEOM, bool WARM, int T, typename P>
hipError_t launch_reverse_tt(const AdjDesc& a, hipStream_t s)
{
    const size_t lds = (size_t)NUM_ADJ_ROWS * lds_stride(a.n_r + 1) * sizeof(double);
    auto kern = k_adjoint_march<GEOM, WARM, T, P>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(a.group), dim3(T), lds, s, a);
    return hipGetLastError();
}

template <int GEOM, bool WARM, typename P>
hipError_t launch_reverse_t(const AdjDesc& a, int threads, hipStream_t s)
{
    switch (threads) {
    case 256: return launch_reverse_tt<GEOM, WARM, 256, P>(a, s);
    case 512: return launch_reverse_tt<GEOM, WARM, 512, P>(a, s);
    default: return launch_reverse_tt<GEOM, WARM, 1024, P>(a, s);
    }
}

template <typename P>
hipError_t launch_reverse_p(const AdjDesc& a, int geom, bool warm, int threads, hipStream_t s)
{
    if (geom == WK_CYL)
        return warm ? launch_reverse_t<WK_CYL, true, P>(a, threads, s) : launch_reverse_t<WK_CYL, false, P>(a, threads, s);
    return warm ? launch_reverse_t<WK_SLAB, true, P>(a, threads, s) : launch_reverse_t<WK_SLAB, false, P>(a, threads, s);
}

// Plasma constants of a mixed plan (float) as double for the reverse pass.
__global__ void k_to_f64(const float* in, double* out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

}  // namespace

size_t adjoint_lds_bytes(int n_nodes) { return (size_t)NUM_ADJ_ROWS * lds_stride(n_nodes) * sizeof(double); }
size_t adjoint_tape_doubles(int n_xi, int n_nodes) { return (size_t)n_xi * 2 * kTapeRows * n_nodes; }
// Particles per member and per-member scratch of a reverse march by G
// workgroups of `threads`.
static int64_t member_particles(int64_t np, int G) { return (np + G - 1) / G; }
static int64_t member_doubles(int64_t np, int every, int threads, int G)
{
    const int64_t kp = (member_particles(np, G) + threads - 1) / threads;
    const int64_t slots = kp * threads;
    return (int64_t)every * 4 * slots + 16 * slots + 4 * slots;
}
static int reverse_group(int64_t np, int threads, int plan_group)
{
    if (plan_group > 0) return std::min(plan_group, kRevMaxGroup);
    const int64_t per = (int64_t)kRevPerThread * threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(kRevMaxGroup, (np + per - 1) / per));
}
static int64_t exchange_doubles() { return 2 * (int64_t)kRevMaxGroup * kRevXRows * kRevXStride + 1; }

// Enough for any group size: the members' scratch, the exchange slots and
// the abort flag.
size_t adjoint_scratch_doubles(int64_t np, int every, int threads)
{
    int64_t most = 0;
    for (int G = 1; G <= kRevMaxGroup; ++G) most = std::max(most, G * member_doubles(np, every, threads, G));
    return (size_t)(most + exchange_doubles());
}

template <typename R>
hipError_t launch_record_r(const MarchDesc& d, int threads, double* tape, double* ckpt, int every, hipStream_t s)
{
    if (d.geom == WK_CYL)
        return d.warm ? launch_record_t<R, WK_CYL, true>(d, threads, tape, ckpt, every, s)
                      : launch_record_t<R, WK_CYL, false>(d, threads, tape, ckpt, every, s);
    return d.warm ? launch_record_t<R, WK_SLAB, true>(d, threads, tape, ckpt, every, s)
                  : launch_record_t<R, WK_SLAB, false>(d, threads, tape, ckpt, every, s);
}

hipError_t launch_march_record(const MarchDesc& d, int prec, int threads, double* tape, double* ckpt, int every,
                               hipStream_t s)
{
    return prec == WK_FP64 ? launch_record_r<double>(d, threads, tape, ckpt, every, s)
                           : launch_record_r<float>(d, threads, tape, ckpt, every, s);
}

hipError_t launch_gradient_backward(const GradDesc& gd, hipStream_t s)
{
    const BeamGeom bg{gd.grid.geom, gd.grid.n_r, gd.grid.n_xi, gd.grid.r_max, gd.grid.h, gd.grid.xi_min,
                      gd.grid.dxi};
    const int N1 = gd.grid.n_r + 1;
    const int64_t plane = (int64_t)gd.grid.n_xi * N1;
    const int64_t nb = gd.n_beam;
    hipLaunchKernelGGL(k_zero_f64, dim3(blocks_for(4 * plane, kBlk)), dim3(kBlk), 0, s, gd.fbar, 4 * plane);
    hipLaunchKernelGGL(k_witness_weight, dim3(1), dim3(1024), 0, s, nb, gd.beam, gd.wsum);
    if (gd.prec == WK_FP64)
        hipLaunchKernelGGL(k_push_adjoint<double>, dim3(blocks_for(nb, kBlk)), dim3(kBlk), 0, s, bg, nb, gd.beam,
                           (const double*)gd.fields, gd.n_steps, gd.dt, gd.hist, gd.wsum, gd.fbar, gd.sb0);
    else
        hipLaunchKernelGGL(k_push_adjoint<float>, dim3(blocks_for(nb, kBlk)), dim3(kBlk), 0, s, bg, nb, gd.beam,
                           (const float*)gd.fields, gd.n_steps, gd.dt, gd.hist, gd.wsum, gd.fbar, gd.sb0);
    const double* pd0 = (const double*)gd.march.d0;
    const double* pw = (const double*)gd.march.w;
    if (gd.prec != WK_FP64) {
        const int64_t np = gd.march.np;
        hipLaunchKernelGGL(k_to_f64, dim3(blocks_for(np, kBlk)), dim3(kBlk), 0, s, (const float*)gd.march.d0,
                           gd.d0_f64, np);
        hipLaunchKernelGGL(k_to_f64, dim3(blocks_for(np, kBlk)), dim3(kBlk), 0, s, (const float*)gd.march.w,
                           gd.w_f64, np);
        pd0 = gd.d0_f64;
        pw = gd.w_f64;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (N1 > kRevXStride) return hipErrorInvalidValue;
    AdjDesc a;
    a.n_r = gd.grid.n_r;
    a.n_xi = gd.grid.n_xi;
    a.every = gd.every;
    a.np = gd.march.np;
    a.group = reverse_group(a.np, gd.threads, gd.march.group);
    a.np_m = member_particles(a.np, a.group);
    a.kp = (int)((a.np_m + gd.threads - 1) / gd.threads);
    a.member_doubles = member_doubles(a.np, gd.every, gd.threads, a.group);
    a.xbuf = gd.scratch + (int64_t)a.group * a.member_doubles;
    a.abort = (unsigned long long*)(a.xbuf + exchange_doubles() - 1);
    hipLaunchKernelGGL(k_zero_f64, dim3(blocks_for(exchange_doubles(), kBlk)), dim3(kBlk), 0, s, a.xbuf,
                       exchange_doubles());
    a.r_max = gd.grid.r_max;
    a.h = gd.grid.h;
    a.dxi = gd.grid.dxi;
    a.d_min = gd.march.d_min;
    a.d0 = pd0;
    a.w = pw;
    a.tape = gd.tape;
    a.ckpt = gd.ckpt;
    a.fbar = gd.fbar;
    a.jbbar = gd.jbbar;
    a.scratch = gd.scratch;
    a.ybar_out = gd.ybar;
    a.d0bar_out = gd.d0bar;
    a.wbar_out = gd.wbar;
    e = gd.prec == WK_FP64 ? launch_reverse_p<double>(a, gd.grid.geom, gd.march.warm != 0, gd.threads, s)
                           : launch_reverse_p<float>(a, gd.grid.geom, gd.march.warm != 0, gd.threads, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_current_adjoint, dim3(blocks_for(nb, kBlk)), dim3(kBlk), 0, s, bg, nb, gd.beam, gd.hist,
                       gd.jbbar, gd.sb0, gd.wbar_beam);
    ThetaArgs t;
    t.geom = gd.grid.geom;
    t.n_beam = nb;
    t.n_drive = gd.n_drive;
    t.np = gd.march.np;
    t.n_d = gd.n_d;
    t.sigma_r = gd.sigma_r;
    t.sigma_zd = gd.sigma_zd;
    t.u_th = gd.u_th;
    t.beam_draws = gd.beam_draws;
    t.sb0 = gd.sb0;
    t.wbar_beam = gd.wbar_beam;
    t.beam_w = gd.beam.d_w;
    t.plasma_draws = gd.plasma_draws;
    t.ybar = gd.ybar;
    t.d0bar = gd.d0bar;
    t.wbar = gd.wbar;
    t.pw = pw;
    t.pd0 = pd0;
    hipLaunchKernelGGL(k_theta_partial, dim3(kThetaBlocks), dim3(kBlk), 0, s, t, gd.partials);
    hipLaunchKernelGGL(k_theta_final, dim3(1), dim3(64), 0, s, gd.partials, kThetaBlocks, gd.gbar, a.abort, gd.grad);
    return hipGetLastError();
}

hipError_t launch_push_record(const GridDesc& g, int64_t n, const wk_beam_bufs& b, const void* fields, int prec,
                              int n_steps, double dt, double* hist, unsigned long long* counters, hipStream_t s)
{
    const BeamGeom bg{g.geom, g.n_r, g.n_xi, g.r_max, g.h, g.xi_min, g.dxi};
    if (n <= 0) return hipSuccess;
    if (prec == WK_FP64)
        hipLaunchKernelGGL(k_push_record<double>, dim3(blocks_for(n, kBlk)), dim3(kBlk), 0, s, bg, n, b,
                           (const double*)fields, n_steps, dt, hist, counters);
    else
        hipLaunchKernelGGL(k_push_record<float>, dim3(blocks_for(n, kBlk)), dim3(kBlk), 0, s, bg, n, b,
                           (const float*)fields, n_steps, dt, hist, counters);
    return hipGetLastError();
}

size_t theta_partials_doubles() { return (size_t)kThetaBlocks * 5; }

}  // namespace wk
