// Plasma response march (a3-a8): one persistent workgroup per instance.
//
// Each workgroup holds the radial grid of its instance in LDS and marches all
// slices of the xi window without leaving the kernel: per slice two Heun
// stages, each stage = deposit of the xi-flux S -> psi solve -> gather psi ->
// deposit of the currents and the moments of d_xi J_r -> E_z quadrature ->
// B_theta tridiagonal solve -> gather -> stage derivative (WAKE paper,
// Section II A, Eqs. (1)-(7)).  Synchronization is workgroup barriers only.
// Particles stream through registers in tiles of `threads * K`; deposits are
// LDS atomics in double; solves are block-wide scans and parallel cyclic
// reduction in double.
#include "wk_internal.h"

namespace wk {
namespace {

__device__ inline double node_volume(int geom, int j, int N, double h)
{
    if (geom == WK_CYL) {
        if (j == 0) return kPi * h * h / 3.0;
        if (j == N) return kPi * h * h * ((double)N - 1.0 / 3.0);
        return 2.0 * kPi * (double)j * h * h;
    }
    return (j == 0 || j == N) ? 0.5 * h : h;
}

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
__device__ inline Rad<R> radial(double xd, double yd, R rmax, R h, int N)
{
    Rad<R> q;
    const R x = (R)xd;
    R r;
    if (GEOM == WK_CYL && WARM) {
        const R y = (R)yd;
        r = sqrt(x * x + y * y);
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
    const R u = rho / h;
    int j = (int)floor(u);
    j = j < 0 ? 0 : (j > N - 1 ? N - 1 : j);
    q.j = j;
    q.t = u - (R)j;
    return q;
}

template <typename R>
__device__ inline R gather(const double* row, const Rad<R>& q)
{
    return ((R)1 - q.t) * (R)row[q.j] + q.t * (R)row[q.j + 1];
}

template <typename R>
__device__ inline void deposit(double* row, const Rad<R>& q, R v)
{
    atomicAdd(row + q.j, (double)(v * ((R)1 - q.t)));
    atomicAdd(row + q.j + 1, (double)(v * q.t));
}

template <typename R>
struct Part {
    double x, y, px, py;
    R d0, w;
};

struct Deriv {
    double fx, fy, fpx, fpy;
};

// Block-wide inclusive prefix (reverse = false) or suffix (reverse = true)
// sum of v[0..n) in LDS, in place.  Three barriers.
__device__ void block_scan(double* v, int n, bool reverse, double* wsum)
{
    const int T = blockDim.x, tid = threadIdx.x;
    const int per = (n + T - 1) / T;
    const int beg = tid * per;
    const int end = beg + per < n ? beg + per : n;
    double run = 0.0;
    for (int i = beg; i < end; ++i) run += v[reverse ? n - 1 - i : i];
    double incl = run;
    const int lane = tid & 63, wid = tid >> 6, nw = T >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        double s = lane < nw ? wsum[lane] : 0.0;
        for (int off = 1; off < 64; off <<= 1) {
            const double o = __shfl_up(s, off, 64);
            if (lane >= off) s += o;
        }
        if (lane < nw) wsum[lane] = s;
    }
    __syncthreads();
    double base = incl - run + (wid > 0 ? wsum[wid - 1] : 0.0);
    for (int i = beg; i < end; ++i) {
        const int ii = reverse ? n - 1 - i : i;
        base += v[ii];
        v[ii] = base;
    }
    __syncthreads();
}

// Parallel cyclic reduction of the tridiagonal system with rows (a, b, c, d)
// in buffer 0 (a[0] and c[n-1] ignored); buffer 1 is scratch.  Solution in x.
__device__ void pcr_solve(double* a0, double* b0, double* c0, double* d0,
                          double* a1, double* b1, double* c1, double* d1, double* x, int n)
{
    const int T = blockDim.x, tid = threadIdx.x;
    for (int i = tid; i < n; i += T) {
        if (i == 0) a0[0] = 0.0;
        if (i == n - 1) c0[n - 1] = 0.0;
    }
    __syncthreads();
    for (int s = 1; s < n; s <<= 1) {
        for (int i = tid; i < n; i += T) {
            double na = 0.0, nb = b0[i], nc = 0.0, nd = d0[i];
            if (i - s >= 0) {
                const double k1 = a0[i] / b0[i - s];
                na = -a0[i - s] * k1;
                nb -= c0[i - s] * k1;
                nd -= d0[i - s] * k1;
            }
            if (i + s < n) {
                const double k2 = c0[i] / b0[i + s];
                nc = -c0[i + s] * k2;
                nb -= a0[i + s] * k2;
                nd -= d0[i + s] * k2;
            }
            a1[i] = na;
            b1[i] = nb;
            c1[i] = nc;
            d1[i] = nd;
        }
        __syncthreads();
        double* t;
        t = a0; a0 = a1; a1 = t;
        t = b0; b0 = b1; b1 = t;
        t = c0; c0 = c1; c1 = t;
        t = d0; d0 = d1; d1 = t;
    }
    for (int i = tid; i < n; i += T) x[i] = d0[i] / b0[i];
    __syncthreads();
}

template <typename R, int GEOM, bool WARM, int K>
struct Marcher {
    const MarchDesc& d;
    double* sm;
    double* wsum;
    int st, N, N1, T, tid;
    double h;
    R hR, rmaxR, dminR;
    unsigned long long clamps, walls;

    __device__ Marcher(const MarchDesc& desc, double* smem)
        : d(desc), sm(smem), clamps(0), walls(0)
    {
        N = d.n_r;
        N1 = N + 1;
        st = (N1 + 1) & ~1;
        wsum = sm + NUM_ROWS * st;
        T = blockDim.x;
        tid = threadIdx.x;
        h = d.h;
        hR = (R)d.h;
        rmaxR = (R)d.r_max;
        dminR = (R)d.d_min;
    }

    __device__ double* row(int r) const { return sm + r * st; }

    __device__ Part<R> load(int64_t i) const
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

    __device__ void store_state(int64_t i, const Part<R>& p) const
    {
        d.x[i] = p.x;
        d.px[i] = p.px;
        if (GEOM == WK_CYL && WARM) {
            d.y[i] = p.y;
            d.py[i] = p.py;
        }
    }

    __device__ Deriv load_fk(int64_t i) const
    {
        const R* f = (const R*)d.fk;
        Deriv g;
        g.fx = (double)f[i];
        g.fpx = (double)f[2 * d.np + i];
        g.fy = (GEOM == WK_CYL && WARM) ? (double)f[d.np + i] : 0.0;
        g.fpy = (GEOM == WK_CYL && WARM) ? (double)f[3 * d.np + i] : 0.0;
        return g;
    }

    __device__ void store_fk(int64_t i, const Deriv& g) const
    {
        R* f = (R*)d.fk;
        f[i] = (R)g.fx;
        f[2 * d.np + i] = (R)g.fpx;
        if (GEOM == WK_CYL && WARM) {
            f[d.np + i] = (R)g.fy;
            f[3 * d.np + i] = (R)g.fpy;
        }
    }

    __device__ Part<R> advance(const Part<R>& p, const Deriv& g, double dt) const
    {
        Part<R> q = p;
        q.x = p.x + dt * g.fx;
        q.px = p.px + dt * g.fpx;
        if (GEOM == WK_CYL && WARM) {
            q.y = p.y + dt * g.fy;
            q.py = p.py + dt * g.fpy;
        }
        return q;
    }

    __device__ void deposit_S(const Part<R>& p)
    {
        const Rad<R> q = radial<R, GEOM, WARM>(p.x, p.y, rmaxR, hR, N);
        deposit(row(ROW_S), q, p.w);
    }

    // Eqs. (1)-(3): D = D0 + psi, gamma, p_z; deposit the currents and the
    // moments of d_xi J_r.
    __device__ void deposit_moments(const Part<R>& p)
    {
        const Rad<R> q = radial<R, GEOM, WARM>(p.x, p.y, rmaxR, hR, N);
        R D = p.d0 + gather(row(ROW_PSI), q);
        if (D < dminR) {
            D = dminR;
            ++clamps;
        }
        const R px = (R)p.px;
        const R py = WARM ? (R)p.py : (R)0;
        const R p2 = px * px + py * py;
        const R gam = ((R)1 + p2 + D * D) / ((R)2 * D);
        const R pz = ((R)1 + p2 - D * D) / ((R)2 * D);
        R pr;
        if (GEOM == WK_CYL) {
            const R x = (R)p.x;
            if (WARM) {
                const R y = (R)p.y;
                pr = q.r > (R)0 ? q.sw * (x * px + y * py) / q.r : (R)0;
            } else {
                pr = q.r > (R)0 ? q.sw * (x * px) / q.r : (R)0;
            }
        } else {
            pr = q.sg * px;
        }
        const R w = p.w;
        deposit(row(ROW_JR), q, -w * pr / D);
        deposit(row(ROW_JZ), q, -w * pz / D);
        deposit(row(ROW_M1), q, w / D);
        deposit(row(ROW_M2), q, w * (gam / (D * D) - pr * pr / (D * D * D)));
        if (GEOM == WK_CYL && WARM) {
            if (q.rho > (R)0) {
                const R l = (R)p.x * py - (R)p.y * px;
                deposit(row(ROW_M3), q, w * (l * l) / (D * D * q.rho * q.rho * q.rho));
            }
        }
        deposit(row(ROW_M4), q, w * pr / (D * D));
        deposit(row(ROW_M5), q, w * pr * pr / (D * D));
    }

    // Eqs. (4)-(5) in the transverse Cartesian frame.
    __device__ Deriv derivative(const Part<R>& p) const
    {
        const Rad<R> q = radial<R, GEOM, WARM>(p.x, p.y, rmaxR, hR, N);
        R D = p.d0 + gather(row(ROW_PSI), q);
        if (D < dminR) D = dminR;
        const R px = (R)p.px;
        const R py = WARM ? (R)p.py : (R)0;
        const R p2 = px * px + py * py;
        const R gam = ((R)1 + p2 + D * D) / ((R)2 * D);
        const R F = (gam / D) * gather(row(ROW_DPSI), q) - gather(row(ROW_B), q);
        Deriv g;
        g.fx = (double)(px / D);
        if (GEOM == WK_CYL) {
            g.fy = WARM ? (double)(py / D) : 0.0;
            if (q.r > (R)0) {
                g.fpx = (double)(q.sw * F * (R)p.x / q.r);
                g.fpy = WARM ? (double)(q.sw * F * (R)p.y / q.r) : 0.0;
            } else {
                g.fpx = 0.0;
                g.fpy = 0.0;
            }
        } else {
            g.fy = 0.0;
            g.fpx = (double)(q.sg * F);
            g.fpy = 0.0;
        }
        return g;
    }

    __device__ void reflect(Part<R>& p)
    {
        const double rmax = d.r_max;
        if (GEOM == WK_CYL) {
            const double r = WARM ? sqrt(p.x * p.x + p.y * p.y) : fabs(p.x);
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

    __device__ void zero_rows(int r0, int r1)
    {
        for (int r = r0; r < r1; ++r)
            for (int j = tid; j < N1; j += T) row(r)[j] = 0.0;
    }

    // S -> psi (conservative Poisson form) and node psi'.
    __device__ void solve_psi()
    {
        double* S = row(ROW_S);
        double* psi = row(ROW_PSI);
        const double* nion = row(ROW_NION);
        const double alpha = GEOM == WK_CYL ? 1.0 : 0.0;
        // Gauss fluxes F_{j+1/2} = sum of (S - n_ion) over the control volumes
        for (int j = tid; j < N; j += T) {
            const double s = S[j] / node_volume(GEOM, j, N, h);
            double g;
            if (j == 0) g = (s - nion[0]) * (GEOM == WK_CYL ? h * h / 8.0 : 0.5 * h);
            else g = (s - nion[j]) * (GEOM == WK_CYL ? (double)j * h : 1.0) * h;
            psi[j] = g;
        }
        __syncthreads();
        block_scan(psi, N, false, wsum);
        for (int j = tid; j < N; j += T) {
            const double rph = GEOM == WK_CYL ? ((double)j + 0.5) * h : 1.0;
            psi[j] = -h * psi[j] / rph;
        }
        __syncthreads();
        (void)alpha;
        block_scan(psi, N, true, wsum);
        for (int j = tid; j < N1; j += T) {
            if (j == N) psi[N] = 0.0;
        }
        __syncthreads();
        double* dpsi = row(ROW_DPSI);
        for (int j = tid; j < N1; j += T) {
            double v;
            if (j == 0) v = 0.0;
            else if (j == N) v = (psi[N] - psi[N - 1]) / h;
            else v = (psi[j + 1] - psi[j - 1]) / (2.0 * h);
            dpsi[j] = v;
        }
        __syncthreads();
    }

    // E_z quadrature of Eq. (7) and the Helmholtz form of Eq. (6) for B_theta.
    __device__ void solve_ez_b(const double* jb_row)
    {
        // finalize the deposits (divide by the node volumes, add the beam current)
        for (int j = tid; j < N1; j += T) {
            const double V = node_volume(GEOM, j, N, h);
            for (int r = ROW_JR; r <= ROW_M5; ++r) row(r)[j] = row(r)[j] / V;
            row(ROW_JZ)[j] += jb_row[j];
        }
        __syncthreads();
        double* ez = row(ROW_EZ);
        const double* jr = row(ROW_JR);
        for (int j = tid; j < N1; j += T) ez[j] = j < N ? -(0.5 * h * (jr[j] + jr[j + 1])) : 0.0;
        __syncthreads();
        block_scan(ez, N, true, wsum);
        const double a = GEOM == WK_CYL ? 1.0 : 0.0;
        const double h2 = h * h;
        double* A = row(ROW_PA);
        double* Bc = row(ROW_PB);
        double* C = row(ROW_PC);
        double* Dd = row(ROW_PD);
        const double* jz = row(ROW_JZ);
        const double* m1 = row(ROW_M1);
        const double* m2 = row(ROW_M2);
        const double* m3 = row(ROW_M3);
        const double* m4 = row(ROW_M4);
        const double* m5 = row(ROW_M5);
        const double* dpsi = row(ROW_DPSI);
        for (int j = tid + 1; j <= N; j += T) {
            const int i = j - 1;
            if (j < N) {
                const double rj = (double)j * h;
                const double ra = GEOM == WK_CYL ? rj : 1.0;
                const double rp = GEOM == WK_CYL ? (double)(j + 1) * h : 1.0;
                const double rm = GEOM == WK_CYL ? (double)(j - 1) * h : 1.0;
                A[i] = 1.0 / h2 - a / (2.0 * rj * h);
                Bc[i] = -2.0 / h2 - a / (rj * rj) - m1[j];
                C[i] = 1.0 / h2 + a / (2.0 * rj * h);
                const double m5flux = (rp * m5[j + 1] - rm * m5[j - 1]) / (2.0 * h * ra);
                Dd[i] = (jz[j + 1] - jz[j - 1]) / (2.0 * h) - m2[j] * dpsi[j] - a * m3[j]
                        + m4[j] * ez[j] + m5flux;
            } else {
                const double rh = GEOM == WK_CYL ? ((double)N - 0.5) * h : 1.0;
                const double rNm = GEOM == WK_CYL ? (double)(N - 1) * h : 1.0;
                const double rN = GEOM == WK_CYL ? (double)N * h : 1.0;
                A[i] = -rNm / (h * rh);
                Bc[i] = rN / (h * rh);
                C[i] = 0.0;
                Dd[i] = 0.5 * (jz[N] + jz[N - 1]);
            }
        }
        __syncthreads();
        // buffer 1 of the reduction reuses rows dead after the right-hand side
        double* Bout = row(ROW_B);
        pcr_solve(A, Bc, C, Dd, row(ROW_M2), row(ROW_M3), row(ROW_M4), row(ROW_M5), Bout + 1, N);
        if (tid == 0) Bout[0] = 0.0;
        __syncthreads();
    }

    __device__ void store_fields(int k)
    {
        R* f = (R*)d.fields;
        const int64_t plane = (int64_t)d.n_xi * N1;
        unsigned long long bad = 0;
        for (int j = tid; j < N1; j += T) {
            const double v0 = row(ROW_PSI)[j], v1 = row(ROW_EZ)[j], v2 = row(ROW_B)[j];
            const double v3 = -row(ROW_DPSI)[j];
            const int64_t o = (int64_t)k * N1 + j;
            f[o] = (R)v0;
            f[plane + o] = (R)v1;
            f[2 * plane + o] = (R)v2;
            f[3 * plane + o] = (R)v3;
            bad += !isfinite(v0) + !isfinite(v1) + !isfinite(v2) + !isfinite(v3);
        }
        if (bad) atomicAdd(d.counters + WK_CNT_NONFINITE, bad);
    }

    template <typename Fn>
    __device__ void for_tiles(Fn fn)
    {
        const int64_t per_tile = (int64_t)T * K;
        for (int64_t base = 0; base < d.np; base += per_tile) {
            const int64_t i0 = base + (int64_t)tid * K;
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const int64_t i = i0 + m;
                if (i < d.np) fn(i);
            }
        }
    }

    __device__ void run()
    {
        const double dxi = d.dxi;
        const double hd = 0.5 * dxi;
        for (int j = tid; j < N1; j += T) row(ROW_NION)[j] = d.nion[j];
        zero_rows(ROW_S, ROW_S + 1);
        __syncthreads();
        for_tiles([&](int64_t i) { deposit_S(load(i)); });
        for (int k = 0; k < d.n_xi; ++k) {
            const double* jb0 = d.jb + (int64_t)k * N1;
            // ---- stage 1 at (Y_k, xi_k) ----
            zero_rows(ROW_JR, ROW_M5 + 1);
            __syncthreads();
            solve_psi();
            for_tiles([&](int64_t i) { deposit_moments(load(i)); });
            __syncthreads();
            solve_ez_b(jb0);
            store_fields(k);
            if (k == d.n_xi - 1) break;
            zero_rows(ROW_S, ROW_S + 1);
            __syncthreads();
            for_tiles([&](int64_t i) {
                const Part<R> p = load(i);
                const Deriv g = derivative(p);
                store_fk(i, g);
                deposit_S(advance(p, g, dxi));
            });
            zero_rows(ROW_JR, ROW_M5 + 1);
            __syncthreads();
            // ---- stage 2 at (Y*, xi_{k+1}) ----
            solve_psi();
            for_tiles([&](int64_t i) { deposit_moments(advance(load(i), load_fk(i), dxi)); });
            __syncthreads();
            solve_ez_b(jb0 + N1);
            zero_rows(ROW_S, ROW_S + 1);
            __syncthreads();
            for_tiles([&](int64_t i) {
                Part<R> p = load(i);
                const Deriv g0 = load_fk(i);
                const Deriv g1 = derivative(advance(p, g0, dxi));
                p.x = p.x + hd * (g0.fx + g1.fx);
                p.px = p.px + hd * (g0.fpx + g1.fpx);
                if (GEOM == WK_CYL && WARM) {
                    p.y = p.y + hd * (g0.fy + g1.fy);
                    p.py = p.py + hd * (g0.fpy + g1.fpy);
                }
                reflect(p);
                store_state(i, p);
                deposit_S(p);
            });
            // the predictor fields of the next slice read S only after
            // the barrier at the top of the loop
        }
        if (clamps) atomicAdd(d.counters + WK_CNT_D_CLAMP, clamps);
        if (walls) atomicAdd(d.counters + WK_CNT_WALL, walls);
    }
};

template <typename R, int GEOM, bool WARM, int T, int K>
__global__ __launch_bounds__(T) void k_march_one(MarchDesc d)
{
    extern __shared__ double smem[];
    Marcher<R, GEOM, WARM, K> m(d, smem);
    m.run();
}

template <typename R, int GEOM, bool WARM, int T, int K>
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
        Marcher<R, GEOM, WARM, K> m(d, smem);
        m.run();
        __syncthreads();
    }
}

template <typename R, int GEOM, bool WARM, int T>
hipError_t launch_one_t(const MarchDesc& d, hipStream_t s)
{
    constexpr int K = 4;
    const size_t lds = march_lds_bytes(d.n_r + 1, T);
    auto kern = k_march_one<R, GEOM, WARM, T, K>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(1), dim3(T), lds, s, d);
    return hipGetLastError();
}

template <typename R, int GEOM, bool WARM, int T>
hipError_t launch_batch_t(const MarchDesc* descs, int n, int max_nodes, int grid, unsigned int* next,
                          hipStream_t s)
{
    constexpr int K = 4;
    const size_t lds = march_lds_bytes(max_nodes, T);
    auto kern = k_march_batch<R, GEOM, WARM, T, K>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(T), lds, s, descs, n, next);
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
hipError_t launch_batch_w(const MarchDesc* descs, int n, int max_nodes, int threads, int grid,
                          unsigned int* next, hipStream_t s)
{
    switch (threads) {
    case 256: return launch_batch_t<R, GEOM, WARM, 256>(descs, n, max_nodes, grid, next, s);
    case 512: return launch_batch_t<R, GEOM, WARM, 512>(descs, n, max_nodes, grid, next, s);
    default: return launch_batch_t<R, GEOM, WARM, 1024>(descs, n, max_nodes, grid, next, s);
    }
}

template <typename R>
hipError_t launch_one_r(const MarchDesc& d, int threads, hipStream_t s)
{
    if (d.geom == WK_CYL) {
        return d.warm ? launch_one_w<R, WK_CYL, true>(d, threads, s)
                      : launch_one_w<R, WK_CYL, false>(d, threads, s);
    }
    return d.warm ? launch_one_w<R, WK_SLAB, true>(d, threads, s)
                  : launch_one_w<R, WK_SLAB, false>(d, threads, s);
}

template <typename R>
hipError_t launch_batch_r(const MarchDesc* descs, int n, int max_nodes, int geom, int warm,
                          int threads, int grid, unsigned int* next, hipStream_t s)
{
    if (geom == WK_CYL) {
        return warm ? launch_batch_w<R, WK_CYL, true>(descs, n, max_nodes, threads, grid, next, s)
                    : launch_batch_w<R, WK_CYL, false>(descs, n, max_nodes, threads, grid, next, s);
    }
    return warm ? launch_batch_w<R, WK_SLAB, true>(descs, n, max_nodes, threads, grid, next, s)
                : launch_batch_w<R, WK_SLAB, false>(descs, n, max_nodes, threads, grid, next, s);
}

}  // namespace

hipError_t launch_march(const MarchDesc& d, int prec, MarchShape shape, hipStream_t stream)
{
    return prec == WK_FP64 ? launch_one_r<double>(d, shape.threads, stream)
                           : launch_one_r<float>(d, shape.threads, stream);
}

hipError_t launch_march_batch(const MarchDesc* d_descs, int n, int max_nodes, int geom, int warm,
                              int prec, MarchShape shape, int grid, unsigned int* d_next,
                              hipStream_t stream)
{
    return prec == WK_FP64
               ? launch_batch_r<double>(d_descs, n, max_nodes, geom, warm, shape.threads, grid, d_next, stream)
               : launch_batch_r<float>(d_descs, n, max_nodes, geom, warm, shape.threads, grid, d_next, stream);
}

}  // namespace wk
