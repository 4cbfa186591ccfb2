// Plasma response with B_theta from Eq. (6) as written,
//   (1/r) d_r (r B) = d_xi E_z + J_z      (slab: d_x B = d_xi E_z + J_z),
// instead of its Helmholtz form: the cross-check of the Helmholtz reading
// (Section II A, Eqs. (6)-(7)).  FP64, one workgroup per response.
//
// d_xi E_z at slice k is taken implicitly and one-sided, (E_z,k+1 - E_z,k) /
// dxi: E_z of slice k + 1 depends on B_k through the Heun step, so B_k is the
// fixed point B = Phi(B) of the trial step
//   1. f0 = f(Y_k; psi_k, psi'_k, B), Y* = Y_k + dxi f0;
//   2. E_z*, J_z* of Y* (B-independent deposits and solves); B* from Eq. (6)
//      with d_xi E_z = (E_z* - E_z,k) / dxi and J_z*;
//   3. f1 = f(Y*; psi*, psi'*, B*), Y_n = Y_k + dxi/2 (f0 + f1);
//   4. E_z of Y_n (the last slice: the backward difference (E_z,k -
//      E_z,k-1) / dxi instead), and Phi(B) from Eq. (6) with
//      d_xi E_z = (E_z(Y_n) - E_z,k) / dxi and J_z,k.
// Plain iteration of Phi diverges (a change of B bends the orbits by about
// B dxi, which moves E_z,k+1 by about B dxi r_max; the difference divides by
// dxi again: a gain of order r_max), so B_k is found by Newton steps on
// B - Phi(B) = 0.  Each step solves its linear system by restarted-free
// GMRES (Saad and Schultz 1986, Arnoldi with modified Gram-Schmidt and Givens
// rotations) with the Jacobian applied as a finite difference of Phi, step
// eps = 1e-7 (1 + |B|).  At most `iters` Newton steps per slice, until
// max |Phi(B) - B| <= tol max |Phi(B)|.  Slice 0 starts from B = 0; later
// slices from the previous slice's B.  The accepted step is Y_n of the last
// Phi(B_k), reflected at the wall.
//
// The deposits, the psi and E_z solves and the particle derivative are those
// of the Helmholtz march (dev::Marcher).  Every particle and node row is
// owned by one thread throughout (particle i by thread i mod T, node j by
// thread j mod T in the elementwise loops), so the trial states and Krylov
// vectors in global memory need no cross-thread ordering; node rows are in
// LDS behind barriers.
#include <algorithm>

#include "wk_direct.h"
#include "wk_marcher.h"

namespace wk {
namespace {

constexpr int kDirT = 256;

// LDS rows beyond the march rows.
enum DirectRow {
    DR_PSIK = NUM_ROWS,   // psi of Y_k
    DR_DPSIK,             // psi' of Y_k
    DR_EZK,               // E_z of Y_k
    DR_JZK,               // J_z of Y_k (with the beam current)
    DR_EZPREV,            // E_z of Y_k-1
    DR_B,                 // the Newton iterate B_k
    DR_PHI,               // Phi(B_k)
    DR_RES,               // Phi(B_k) - B_k
    DR_DX,                // Newton correction
    DR_OUT,               // Phi of a Krylov probe
    DR_TMP,               // Krylov probe B_k + eps v
    DR_DEZ,               // d_xi E_z
    DR_BSTAR,             // B* of the predicted state
    DR_W,                 // Arnoldi vector
    NUM_DIRECT_ROWS
};

// Small GMRES arrays after the rows: H [(m + 1) m], cs, sn [m], g [m + 1],
// y [m], and 4 scalars.
constexpr int kSmall = (kDirectKrylov + 1) * kDirectKrylov + 4 * kDirectKrylov + 1 + 4;

template <int GEOM, bool WARM>
struct Direct {
    using M = dev::Marcher<double, GEOM, WARM, kDirT, 1, false, false>;
    M& m;
    const DirectDesc& dd;
    int64_t np;
    int N, N1, st, tid, lane, wid;
    double dxi, h;
    double* small;

    __device__ __forceinline__ Direct(M& mm, const DirectDesc& d, double* sm_small)
        : m(mm), dd(d), small(sm_small)
    {
        np = m.d.np;
        N = m.N;
        N1 = m.N1;
        st = m.st;
        tid = threadIdx.x;
        lane = tid & 63;
        wid = tid >> 6;
        dxi = m.d.dxi;
        h = m.d.h;
    }

    __device__ __forceinline__ double* row(int r) const { return m.sm + r * st; }
    __device__ __forceinline__ void sync() const { dev::lds_barrier(); }

    // ---- particle states: Y_k in the plasma buffers, trial states [4][np] --
    __device__ __forceinline__ dev::Part<double> load_k(int64_t i) const { return m.load(i); }
    __device__ __forceinline__ dev::Part<double> load_arr(const double* a, int64_t i) const
    {
        dev::Part<double> p = m.load(i);   // D0 and w
        p.x = a[i];
        p.px = a[2 * np + i];
        if (GEOM == WK_CYL && WARM) {
            p.y = a[np + i];
            p.py = a[3 * np + i];
        }
        return p;
    }
    __device__ __forceinline__ void store_arr(double* a, int64_t i, const dev::Part<double>& p) const
    {
        a[i] = p.x;
        a[2 * np + i] = p.px;
        if (GEOM == WK_CYL && WARM) {
            a[np + i] = p.y;
            a[3 * np + i] = p.py;
        }
    }

    // ---- block reductions (fixed order: lanes, then waves) ------------------
    __device__ __forceinline__ double block_sum(double v) const
    {
        __shared__ double red[kDirT / 64];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[wid] = v;
        sync();
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kDirT / 64; ++w) s += red[w];
        sync();
        return s;
    }
    __device__ __forceinline__ double block_max(double v) const
    {
        __shared__ double red[kDirT / 64];
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
        if (lane == 0) red[wid] = v;
        sync();
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kDirT / 64; ++w) s = fmax(s, red[w]);
        sync();
        return s;
    }

    // ---- the B-independent evaluation of a state ----------------------------
    // psi (ROW_PSI2), psi' (ROW_DPSI2), J_z with the beam current (ROW_JZ) and
    // E_z (ROW_EZ) of the state `src` (nullptr: Y_k); returns this thread's
    // clamped D evaluations.
    __device__ __forceinline__ unsigned long long eval(const double* src, const double* jb_row)
    {
        for (int j = tid; j < N1; j += kDirT) {
            row(ROW_S)[j] = 0.0;
            for (int r = ROW_JR; r <= ROW_M5; ++r) row(r)[j] = 0.0;
        }
        sync();
        {
            dev::Acc<double, 1> a;
            a.reset(-1);
            for (int64_t i = tid; i < np; i += kDirT) m.dep_S(a, src ? load_arr(src, i) : load_k(i));
            a.flush(row(ROW_S), st);
        }
        sync();
        m.solve_psi(row(ROW_PSI2));
        sync();
        const unsigned long long c0 = m.clamps;
        {
            dev::Acc<double, 7> a;
            a.reset(-1);
            for (int64_t i = tid; i < np; i += kDirT) m.dep_moments(a, src ? load_arr(src, i) : load_k(i));
            m.flush_moments(a);
        }
        sync();
        m.finalize_moments(jb_row);
        sync();
        m.solve_ez(row(ROW_EZ));
        sync();
        return m.clamps - c0;
    }

    // Eq. (6) integrated from the axis by the trapezoid rule: r_j B_j =
    // r_j-1 B_j-1 + h/2 (r_j-1 q_j-1 + r_j q_j), q = dez + jz, B_0 = 0 (slab:
    // without the r weights).  A block-wide scan; barriers before and after.
    __device__ __forceinline__ void b_direct(const double* dez, const double* jz, double* out)
    {
        const auto term = [&](int j) {
            const double a = GEOM == WK_CYL ? (double)(j - 1) * h : 1.0;
            const double b = GEOM == WK_CYL ? (double)j * h : 1.0;
            return 0.5 * h * (a * (dez[j - 1] + jz[j - 1]) + b * (dez[j] + jz[j]));
        };
        int i0, i1;
        m.owned(N, i0, i1);   // items i = j - 1, j = 1..N
        double s = 0.0;
        for (int i = i0; i < i1; ++i) s += term(i + 1);
        double tot;
        double run = m.block_excl(s, dev::scan_scratch(), tot);
        for (int i = i0; i < i1; ++i) {
            const int j = i + 1;
            run += term(j);
            out[j] = GEOM == WK_CYL ? run / ((double)j * h) : run;
        }
        if (tid == 0) out[0] = 0.0;
        sync();
    }

    // Phi(b) -> out; the trial states are left in dd.ys (Y*) and dd.yn (Y_n).
    // Returns this thread's clamped evaluations of the step (2 at Y*, as
    // the predicted state is evaluated for its E_z and for its derivative,
    // and 1 at Y_n).
    __device__ __forceinline__ unsigned long long phi(const double* b, double* out, bool last, const double* jb_n)
    {
        const double hd = 0.5 * dxi;
        for (int64_t i = tid; i < np; i += kDirT) {
            const dev::Part<double> p = load_k(i);
            const dev::Deriv<double> g = m.derivative(p, row(DR_PSIK), row(DR_DPSIK), b);
            dd.f0[i] = g.fx;
            dd.f0[np + i] = g.fy;
            dd.f0[2 * np + i] = g.fpx;
            dd.f0[3 * np + i] = g.fpy;
            store_arr(dd.ys, i, M::advance(p, g, dxi));
        }
        const unsigned long long cs = eval(dd.ys, jb_n);
        for (int j = tid; j < N1; j += kDirT) row(DR_DEZ)[j] = (row(ROW_EZ)[j] - row(DR_EZK)[j]) / dxi;
        sync();
        b_direct(row(DR_DEZ), row(ROW_JZ), row(DR_BSTAR));
        for (int64_t i = tid; i < np; i += kDirT) {
            const dev::Part<double> p = load_k(i);
            const dev::Part<double> q = load_arr(dd.ys, i);
            const dev::Deriv<double> g1 = m.derivative(q, row(ROW_PSI2), row(ROW_DPSI2), row(DR_BSTAR));
            dev::Part<double> n = p;
            n.x = p.x + hd * (dd.f0[i] + g1.fx);
            n.px = p.px + hd * (dd.f0[2 * np + i] + g1.fpx);
            if (GEOM == WK_CYL && WARM) {
                n.y = p.y + hd * (dd.f0[np + i] + g1.fy);
                n.py = p.py + hd * (dd.f0[3 * np + i] + g1.fpy);
            }
            store_arr(dd.yn, i, n);
        }
        unsigned long long cn = 0;
        if (last) {
            for (int j = tid; j < N1; j += kDirT) row(DR_DEZ)[j] = (row(DR_EZK)[j] - row(DR_EZPREV)[j]) / dxi;
        } else {
            cn = eval(dd.yn, jb_n);
            for (int j = tid; j < N1; j += kDirT) row(DR_DEZ)[j] = (row(ROW_EZ)[j] - row(DR_EZK)[j]) / dxi;
        }
        sync();
        b_direct(row(DR_DEZ), row(DR_JZK), out);
        return 2 * cs + cn;
    }

    __device__ __forceinline__ double* V(int k) const { return dd.V + (int64_t)k * st; }

    // Solve (I - J) dx = r by GMRES with J v = (Phi(b + eps v) - Phi(b)) /
    // eps: b in DR_B, Phi(b) in DR_PHI, r in DR_RES, dx to DR_DX.
    __device__ __forceinline__ void gmres(bool last, const double* jb_n)
    {
        constexpr int m_ = kDirectKrylov;
        double* H = small;                    // H[q * m + k]
        double* cs = H + (m_ + 1) * m_;
        double* sn = cs + m_;
        double* gv = sn + m_;
        double* yv = gv + m_ + 1;
        double* sc = yv + m_;                 // sc[0]: stop flag
        const double* b = row(DR_B);
        const double* phib = row(DR_PHI);
        const double* r = row(DR_RES);
        double* dx = row(DR_DX);
        double* w = row(DR_W);
        double* tmp = row(DR_TMP);
        double* outp = row(DR_OUT);
        double s2 = 0.0, b2 = 0.0;
        for (int j = tid; j < N1; j += kDirT) {
            dx[j] = 0.0;
            s2 += r[j] * r[j];
            b2 += b[j] * b[j];
        }
        const double beta = sqrt(block_sum(s2));
        const double bn = sqrt(block_sum(b2));
        if (beta == 0.0) return;
        for (int j = tid; j < N1; j += kDirT) V(0)[j] = r[j] / beta;
        if (tid == 0) {
            for (int i = 0; i <= m_; ++i) gv[i] = 0.0;
            gv[0] = beta;
        }
        sync();
        const double eps = 1e-7 * (1.0 + bn);
        int used = 0;
        for (int k = 0; k < m_; ++k) {
            const double* vk = V(k);
            for (int j = tid; j < N1; j += kDirT) tmp[j] = b[j] + eps * vk[j];
            sync();
            phi(tmp, outp, last, jb_n);
            for (int j = tid; j < N1; j += kDirT) w[j] = vk[j] - (outp[j] - phib[j]) / eps;
            // modified Gram-Schmidt against v_0 .. v_k
            for (int q = 0; q <= k; ++q) {
                const double* vq = V(q);
                double s = 0.0;
                for (int j = tid; j < N1; j += kDirT) s += w[j] * vq[j];
                const double hq = block_sum(s);
                if (tid == 0) H[q * m_ + k] = hq;
                for (int j = tid; j < N1; j += kDirT) w[j] -= hq * vq[j];
            }
            double s = 0.0;
            for (int j = tid; j < N1; j += kDirT) s += w[j] * w[j];
            const double hn = sqrt(block_sum(s));
            double* vn = V(k + 1);
            for (int j = tid; j < N1; j += kDirT) vn[j] = hn > 0.0 ? w[j] / hn : w[j];
            if (tid == 0) {
                H[(k + 1) * m_ + k] = hn;
                for (int q = 0; q < k; ++q) {
                    const double a0 = H[q * m_ + k], a1 = H[(q + 1) * m_ + k];
                    H[q * m_ + k] = cs[q] * a0 + sn[q] * a1;
                    H[(q + 1) * m_ + k] = -sn[q] * a0 + cs[q] * a1;
                }
                const double a0 = H[k * m_ + k], a1 = H[(k + 1) * m_ + k];
                const double den = sqrt(a0 * a0 + a1 * a1);
                cs[k] = den > 0.0 ? a0 / den : 1.0;
                sn[k] = den > 0.0 ? a1 / den : 0.0;
                H[k * m_ + k] = den;
                H[(k + 1) * m_ + k] = 0.0;
                gv[k + 1] = -sn[k] * gv[k];
                gv[k] = cs[k] * gv[k];
                sc[0] = (fabs(gv[k + 1]) <= 1e-13 * beta || hn == 0.0) ? 1.0 : 0.0;
            }
            sync();
            used = k + 1;
            if (sc[0] != 0.0) break;
        }
        if (tid == 0) {
            for (int k = used - 1; k >= 0; --k) {
                double t = gv[k];
                for (int q = k + 1; q < used; ++q) t -= H[k * m_ + q] * yv[q];
                yv[k] = t / H[k * m_ + k];
            }
        }
        sync();
        for (int k = 0; k < used; ++k) {
            const double yk = yv[k];
            const double* vk = V(k);
            for (int j = tid; j < N1; j += kDirT) dx[j] += yk * vk[j];
        }
        sync();
    }

    __device__ __forceinline__ void run()
    {
        const int n_xi = m.d.n_xi;
        for (int j = tid; j < N1; j += kDirT) {
            row(ROW_NION)[j] = m.d.nion[j];
            row(DR_B)[j] = 0.0;
            row(DR_EZPREV)[j] = 0.0;
        }
        sync();
        unsigned long long acc = 0;
        for (int k = 0; k < n_xi; ++k) {
            const double* jb_k = m.d.jb + (int64_t)k * N1;
            const double* jb_n = m.d.jb + (int64_t)(k + 1 < n_xi ? k + 1 : k) * N1;
            const bool last = k + 1 >= n_xi;
            const unsigned long long ck = eval(nullptr, jb_k);
            for (int j = tid; j < N1; j += kDirT) {
                row(DR_PSIK)[j] = row(ROW_PSI2)[j];
                row(DR_DPSIK)[j] = row(ROW_DPSI2)[j];
                row(DR_EZK)[j] = row(ROW_EZ)[j];
                row(DR_JZK)[j] = row(ROW_JZ)[j];
            }
            sync();
            int it = 0;
            unsigned long long cphi = 0;
            for (;;) {
                cphi = phi(row(DR_B), row(DR_PHI), last, jb_n);
                double rmax = 0.0, bmax = 0.0;
                for (int j = tid; j < N1; j += kDirT) {
                    const double res = row(DR_PHI)[j] - row(DR_B)[j];
                    row(DR_RES)[j] = res;
                    rmax = fmax(rmax, fabs(res));
                    bmax = fmax(bmax, fabs(row(DR_PHI)[j]));
                }
                rmax = block_max(rmax);
                bmax = block_max(bmax);
                if (rmax <= dd.tol * bmax || it >= dd.iters) break;
                ++it;
                gmres(last, jb_n);
                for (int j = tid; j < N1; j += kDirT) row(DR_B)[j] += row(DR_DX)[j];
                sync();
            }
            if (tid == 0 && dd.iterations) dd.iterations[k] = it;
            m.store_fields(k, row(DR_PSIK), row(DR_EZK), row(DR_B), row(DR_DPSIK));
            if (last) break;
            // accept Y_n of Phi(B_k), reflected at the wall
            acc += ck + cphi;
            for (int64_t i = tid; i < np; i += kDirT) {
                dev::Part<double> p = load_arr(dd.yn, i);
                m.reflect(p);
                m.store_state(i, p);
            }
            for (int j = tid; j < N1; j += kDirT) row(DR_EZPREV)[j] = row(DR_EZK)[j];
            sync();
        }
        if (acc) atomicAdd(m.d.counters + WK_CNT_D_CLAMP, acc);
        if (m.walls) atomicAdd(m.d.counters + WK_CNT_WALL, m.walls);
    }
};

template <int GEOM, bool WARM>
__global__ __launch_bounds__(kDirT) void k_march_direct(DirectDesc dd)
{
    extern __shared__ double smem[];
    using D = Direct<GEOM, WARM>;
    typename D::M m(dd.march, smem);
    D run(m, dd, smem + (size_t)NUM_DIRECT_ROWS * lds_stride(dd.march.n_r + 1));
    run.run();
}

template <int GEOM, bool WARM>
hipError_t launch_t(const DirectDesc& dd, hipStream_t s)
{
    const size_t lds = direct_lds_bytes(dd.march.n_r + 1);
    auto kern = k_march_direct<GEOM, WARM>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(1), dim3(kDirT), lds, s, dd);
    return hipGetLastError();
}

}  // namespace

size_t direct_lds_bytes(int n_nodes)
{
    return ((size_t)NUM_DIRECT_ROWS * lds_stride(n_nodes) + kSmall) * sizeof(double);
}

size_t direct_ws_doubles(int64_t np, int n_nodes)
{
    return (size_t)12 * (size_t)std::max<int64_t>(np, 1) + (size_t)(kDirectKrylov + 1) * lds_stride(n_nodes);
}

hipError_t launch_march_direct(const DirectDesc& dd, hipStream_t s)
{
    if (!lds_fits(direct_lds_bytes(dd.march.n_r + 1))) return hipErrorInvalidValue;
    if (dd.march.geom == WK_CYL)
        return dd.march.warm ? launch_t<WK_CYL, true>(dd, s) : launch_t<WK_CYL, false>(dd, s);
    return dd.march.warm ? launch_t<WK_SLAB, true>(dd, s) : launch_t<WK_SLAB, false>(dd, s);
}

}  // namespace wk
