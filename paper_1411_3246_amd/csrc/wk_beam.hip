// Loaders, beam current, beam push and diagnostics.
#include <algorithm>

#include "wk_beam_dev.h"

namespace wk {
namespace {

constexpr int kBlock = 256;

__device__ inline double node_vol(const GridDesc& g, int j)
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

__device__ inline void hat(const GridDesc& g, double rho, int& j, double& t)
{
    const double u = rho / g.h;
    int jj = (int)floor(u);
    jj = jj < 0 ? 0 : (jj > g.n_r - 1 ? g.n_r - 1 : jj);
    j = jj;
    t = u - (double)jj;
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_zero_u32(unsigned int* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Plasma loader (cell-uniform rings; mirrored thermal pairs).  One
// workgroup; n_ion is deposited in LDS and divided by the node volumes.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(1024) void k_init_plasma(GridDesc g, int ppc, double u_th, double n0,
                                                      wk_plasma_bufs b, const double* draws)
{
    extern __shared__ double acc[];
    const int N = g.n_r, N1 = N + 1;
    const bool warm = u_th > 0.0;
    const int npos = warm ? ppc / 2 : ppc;
    for (int j = threadIdx.x; j < N1; j += blockDim.x) acc[j] = 0.0;
    __syncthreads();
    const int64_t nsite = (int64_t)N * npos;
    R* d0 = (R*)b.d_d0;
    R* w = (R*)b.d_w;
    for (int64_t q = threadIdx.x; q < nsite; q += blockDim.x) {
        const int c = (int)(q / npos), m = (int)(q % npos);
        const double rlo = (c + (double)m / npos) * g.h;
        const double rhi = (c + (double)(m + 1) / npos) * g.h;
        const double r0 = (c + (m + 0.5) / npos) * g.h;
        const double area = g.geom == WK_CYL ? n0 * kPi * (rhi * rhi - rlo * rlo) : n0 * (rhi - rlo);
        int j;
        double t;
        hat(g, r0, j, t);
        atomicAdd(acc + j, area * (1.0 - t));
        atomicAdd(acc + j + 1, area * t);
        if (!warm) {
            b.d_x[q] = r0;
            b.d_px[q] = 0.0;
            if (b.d_y) b.d_y[q] = 0.0;
            if (b.d_py) b.d_py[q] = 0.0;
            d0[q] = (R)1.0;
            w[q] = (R)area;
            continue;
        }
        const double pr0 = u_th * draws[3 * q + 0];
        const double pt0 = u_th * draws[3 * q + 1];
        const double pz0 = u_th * draws[3 * q + 2];
        const double g0 = sqrt(1.0 + pr0 * pr0 + pt0 * pt0 + pz0 * pz0);
        const double half = 0.5 * area;
        for (int s = 0; s < 2; ++s) {
            const double sg = s == 0 ? 1.0 : -1.0;
            const double dd = g0 - sg * pz0;
            const int64_t i = 2 * q + s;
            b.d_x[i] = r0;
            if (b.d_y) b.d_y[i] = 0.0;
            b.d_px[i] = sg * pr0;
            b.d_py[i] = sg * pt0;
            d0[i] = (R)dd;
            w[i] = (R)(half * dd / g0);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N1; j += blockDim.x) b.d_nion[j] = acc[j] / node_vol(g, j);
}

// ---------------------------------------------------------------------------
// Beam loader (Eq. (12) sampled with the given standard normals)
// ---------------------------------------------------------------------------
struct BeamLoad {
    double sigma_r, gamma0, rel;
    double xi_c[2], sigma_z[2], weight[2];
    int64_t n_drive;
    int geom;
};

__global__ void k_init_beam(BeamLoad L, int64_t n, wk_beam_bufs b, const double* draws)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = i < L.n_drive ? 0 : 1;
    const double* e = draws + 4 * i;
    b.d_x[i] = L.sigma_r * e[0];
    b.d_y[i] = L.geom == WK_CYL ? L.sigma_r * e[1] : 0.0;
    b.d_xi[i] = L.xi_c[t] + L.sigma_z[t] * e[2];
    const double gam = L.gamma0 * (1.0 + L.rel * e[3]);
    b.d_px[i] = 0.0;
    b.d_py[i] = 0.0;
    const double pz = sqrt(gam * gam - 1.0);
    b.d_pz[i] = pz;
    b.d_w[i] = L.weight[t];
    b.d_tag[i] = t;
    b.d_gamma_init[i] = sqrt(1.0 + pz * pz);
}

// ---------------------------------------------------------------------------
// Analytic beam current, J_bz = -n_b of Eq. (12)
// ---------------------------------------------------------------------------
struct BeamShape {
    double sigma_r;
    int n_bunch;
    double n_peak[2], sigma_z[2], xi_c[2];
};

__global__ void k_beam_current_analytic(GridDesc g, BeamShape s, double* jb)
{
    const int64_t N1 = g.n_r + 1;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)g.n_xi * N1) return;
    const int k = (int)(q / N1), j = (int)(q % N1);
    const double xi = g.xi_min + k * g.dxi;
    double sum = 0.0;
    for (int b = 0; b < s.n_bunch; ++b) {
        const double u = (xi - s.xi_c[b]) / s.sigma_z[b];
        sum += s.n_peak[b] * exp(-0.5 * u * u);
    }
    const double v = (j * g.h) / s.sigma_r;
    jb[q] = -(exp(-0.5 * v * v) * sum);
}

// ---------------------------------------------------------------------------
// Macroparticle beam current.  The beam is binned by xi cell (counting
// sort into an index array in the workspace); one workgroup per slice then
// gathers the particles of the two adjacent cells into an LDS row.  Every row
// of J_bz is written by exactly one workgroup (no global float atomics).
// ---------------------------------------------------------------------------
__device__ inline int beam_cell(const GridDesc& g, double x, double y, double xi)
{
    const double r = g.geom == WK_CYL ? sqrt(x * x + y * y) : fabs(x);
    const double xi_max = g.xi_min + g.n_xi * g.dxi;
    if (r > g.r_max || xi < g.xi_min || xi >= xi_max) return -1;
    int k = (int)floor((xi - g.xi_min) / g.dxi);
    return k > g.n_xi - 1 ? g.n_xi - 1 : k;
}

__global__ void k_beam_count(GridDesc g, int64_t n, wk_beam_bufs b, unsigned int* count,
                             unsigned long long* counters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = beam_cell(g, b.d_x[i], b.d_y[i], b.d_xi[i]);
    if (c < 0) {
        atomicAdd(counters + WK_CNT_BEAM_OUT_DEPOSIT, 1ull);
        return;
    }
    atomicAdd(count + c, 1u);
}

// Exclusive scan of n counts in one workgroup (start[0..n], start[n] = total);
// fill[] receives a copy of the starts.
__global__ __launch_bounds__(1024) void k_scan_counts(const unsigned int* count, int n,
                                                      unsigned int* start, unsigned int* fill)
{
    __shared__ unsigned int wsum[16];
    __shared__ unsigned int carry;
    const int T = blockDim.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += T) {
        const int i = base + tid;
        const unsigned int v = i < n ? count[i] : 0u;
        unsigned int incl = v;
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned int o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        if (wid == 0) {
            unsigned int s = lane < (T >> 6) ? wsum[lane] : 0u;
            for (int off = 1; off < 64; off <<= 1) {
                const unsigned int o = __shfl_up(s, off, 64);
                if (lane >= off) s += o;
            }
            if (lane < (T >> 6)) wsum[lane] = s;
        }
        __syncthreads();
        const unsigned int excl = carry + incl - v + (wid > 0 ? wsum[wid - 1] : 0u);
        if (i < n) {
            start[i] = excl;
            fill[i] = excl;
        }
        __syncthreads();
        if (tid == T - 1) carry = excl + v;
        __syncthreads();
    }
    if (tid == 0) start[n] = carry;
}

// Subset of particle i when n particles are split into G contiguous ranges
// [n s / G, n (s + 1) / G).
__device__ inline int subset_of(int64_t i, int64_t n, int G)
{
    int s = (int)((i * G) / n);
    while (s + 1 < G && n * (s + 1) / G <= i) ++s;
    while (s > 0 && n * s / G > i) --s;
    return s;
}

__global__ void k_bin_count_split(GridDesc g, int64_t n, int G, const double* xi, unsigned int* count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = subset_of(i, n, G);
    atomicAdd(count + (int64_t)s * (g.n_xi + 1) + dev::beam_xi_bin(g, xi[i]), 1u);
}

__global__ void k_bin_scatter_split(GridDesc g, int64_t n, int G, const double* xi, unsigned int* fill,
                                    unsigned int* order)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = subset_of(i, n, G);
    const unsigned int pos = atomicAdd(fill + (int64_t)s * (g.n_xi + 1) + dev::beam_xi_bin(g, xi[i]), 1u);
    order[pos] = (unsigned int)(i - n * s / G);
}

// Per-subset bin starts relative to the subset's first particle:
// out[s][b] for b = 0..n_xi+1 from the global starts of the (subset, bin) keys.
__global__ void k_split_starts(int nb, int64_t n, int G, const unsigned int* start_all, unsigned int* out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)G * (nb + 1)) return;
    const int s = (int)(q / (nb + 1)), b = (int)(q % (nb + 1));
    const int64_t b0 = n * s / G;
    out[q] = b < nb ? (unsigned int)(start_all[(int64_t)s * nb + b] - b0) : (unsigned int)(n * (s + 1) / G - b0);
}

__global__ void k_beam_scatter(GridDesc g, int64_t n, wk_beam_bufs b, unsigned int* fill,
                               unsigned int* order)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = beam_cell(g, b.d_x[i], b.d_y[i], b.d_xi[i]);
    if (c < 0) return;
    const unsigned int pos = atomicAdd(fill + c, 1u);
    order[pos] = (unsigned int)i;
}

// The particle indices of each xi cell in ascending order (one workgroup per
// cell): the scatter's atomic counter hands out the slots of a cell in an
// order that depends on scheduling, and the sort makes the order, and so the
// summation order of the rows, a function of the beam alone.  Runs of up to
// kSortCap indices are sorted in LDS (bitonic network); longer cells then
// merge their runs pairwise through `tmp` (each output element placed by a
// binary search along the merge path).
constexpr int kSortT = 1024;
constexpr int kSortCap = 8192;

__device__ __forceinline__ void bitonic_lds(unsigned* v, int n2)
{
    for (int k = 2; k <= n2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n2; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const unsigned x = v[i], y = v[l];
                    if ((x > y) == up) {
                        v[i] = y;
                        v[l] = x;
                    }
                }
            }
            __syncthreads();
        }
}

__global__ __launch_bounds__(kSortT) void k_bin_sort(const unsigned int* start, unsigned int* order,
                                                     unsigned int* tmp)
{
    __shared__ unsigned v[kSortCap];
    const int c = blockIdx.x, tid = threadIdx.x;
    const unsigned beg = start[c], n = start[c + 1] - beg;
    if (n <= 1) return;
    unsigned* src = order + beg;
    unsigned* dst = tmp + beg;
    for (unsigned r0 = 0; r0 < n; r0 += kSortCap) {
        const unsigned m = min(n - r0, (unsigned)kSortCap);
        int m2 = 1;
        while ((unsigned)m2 < m) m2 <<= 1;
        for (int i = tid; i < m2; i += kSortT) v[i] = (unsigned)i < m ? src[r0 + i] : 0xffffffffu;
        __syncthreads();
        bitonic_lds(v, m2);
        for (unsigned i = tid; i < m; i += kSortT) src[r0 + i] = v[i];
        __syncthreads();
    }
    for (unsigned w = kSortCap; w < n; w <<= 1) {
        for (unsigned t = tid; t < n; t += kSortT) {
            const unsigned s0 = (t / (2 * w)) * (2 * w);
            const unsigned a1 = min(s0 + w, n), b1 = min(s0 + 2 * w, n);
            const unsigned na = a1 - s0, nb = b1 - a1, o = t - s0;
            const unsigned* A = src + s0;
            const unsigned* B = src + a1;
            // elements of A among the first o outputs (indices are distinct)
            unsigned lo = o > nb ? o - nb : 0, hi = min(o, na);
            while (lo < hi) {
                const unsigned mid = (lo + hi) >> 1;
                if (A[mid] < B[o - 1 - mid]) lo = mid + 1;
                else hi = mid;
            }
            const unsigned ia = lo, ib = o - lo;
            dst[t] = (ia < na && (ib >= nb || A[ia] < B[ib])) ? A[ia] : B[ib];
        }
        __syncthreads();
        unsigned* t2 = src;
        src = dst;
        dst = t2;
    }
    if (src != order + beg) {
        for (unsigned t = tid; t < n; t += kSortT) order[beg + t] = src[t];
    }
}

// Row k of J_bz from the particles of cells k-1 (weight tk towards slice k)
// and k (weight 1 - tk), in their sorted order.  Each node's sum is formed by
// one thread, adding the particles' contributions in list order, so that the
// row does not depend on scheduling: chunks of kRowChunk particles are
// staged in LDS (hat cell and the two node contributions) and every thread
// walks the chunk for the nodes it owns.
constexpr int kRowChunk = 1024;

__global__ __launch_bounds__(kBlock) void k_beam_rows(GridDesc g, wk_beam_bufs b,
                                                      const unsigned int* start,
                                                      const unsigned int* order, double* jb)
{
    extern __shared__ double acc[];
    const int k = blockIdx.x;
    const int N1 = g.n_r + 1;
    double* clo = acc + ((N1 + 1) & ~1);
    double* chi = clo + kRowChunk;
    int* cj = (int*)(chi + kRowChunk);
    for (int j = threadIdx.x; j < N1; j += blockDim.x) acc[j] = 0.0;
    const int c0 = k > 0 ? k - 1 : 0;
    const unsigned beg = start[c0], end = start[k + 1];
    for (unsigned base = beg; base < end; base += kRowChunk) {
        const unsigned m = min(end - base, (unsigned)kRowChunk);
        __syncthreads();
        for (unsigned p = threadIdx.x; p < m; p += blockDim.x) {
            const unsigned i = order[base + p];
            const double x = b.d_x[i], y = b.d_y[i];
            const double r = g.geom == WK_CYL ? sqrt(x * x + y * y) : fabs(x);
            int j;
            double tr;
            hat(g, r, j, tr);
            const double u = (b.d_xi[i] - g.xi_min) / g.dxi;
            int kk = (int)floor(u);
            if (kk > g.n_xi - 1) kk = g.n_xi - 1;
            const double tk = u - kk;
            double wk;
            if (kk == k) wk = 1.0 - tk;
            else if (kk == k - 1) wk = tk;
            else {
                cj[p] = -2;
                continue;
            }
            const double wb = b.d_w[i];
            cj[p] = j;
            clo[p] = wb * (1.0 - tr) * wk;
            chi[p] = wb * tr * wk;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < N1; j += blockDim.x) {
            double sum = acc[j];
            for (unsigned p = 0; p < m; ++p) {
                const int q = cj[p];
                if (q == j) sum += clo[p];
                else if (q + 1 == j) sum += chi[p];
            }
            acc[j] = sum;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N1; j += blockDim.x)
        jb[(int64_t)k * N1 + j] = -acc[j] / (node_vol(g, j) * g.dxi);
}

// ---------------------------------------------------------------------------
// Beam push, Eqs. (8)-(11) with the Boris rotation (q = -1)
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBlock) void k_beam_push(GridDesc g, int64_t n, wk_beam_bufs b,
                                                      const R* __restrict__ fields, int n_steps,
                                                      double dt, unsigned long long* counters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = b.d_x[i], y = b.d_y[i], xi = b.d_xi[i];
    double px = b.d_px[i], py = b.d_py[i], pz = b.d_pz[i];
    const unsigned long long out = dev::beam_push_particle<R>(g, fields, x, y, xi, px, py, pz, n_steps, dt);
    b.d_x[i] = x;
    b.d_y[i] = y;
    b.d_xi[i] = xi;
    b.d_px[i] = px;
    b.d_py[i] = py;
    b.d_pz[i] = pz;
    if (out) atomicAdd(counters + WK_CNT_BEAM_OUT_PUSH, out);
}

// ---------------------------------------------------------------------------
// Diagnostics (deterministic two-level reductions)
// ---------------------------------------------------------------------------
constexpr int kGainBlocks = 512;

__global__ __launch_bounds__(kBlock) void k_gain_partial(int64_t n, wk_beam_bufs b, int which,
                                                         double* part)
{
    __shared__ double sn[kBlock], sd[kBlock];
    double num = 0.0, den = 0.0;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * per;
    const int64_t end = beg + per < n ? beg + per : n;
    for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        if (b.d_tag[i] != which) continue;
        const double px = b.d_px[i], py = b.d_py[i], pz = b.d_pz[i];
        const double gam = sqrt(1.0 + px * px + py * py + pz * pz);
        num += b.d_w[i] * (gam - b.d_gamma_init[i]);
        den += b.d_w[i];
    }
    sn[threadIdx.x] = num;
    sd[threadIdx.x] = den;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sn[threadIdx.x] += sn[threadIdx.x + s];
            sd[threadIdx.x] += sd[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sn[0];
        part[2 * blockIdx.x + 1] = sd[0];
    }
}

__global__ void k_gain_final(const double* part, int nb, double* out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double num = 0.0, den = 0.0;
    for (int i = 0; i < nb; ++i) {
        num += part[2 * i];
        den += part[2 * i + 1];
    }
    out[0] = den > 0.0 ? num / den : 0.0;
}

// Energy spectrum: counts of gamma - gamma_init in n_bins equal bins of
// [lo, hi), with an underflow (index 0) and an overflow (n_bins + 1) bin.
// The bin of a particle is decided in double with every operation rounded on
// its own (no contracted multiply-adds), as a plain C evaluation decides it;
// integer counts make the result independent of the order of the adds.
constexpr int kHistMax = 4096;

__global__ __launch_bounds__(kBlock) void k_gain_hist(int64_t n, wk_beam_bufs b, int which, int n_bins,
                                                      double lo, double hi, unsigned long long* hist)
{
#pragma clang fp contract(off)
    __shared__ unsigned int h[kHistMax + 2];
    for (int q = threadIdx.x; q < n_bins + 2; q += blockDim.x) h[q] = 0u;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (which >= 0 && b.d_tag[i] != which) continue;
        const double px = b.d_px[i], py = b.d_py[i], pz = b.d_pz[i];
        const double px2 = px * px, py2 = py * py, pz2 = pz * pz;
        const double gain = sqrt(((1.0 + px2) + py2) + pz2) - b.d_gamma_init[i];
        int q;
        if (!(gain >= lo)) {
            q = 0;
        } else if (gain >= hi) {
            q = n_bins + 1;
        } else {
            const double u = (gain - lo) / (hi - lo);
            int k = (int)floor(u * (double)n_bins);
            k = k < 0 ? 0 : (k > n_bins - 1 ? n_bins - 1 : k);
            q = 1 + k;
        }
        atomicAdd(h + q, 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n_bins + 2; q += blockDim.x)
        if (h[q]) atomicAdd(hist + q, (unsigned long long)h[q]);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_ez_peak(GridDesc g, const R* fields, double xi_from,
                                                    double* out)
{
    __shared__ double sm[kBlock];
    __shared__ int sv[kBlock];
    const int N1 = g.n_r + 1;
    const int64_t plane = (int64_t)g.n_xi * N1;
    double m = 0.0;
    int valid = 0;
    for (int k = threadIdx.x; k < g.n_xi; k += blockDim.x) {
        const double xi = g.xi_min + k * g.dxi;
        if (xi < xi_from) continue;
        const double v = (double)fields[plane + (int64_t)k * N1];
        if (!valid || v < m) m = v;
        valid = 1;
    }
    sm[threadIdx.x] = m;
    sv[threadIdx.x] = valid;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s && sv[threadIdx.x + s]) {
            if (!sv[threadIdx.x] || sm[threadIdx.x + s] < sm[threadIdx.x]) sm[threadIdx.x] = sm[threadIdx.x + s];
            sv[threadIdx.x] = 1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

inline unsigned int nblocks(int64_t n, int b) { return (unsigned int)((n + b - 1) / b); }

}  // namespace

size_t beam_ws_bytes(int n_xi, int64_t n_beam)
{
    const size_t order = align256(sizeof(unsigned int) * (size_t)(n_beam > 0 ? n_beam : 1));
    return align256(sizeof(unsigned int) * (size_t)n_xi) + align256(sizeof(unsigned int) * (size_t)(n_xi + 1)) +
           align256(sizeof(unsigned int) * (size_t)n_xi) + 2 * order + align256(sizeof(double) * 2 * kGainBlocks);
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_init_plasma(const GridDesc& g, int ppc, double u_th, double n0, int prec,
                              const wk_plasma_bufs& b, const double* draws, hipStream_t s)
{
    const size_t lds = sizeof(double) * (g.n_r + 1);
    if (prec == WK_FP64)
        hipLaunchKernelGGL(k_init_plasma<double>, dim3(1), dim3(1024), lds, s, g, ppc, u_th, n0, b, draws);
    else
        hipLaunchKernelGGL(k_init_plasma<float>, dim3(1), dim3(1024), lds, s, g, ppc, u_th, n0, b, draws);
    return hipGetLastError();
}

hipError_t launch_init_beam(const GridDesc& g, const wk_problem& p, const wk_beam_bufs& b,
                            const double* draws, hipStream_t s)
{
    BeamLoad L;
    L.sigma_r = p.sigma_r;
    L.gamma0 = p.gamma0;
    L.rel = p.rel_spread;
    L.n_drive = p.n_drive;
    L.geom = p.geom;
    for (int t = 0; t < 2; ++t) {
        const wk_bunch& bb = p.bunch[t < p.n_bunch ? t : 0];
        L.xi_c[t] = bb.xi_c;
        L.sigma_z[t] = bb.sigma_z;
        const double sz = sqrt(2.0 * kPi) * bb.sigma_z;
        const double sperp = p.geom == WK_CYL ? 2.0 * kPi * p.sigma_r * p.sigma_r
                                              : sqrt(0.5 * kPi) * p.sigma_r;
        const int64_t nb = t == 0 ? p.n_drive : p.n_beam - p.n_drive;
        L.weight[t] = (t < p.n_bunch && nb > 0) ? bb.n_peak * sz * sperp / (double)nb : 0.0;
    }
    hipLaunchKernelGGL(k_init_beam, dim3(nblocks(p.n_beam, kBlock)), dim3(kBlock), 0, s, L, p.n_beam, b, draws);
    return hipGetLastError();
}

hipError_t launch_beam_current_analytic(const GridDesc& g, const wk_problem& p, double* jb, hipStream_t s)
{
    BeamShape sh;
    sh.sigma_r = p.sigma_r;
    sh.n_bunch = p.n_bunch;
    for (int t = 0; t < 2; ++t) {
        sh.n_peak[t] = p.bunch[t].n_peak;
        sh.sigma_z[t] = p.bunch[t].sigma_z;
        sh.xi_c[t] = p.bunch[t].xi_c;
    }
    const int64_t n = (int64_t)g.n_xi * (g.n_r + 1);
    hipLaunchKernelGGL(k_beam_current_analytic, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s, g, sh, jb);
    return hipGetLastError();
}

hipError_t launch_beam_current(const GridDesc& g, int64_t n_beam, const wk_beam_bufs& b, double* jb,
                               void* ws, unsigned long long* counters, hipStream_t s)
{
    char* p = (char*)ws;
    unsigned int* count = (unsigned int*)p;
    p += align256(sizeof(unsigned int) * (size_t)g.n_xi);
    unsigned int* start = (unsigned int*)p;
    p += align256(sizeof(unsigned int) * (size_t)(g.n_xi + 1));
    unsigned int* fill = (unsigned int*)p;
    p += align256(sizeof(unsigned int) * (size_t)g.n_xi);
    unsigned int* order = (unsigned int*)p;
    p += align256(sizeof(unsigned int) * (size_t)(n_beam > 0 ? n_beam : 1));
    unsigned int* sort_tmp = (unsigned int*)p;
    hipError_t e = launch_zero_u32(count, g.n_xi, s);
    if (e != hipSuccess) return e;
    if (n_beam > 0) {
        hipLaunchKernelGGL(k_beam_count, dim3(nblocks(n_beam, kBlock)), dim3(kBlock), 0, s, g, n_beam, b,
                           count, counters);
    }
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, count, g.n_xi, start, fill);
    if (n_beam > 0) {
        hipLaunchKernelGGL(k_beam_scatter, dim3(nblocks(n_beam, kBlock)), dim3(kBlock), 0, s, g, n_beam, b,
                           fill, order);
    }
    if (n_beam > 0)
        hipLaunchKernelGGL(k_bin_sort, dim3(g.n_xi), dim3(kSortT), 0, s, start, order, sort_tmp);
    const size_t lds = sizeof(double) * (((g.n_r + 2) & ~1) + 2 * kRowChunk) + sizeof(int) * kRowChunk;
    hipLaunchKernelGGL(k_beam_rows, dim3(g.n_xi), dim3(kBlock), lds, s, g, b, start, order, jb);
    return hipGetLastError();
}

hipError_t launch_beam_bins_split(const GridDesc& g, int64_t n_beam, int group, const wk_beam_bufs& b,
                                  unsigned int* count, unsigned int* bin_start, unsigned int* fill,
                                  unsigned int* order, hipStream_t s)
{
    const int nb = g.n_xi + 1;
    const int64_t keys = (int64_t)group * nb;
    // the global starts of the keys go to the second slot of bin_start
    // (G (nb + 1) >= keys + 1 entries), which the cycle writes later
    unsigned int* start_all = bin_start + (int64_t)group * (nb + 1);
    hipError_t e = launch_zero_u32(count, keys, s);
    if (e != hipSuccess) return e;
    if (n_beam > 0)
        hipLaunchKernelGGL(k_bin_count_split, dim3(nblocks(n_beam, kBlock)), dim3(kBlock), 0, s, g, n_beam, group,
                           (const double*)b.d_xi, count);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, count, (int)keys, start_all, fill);
    if (n_beam > 0)
        hipLaunchKernelGGL(k_bin_scatter_split, dim3(nblocks(n_beam, kBlock)), dim3(kBlock), 0, s, g, n_beam, group,
                           (const double*)b.d_xi, fill, order);
    hipLaunchKernelGGL(k_split_starts, dim3(nblocks((int64_t)group * (nb + 1), kBlock)), dim3(kBlock), 0, s, nb,
                       n_beam, group, start_all, bin_start);
    return hipGetLastError();
}

hipError_t launch_beam_push(const GridDesc& g, int64_t n_beam, const wk_beam_bufs& b, const void* fields,
                            int prec, int n_steps, double dt, unsigned long long* counters, hipStream_t s)
{
    if (n_beam <= 0 || n_steps <= 0) return hipSuccess;
    if (prec == WK_FP64)
        hipLaunchKernelGGL(k_beam_push<double>, dim3(nblocks(n_beam, kBlock)), dim3(kBlock), 0, s, g, n_beam,
                           b, (const double*)fields, n_steps, dt, counters);
    else
        hipLaunchKernelGGL(k_beam_push<float>, dim3(nblocks(n_beam, kBlock)), dim3(kBlock), 0, s, g, n_beam,
                           b, (const float*)fields, n_steps, dt, counters);
    return hipGetLastError();
}

hipError_t launch_mean_gain(int64_t n_beam, const wk_beam_bufs& b, int which, double* out, void* ws,
                            hipStream_t s)
{
    // partials live after the binning area of the workspace
    double* part = (double*)ws;
    hipLaunchKernelGGL(k_gain_partial, dim3(kGainBlocks), dim3(kBlock), 0, s, n_beam, b, which, part);
    hipLaunchKernelGGL(k_gain_final, dim3(1), dim3(64), 0, s, part, kGainBlocks, out);
    return hipGetLastError();
}

hipError_t launch_gain_hist(int64_t n_beam, const wk_beam_bufs& b, int which, int n_bins, double lo, double hi,
                            unsigned long long* hist, hipStream_t s)
{
    if (n_bins < 1 || n_bins > kHistMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(kBlock), 0, s, hist, (int64_t)n_bins + 2);
    if (n_beam > 0) {
        const int blocks = (int)std::min<int64_t>(1024, (n_beam + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_gain_hist, dim3(blocks), dim3(kBlock), 0, s, n_beam, b, which, n_bins, lo, hi, hist);
    }
    return hipGetLastError();
}

hipError_t launch_ez_peak(const GridDesc& g, const void* fields, int prec, double xi_from, double* out,
                          hipStream_t s)
{
    if (prec == WK_FP64)
        hipLaunchKernelGGL(k_ez_peak<double>, dim3(1), dim3(kBlock), 0, s, g, (const double*)fields, xi_from, out);
    else
        hipLaunchKernelGGL(k_ez_peak<float>, dim3(1), dim3(kBlock), 0, s, g, (const float*)fields, xi_from, out);
    return hipGetLastError();
}

}  // namespace wk
