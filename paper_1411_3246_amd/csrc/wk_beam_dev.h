// Device functions of the beam (shared by the standalone beam kernels and the
// pipelined quasi-static cycle).  Internal header of libwake.
#pragma once

#include "wk_internal.h"

namespace wk {
namespace dev {

__device__ __forceinline__ double grid_node_volume(const GridDesc& g, int j)
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

__device__ __forceinline__ void grid_hat(const GridDesc& g, double rho, int& j, double& t)
{
    const double u = rho / g.h;
    int jj = (int)floor(u);
    jj = jj < 0 ? 0 : (jj > g.n_r - 1 ? g.n_r - 1 : jj);
    j = jj;
    t = u - (double)jj;
}

__device__ __forceinline__ double beam_radius(const GridDesc& g, double x, double y)
{
    return g.geom == WK_CYL ? sqrt(x * x + y * y) : fabs(x);
}

// xi cell of a beam particle, or n_xi when it is outside [xi_min, xi_max).
__device__ __forceinline__ int beam_xi_bin(const GridDesc& g, double xi)
{
    const double xi_max = g.xi_min + g.n_xi * g.dxi;
    if (xi < g.xi_min || xi >= xi_max) return g.n_xi;
    const int k = (int)floor((xi - g.xi_min) / g.dxi);
    return k > g.n_xi - 1 ? g.n_xi - 1 : k;
}

// Field value for the push: a plain load, or (COH) a device-coherent load of
// fields that another compute unit stored during the same launch.
template <bool COH, typename R>
__device__ __forceinline__ double field_at(const R* p)
{
    if (COH) return (double)__hip_atomic_load(const_cast<R*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (double)*p;
}

// Eqs. (8)-(11) for an electron (q = -1) in the frozen fields: E = (E_r x/r,
// E_r y/r, E_z), B = B_theta e_theta with E_r = W + B_theta, bilinear in
// (r, xi); Boris rotation; d xi/dt = (1 + p_perp^2) / (gamma (gamma + p_z)).
// Returns the number of steps taken outside the window (zero fields).
template <typename R, bool COH = false>
__device__ __forceinline__ unsigned long long beam_push_particle(const GridDesc& g, const R* __restrict__ fields,
                                                        double& x, double& y, double& xi, double& px,
                                                        double& py, double& pz, int n_steps, double dt)
{
    const int N1 = g.n_r + 1;
    const int64_t plane = (int64_t)g.n_xi * N1;
    const R* fez = fields + plane;
    const R* fb = fields + 2 * plane;
    const R* fw = fields + 3 * plane;
    const double xi_max = g.xi_min + g.n_xi * g.dxi;
    const double qh = -0.5 * dt;
    unsigned long long out = 0;
    for (int s = 0; s < n_steps; ++s) {
        const double r = beam_radius(g, x, y);
        double ez = 0.0, bt = 0.0, wv = 0.0;
        if (r <= g.r_max && xi >= g.xi_min && xi < xi_max) {
            int j;
            double tr;
            grid_hat(g, r, j, tr);
            const double u = (xi - g.xi_min) / g.dxi;
            int k = (int)floor(u);
            if (k > g.n_xi - 1) k = g.n_xi - 1;
            const double tk = u - k;
            const int k1 = k + 1 < g.n_xi ? k + 1 : k;
            const double tk1 = k + 1 < g.n_xi ? tk : 0.0;
            const double w00 = (1.0 - tr) * (1.0 - tk1), w01 = tr * (1.0 - tk1);
            const double w10 = (1.0 - tr) * tk1, w11 = tr * tk1;
            const int64_t o0 = (int64_t)k * N1 + j, o1 = (int64_t)k1 * N1 + j;
            ez = w00 * field_at<COH>(fez + o0) + w01 * field_at<COH>(fez + o0 + 1) +
                 w10 * field_at<COH>(fez + o1) + w11 * field_at<COH>(fez + o1 + 1);
            bt = w00 * field_at<COH>(fb + o0) + w01 * field_at<COH>(fb + o0 + 1) + w10 * field_at<COH>(fb + o1) +
                 w11 * field_at<COH>(fb + o1 + 1);
            wv = w00 * field_at<COH>(fw + o0) + w01 * field_at<COH>(fw + o0 + 1) + w10 * field_at<COH>(fw + o1) +
                 w11 * field_at<COH>(fw + o1 + 1);
        } else {
            ++out;
        }
        const double er = wv + bt;
        double ux, uy;
        if (g.geom == WK_CYL) {
            ux = r > 0.0 ? x / r : 0.0;
            uy = r > 0.0 ? y / r : 0.0;
        } else {
            ux = x < 0.0 ? -1.0 : 1.0;
            uy = 0.0;
        }
        const double Ex = er * ux, Ey = er * uy, Ez = ez;
        const double Bx = -bt * uy, By = bt * ux;
        const double mx = px + qh * Ex, my = py + qh * Ey, mz = pz + qh * Ez;
        const double gm = sqrt(1.0 + mx * mx + my * my + mz * mz);
        const double tx = qh * Bx / gm, ty = qh * By / gm, tz = 0.0;
        const double t2 = tx * tx + ty * ty + tz * tz;
        const double qx = mx + (my * tz - mz * ty);
        const double qy = my + (mz * tx - mx * tz);
        const double qz = mz + (mx * ty - my * tx);
        const double sx = 2.0 * tx / (1.0 + t2), sy = 2.0 * ty / (1.0 + t2), sz = 2.0 * tz / (1.0 + t2);
        const double nx = mx + (qy * sz - qz * sy);
        const double ny = my + (qz * sx - qx * sz);
        const double nz = mz + (qx * sy - qy * sx);
        px = nx + qh * Ex;
        py = ny + qh * Ey;
        pz = nz + qh * Ez;
        const double pp2 = px * px + py * py;
        const double gam = sqrt(1.0 + pp2 + pz * pz);
        x = x + dt * px / gam;
        y = y + dt * py / gam;
        xi = xi + dt * (1.0 + pp2) / (gam * (gam + pz));
    }
    return out;
}

}  // namespace dev
}  // namespace wk
