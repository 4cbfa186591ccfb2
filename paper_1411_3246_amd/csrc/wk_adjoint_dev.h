// Per-particle pieces of the adjoint (reverse-mode derivative) of the FP64
// plasma march and of the beam push: vector-Jacobian products of the hat
// geometry, of the stage derivative (Eqs. (4)-(5)), of the deposited terms
// (S and the currents/moments of Eqs. (1)-(3)), of the wall reflection and
// of one Boris step (Eqs. (8)-(11)).  Plain double arithmetic, usable on the
// host (checked there against finite differences) and on the device.
// Internal header of libwake.
#pragma once

#include <math.h>

#include "wk_internal.h"

namespace wk {
namespace adj {

// Grid constants seen by one particle.
struct Grid {
    int N;          // cells
    double h, rmax, dmin;
};

struct St {
    double x, y, px, py;
};

// Hat geometry of a particle (as in the march: the radius is |(x, y)| for a
// warm cylindrical plasma and |x| otherwise, folded at the wall).
template <typename P = double>
struct GeoT {
    P r, rho, sw, sg, t;
    int j;
    bool rho_clamped;
};
using Geo = GeoT<double>;

template <int GEOM, bool WARM, typename P = double>
__host__ __device__ inline GeoT<P> geo_of(const St& s, const Grid& G)
{
    GeoT<P> g;
    const P r = (GEOM == WK_CYL && WARM) ? sqrt(s.x * s.x + s.y * s.y) : fabs(s.x);
    g.r = r;
    P rho = r, sw = P(1.0);
    g.rho_clamped = false;
    if (r > G.rmax) {
        sw = -P(1.0);
        rho = P(2.0) * G.rmax - r;
        if (rho < P(0.0)) {
            rho = P(0.0);
            g.rho_clamped = true;
        }
    }
    g.rho = rho;
    g.sw = sw;
    g.sg = (GEOM == WK_SLAB) ? ((s.x < P(0.0)) ? -sw : sw) : sw;
    const P u = rho / G.h;
    int j = (int)floor(u);
    j = j < 0 ? 0 : (j > G.N - 1 ? G.N - 1 : j);
    g.j = j;
    g.t = u - (P)j;
    return g;
}

// Adjoint of the radius: add r_bar d r / d(x, y) to (xb, yb).
template <int GEOM, bool WARM, typename P = double>
__host__ __device__ inline void radius_vjp(const St& s, const GeoT<P>& g, P rb, double& xb, double& yb)
{
    if (GEOM == WK_CYL && WARM) {
        if (g.r > P(0.0)) {
            xb += rb * s.x / g.r;
            yb += rb * s.y / g.r;
        }
    } else {
        xb += rb * (s.x < P(0.0) ? -P(1.0) : (s.x > P(0.0) ? P(1.0) : P(0.0)));
    }
}

// Adjoint of the hat coordinate t = rho / h - j (and of a direct dependence
// on the folded radius rho_b and the unfolded radius r_b).
template <int GEOM, bool WARM, typename P = double>
__host__ __device__ inline void geo_vjp(const St& s, const GeoT<P>& g, const Grid& G, P tb, P rhob,
                                        P rb, double& xb, double& yb)
{
    const P rho_bar = tb / G.h + rhob;
    if (!g.rho_clamped) rb += g.sw * rho_bar;
    radius_vjp<GEOM, WARM, P>(s, g, rb, xb, yb);
}

template <typename P = double>
__host__ __device__ inline P hat_gather(const double* row, const GeoT<P>& g)
{
    return (P(1.0) - g.t) * (P)row[g.j] + g.t * (P)row[g.j + 1];
}

// ---------------------------------------------------------------------------
// Stage derivative of Eqs. (4)-(5) in the transverse Cartesian frame
// ---------------------------------------------------------------------------
struct Der {
    double fx, fy, fpx, fpy;
};

template <int GEOM, bool WARM, typename P = double>
__host__ __device__ inline Der derivative(const St& s, P d0, const double* psi, const double* dpsi,
                                          const double* bt, const Grid& G)
{
    const GeoT<P> g = geo_of<GEOM, WARM, P>(s, G);
    P D = d0 + hat_gather<P>(psi, g);
    if (D < G.dmin) D = G.dmin;
    const P px = s.px;
    const P py = WARM ? s.py : P(0.0);
    const P p2 = px * px + py * py;
    const P iD = P(1.0) / D;
    const P gam = (P(1.0) + p2 + D * D) * (P(0.5) * iD);
    const P F = (gam * iD) * hat_gather<P>(dpsi, g) - hat_gather<P>(bt, g);
    Der f;
    f.fx = px * iD;
    if (GEOM == WK_CYL) {
        f.fy = WARM ? py * iD : P(0.0);
        if (g.r > P(0.0)) {
            const P fr = g.sw * F * (P(1.0) / g.r);
            f.fpx = fr * s.x;
            f.fpy = WARM ? fr * s.y : P(0.0);
        } else {
            f.fpx = P(0.0);
            f.fpy = P(0.0);
        }
    } else {
        f.fy = P(0.0);
        f.fpx = g.sg * F;
        f.fpy = P(0.0);
    }
    return f;
}

// Adjoint of derivative(): given fb (adjoint of fx, fy, fpx, fpy) add to the
// state adjoint sb and to d0b; return the adjoints of the three gathered
// values (psi, psi', B) with the hat position, for deposit onto node rows.
struct DerAdj {
    double gpsi, gdpsi, gb, t;
    int j;
};

template <int GEOM, bool WARM, typename P = double>
__host__ __device__ inline DerAdj derivative_vjp(const St& s, P d0, const double* psi, const double* dpsi,
                                                 const double* bt, const Grid& G, const Der& fb, St& sb,
                                                 double& d0b)
{
    const GeoT<P> g = geo_of<GEOM, WARM, P>(s, G);
    const P ps0 = psi[g.j], ps1 = psi[g.j + 1];
    const P dp0 = dpsi[g.j], dp1 = dpsi[g.j + 1];
    const P b0 = bt[g.j], b1 = bt[g.j + 1];
    const P psig = (P(1.0) - g.t) * ps0 + g.t * ps1;
    const P dpg = (P(1.0) - g.t) * dp0 + g.t * dp1;
    const P bg = (P(1.0) - g.t) * b0 + g.t * b1;
    P D = d0 + psig;
    const bool clamped = D < G.dmin;
    if (clamped) D = G.dmin;
    const P px = s.px;
    const P py = WARM ? s.py : P(0.0);
    const P p2 = px * px + py * py;
    const P iD = P(1.0) / D;
    const P gam = (P(1.0) + p2 + D * D) * (P(0.5) * iD);
    const P F = (gam * iD) * dpg - bg;

    P Fb = P(0.0), rb = P(0.0);
    double xb = 0.0, yb = 0.0;
    if (GEOM == WK_CYL) {
        if (g.r > P(0.0)) {
            const P fr = g.sw * F / g.r;
            const P frb = fb.fpx * s.x + (WARM ? fb.fpy * s.y : P(0.0));
            xb += fr * fb.fpx;
            if (WARM) yb += fr * fb.fpy;
            Fb = g.sw * frb / g.r;
            rb -= g.sw * F * frb / (g.r * g.r);
        }
    } else {
        Fb = g.sg * fb.fpx;
    }
    const bool has_y = GEOM == WK_CYL && WARM;
    P iDb = fb.fx * px + (has_y ? fb.fy * py : P(0.0));
    P pxb = fb.fx * iD;
    P pyb = has_y ? fb.fy * iD : P(0.0);
    const P gamb = Fb * iD * dpg;
    iDb += Fb * gam * dpg;
    const P dpgb = Fb * gam * iD;
    const P bgb = -Fb;
    const P p2b = gamb * P(0.5) * iD;
    const P Db = gamb * (P(0.5) - P(0.5) * (P(1.0) + p2) * iD * iD) - iDb * iD * iD;
    pxb += P(2.0) * px * p2b;
    if (WARM) pyb += P(2.0) * py * p2b;
    P psigb = P(0.0);
    if (!clamped) {
        psigb = Db;
        d0b += Db;
    }
    const P tb = psigb * (ps1 - ps0) + dpgb * (dp1 - dp0) + bgb * (b1 - b0);
    geo_vjp<GEOM, WARM, P>(s, g, G, tb, P(0.0), rb, xb, yb);
    sb.x += xb;
    sb.y += yb;
    sb.px += pxb;
    sb.py += pyb;
    DerAdj o;
    o.gpsi = psigb;
    o.gdpsi = dpgb;
    o.gb = bgb;
    o.j = g.j;
    o.t = g.t;
    return o;
}

// ---------------------------------------------------------------------------
// Deposited terms of one particle: currents and moments (Eqs. (1)-(3))
// ---------------------------------------------------------------------------
// c[0..6] = J_r, J_z, M1, M2, M3, M4, M5 contributions (before the hat
// weights and the node volumes), as deposited by the march.
template <int GEOM, bool WARM, typename P = double>
__host__ __device__ inline GeoT<P> moment_terms(const St& s, P d0, P w, const double* psi, const Grid& G,
                                            P c[7])
{
    const GeoT<P> g = geo_of<GEOM, WARM, P>(s, G);
    P D = d0 + hat_gather<P>(psi, g);
    if (D < G.dmin) D = G.dmin;
    const P px = s.px;
    const P py = WARM ? s.py : P(0.0);
    const P p2 = px * px + py * py;
    const P iD = P(1.0) / D;
    const P h2D = P(0.5) * iD;
    const P gam = (P(1.0) + p2 + D * D) * h2D;
    const P pz = (P(1.0) + p2 - D * D) * h2D;
    P pr;
    if (GEOM == WK_CYL) {
        if (WARM)
            pr = g.r > P(0.0) ? g.sw * (s.x * px + s.y * py) * (P(1.0) / g.r) : P(0.0);
        else
            pr = g.r > P(0.0) ? g.sw * (s.x * px) * (P(1.0) / g.r) : P(0.0);
    } else {
        pr = g.sg * px;
    }
    const P wiD = w * iD;
    const P wiD2 = wiD * iD;
    c[0] = -wiD * pr;
    c[1] = -wiD * pz;
    c[2] = wiD;
    c[3] = wiD2 * (gam - pr * pr * iD);
    c[4] = P(0.0);
    if (GEOM == WK_CYL && WARM && g.rho > P(0.0)) {
        const P l = s.x * py - s.y * px;
        const P ir = P(1.0) / g.rho;
        c[4] = wiD2 * (l * l) * (ir * ir * ir);
    }
    c[5] = wiD2 * pr;
    c[6] = wiD2 * pr * pr;
    return g;
}

// Adjoint of the deposited terms.  gr[r] = row adjoint of term r gathered at
// the particle, dr[r] = its difference across the cell (row[j+1] - row[j]).
// Adds to sb, d0b, wb; returns the adjoint of the gathered psi (deposited
// onto the psi adjoint row at the returned hat position).
template <int GEOM, bool WARM, typename P = double>
__host__ __device__ inline DerAdj moment_terms_vjp(const St& s, P d0, P w, const double* psi,
                                                   const Grid& G, const double gr[7], const double dr[7], St& sb,
                                                   double& d0b, double& wb)
{
    P c[7];
    const GeoT<P> g = moment_terms<GEOM, WARM, P>(s, d0, w, psi, G, c);
    const P ps0 = psi[g.j], ps1 = psi[g.j + 1];
    P D = d0 + ((P(1.0) - g.t) * ps0 + g.t * ps1);
    const bool clamped = D < G.dmin;
    if (clamped) D = G.dmin;
    const P px = s.px;
    const P py = WARM ? s.py : P(0.0);
    const P p2 = px * px + py * py;
    const P iD = P(1.0) / D;
    const P gam = (P(1.0) + p2 + D * D) * (P(0.5) * iD);
    const P pz = (P(1.0) + p2 - D * D) * (P(0.5) * iD);
    P pr;
    if (GEOM == WK_CYL) {
        if (WARM) pr = g.r > P(0.0) ? g.sw * (s.x * px + s.y * py) / g.r : P(0.0);
        else pr = g.r > P(0.0) ? g.sw * (s.x * px) / g.r : P(0.0);
    } else {
        pr = g.sg * px;
    }
    const bool m3 = GEOM == WK_CYL && WARM && g.rho > P(0.0);
    const P l = (GEOM == WK_CYL && WARM) ? s.x * py - s.y * px : P(0.0);
    const P ir = m3 ? P(1.0) / g.rho : P(0.0);
    const P ir3 = ir * ir * ir;

    P tb = P(0.0);
    for (int r = 0; r < 7; ++r) tb += c[r] * dr[r];
    const P iD2 = iD * iD;
    wb += -iD * pr * gr[0] - iD * pz * gr[1] + iD * gr[2] + iD2 * (gam - pr * pr * iD) * gr[3] +
          iD2 * l * l * ir3 * gr[4] + iD2 * pr * gr[5] + iD2 * pr * pr * gr[6];
    const P iDb = -w * pr * gr[0] - w * pz * gr[1] + w * gr[2] +
                       w * (P(2.0) * iD * gam - P(3.0) * iD2 * pr * pr) * gr[3] + P(2.0) * w * iD * l * l * ir3 * gr[4] +
                       P(2.0) * w * iD * pr * gr[5] + P(2.0) * w * iD * pr * pr * gr[6];
    const P prb = -w * iD * gr[0] - P(2.0) * w * iD2 * iD * pr * gr[3] + w * iD2 * gr[5] +
                       P(2.0) * w * iD2 * pr * gr[6];
    const P pzb = -w * iD * gr[1];
    const P gamb = w * iD2 * gr[3];
    const P lb = P(2.0) * w * iD2 * l * ir3 * gr[4];
    const P rhob_direct = m3 ? -P(3.0) * w * iD2 * l * l * ir3 * ir * gr[4] : P(0.0);

    const P p2b = P(0.5) * iD * (gamb + pzb);
    const P Db = gamb * (P(0.5) - P(0.5) * (P(1.0) + p2) * iD2) + pzb * (-P(0.5) - P(0.5) * (P(1.0) + p2) * iD2) - iDb * iD2;
    double xb = 0.0, yb = 0.0;
    P pxb = P(2.0) * px * p2b, pyb = WARM ? P(2.0) * py * p2b : P(0.0), rb = P(0.0);
    if (GEOM == WK_CYL) {
        if (g.r > P(0.0)) {
            if (WARM) {
                xb += g.sw * px / g.r * prb;
                yb += g.sw * py / g.r * prb;
                pxb += g.sw * s.x / g.r * prb;
                pyb += g.sw * s.y / g.r * prb;
            } else {
                xb += g.sw * px / g.r * prb;
                pxb += g.sw * s.x / g.r * prb;
            }
            rb -= pr / g.r * prb;
        }
        if (WARM) {
            xb += py * lb;
            pyb += s.x * lb;
            yb -= px * lb;
            pxb -= s.y * lb;
        }
    } else {
        pxb += g.sg * prb;
    }
    P psigb = P(0.0);
    if (!clamped) {
        psigb = Db;
        d0b += Db;
        tb += Db * (ps1 - ps0);
    }
    geo_vjp<GEOM, WARM, P>(s, g, G, tb, rhob_direct, rb, xb, yb);
    sb.x += xb;
    sb.y += yb;
    sb.px += pxb;
    sb.py += pyb;
    DerAdj o;
    o.gpsi = psigb;
    o.gdpsi = P(0.0);
    o.gb = P(0.0);
    o.j = g.j;
    o.t = g.t;
    return o;
}

// Adjoint of the S deposit (weight w at the hat): gsb = S adjoint row
// gathered at the particle, dsb = its difference across the cell.
template <int GEOM, bool WARM, typename P = double>
__host__ __device__ inline void s_term_vjp(const St& s, P w, const Grid& G, const double* sbar, St& sb, double& wb)
{
    const GeoT<P> g = geo_of<GEOM, WARM, P>(s, G);
    const P a0 = sbar[g.j], a1 = sbar[g.j + 1];
    wb += (P(1.0) - g.t) * a0 + g.t * a1;
    double xb = 0.0, yb = 0.0;
    geo_vjp<GEOM, WARM, P>(s, g, G, w * (a1 - a0), P(0.0), P(0.0), xb, yb);
    sb.x += xb;
    sb.y += yb;
}

// ---------------------------------------------------------------------------
// Wall reflection at the end of a step
// ---------------------------------------------------------------------------
template <int GEOM, bool WARM>
__host__ __device__ inline bool reflect(St& p, double rmax)
{
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
            return true;
        }
        return false;
    }
    const double ax = fabs(p.x);
    if (ax > rmax) {
        double xn = 2.0 * rmax - ax;
        if (xn < 0.0) xn = 0.0;
        p.x = p.x < 0.0 ? -xn : xn;
        p.px = -p.px;
        return true;
    }
    return false;
}

// Adjoint of reflect() at the pre-reflection state p (when it reflected):
// maps the adjoint of the reflected state to that of p, in place.
template <int GEOM, bool WARM>
__host__ __device__ inline void reflect_vjp(const St& p, double rmax, St& b)
{
    if (GEOM == WK_CYL) {
        const double r = WARM ? sqrt(p.x * p.x + p.y * p.y) : fabs(p.x);
        double rn = 2.0 * rmax - r;
        const bool rn_clamped = rn < 0.0;
        if (rn_clamped) rn = 0.0;
        const double ux = p.x / r, uy = WARM ? p.y / r : 0.0;
        const double pr = ux * p.px + uy * p.py;
        const double xb = b.x, yb = WARM ? b.y : 0.0, pxb = b.px, pyb = WARM ? b.py : 0.0;
        const double prb = -2.0 * (pxb * ux + pyb * uy);
        double opx = pxb + prb * ux;
        double opy = pyb + prb * uy;
        const double uxb = rn * xb - 2.0 * pr * pxb + prb * p.px;
        const double uyb = WARM ? rn * yb - 2.0 * pr * pyb + prb * p.py : 0.0;
        double rb = rn_clamped ? 0.0 : -(xb * ux + yb * uy);
        double ox = uxb / r, oy = WARM ? uyb / r : 0.0;
        rb -= (uxb * p.x + uyb * (WARM ? p.y : 0.0)) / (r * r);
        ox += rb * p.x / r;
        if (WARM) oy += rb * p.y / r;
        b.x = ox;
        b.px = opx;
        if (WARM) {
            b.y = oy;
            b.py = opy;
        }
        return;
    }
    const double ax = fabs(p.x);
    const bool clamped = 2.0 * rmax - ax < 0.0;
    b.x = clamped ? 0.0 : -b.x;
    b.px = -b.px;
}

// ---------------------------------------------------------------------------
// Beam push: one Boris step, Eqs. (8)-(11) with q = -1, as a function of the
// state and of the three gathered field values, differentiated in forward
// mode with a small dual-number type (6 state + 3 field directions).
// ---------------------------------------------------------------------------
constexpr int kDualN = 9;

struct Dual {
    double v;
    double d[kDualN];
    __host__ __device__ Dual() : v(0.0)
    {
        for (int i = 0; i < kDualN; ++i) d[i] = 0.0;
    }
    __host__ __device__ Dual(double a) : v(a)
    {
        for (int i = 0; i < kDualN; ++i) d[i] = 0.0;
    }
};

__host__ __device__ inline Dual operator+(const Dual& a, const Dual& b)
{
    Dual c(a.v + b.v);
    for (int i = 0; i < kDualN; ++i) c.d[i] = a.d[i] + b.d[i];
    return c;
}
__host__ __device__ inline Dual operator-(const Dual& a, const Dual& b)
{
    Dual c(a.v - b.v);
    for (int i = 0; i < kDualN; ++i) c.d[i] = a.d[i] - b.d[i];
    return c;
}
__host__ __device__ inline Dual operator-(const Dual& a)
{
    Dual c(-a.v);
    for (int i = 0; i < kDualN; ++i) c.d[i] = -a.d[i];
    return c;
}
__host__ __device__ inline Dual operator*(const Dual& a, const Dual& b)
{
    Dual c(a.v * b.v);
    for (int i = 0; i < kDualN; ++i) c.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return c;
}
__host__ __device__ inline Dual operator/(const Dual& a, const Dual& b)
{
    const double ib = 1.0 / b.v;
    Dual c(a.v * ib);
    for (int i = 0; i < kDualN; ++i) c.d[i] = (a.d[i] - c.v * b.d[i]) * ib;
    return c;
}
__host__ __device__ inline Dual dsqrt(const Dual& a)
{
    const double s = sqrt(a.v);
    Dual c(s);
    const double k = s > 0.0 ? 0.5 / s : 0.0;
    for (int i = 0; i < kDualN; ++i) c.d[i] = a.d[i] * k;
    return c;
}
__host__ __device__ inline double val(const Dual& a) { return a.v; }
__host__ __device__ inline double val(double a) { return a; }
__host__ __device__ inline double dsqrt(double a) { return sqrt(a); }

// Bilinear (r, xi) cell of a beam particle and whether it is inside the
// window (outside: zero fields).
struct BeamCell {
    bool inside;
    int j, k, k1;
};

// One Boris step of a beam particle in the fields (fez, fb, fw planes of
// [n_xi][n_r + 1], stored as FT: double, or float for mixed plans); S =
// double or Dual.  When `seed` the field values get the dual directions 6,
// 7, 8 (E_z, B_theta, W).
template <typename S, typename FT = double>
__host__ __device__ inline BeamCell boris_step(int geom, int n_r, int n_xi, double r_max, double h, double xi_min,
                                               double dxi, const FT* fez, const FT* fb, const FT* fw,
                                               S& x, S& y, S& xi, S& px, S& py, S& pz, double dt, bool seed)
{
    const int N1 = n_r + 1;
    const double xi_max = xi_min + n_xi * dxi;
    const double qh = -0.5 * dt;
    BeamCell cell;
    cell.inside = false;
    cell.j = cell.k = cell.k1 = 0;
    const S r = geom == WK_CYL ? dsqrt(x * x + y * y) : (val(x) < 0.0 ? -x : x);
    S ez(0.0), bt(0.0), wv(0.0);
    if (val(r) <= r_max && val(xi) >= xi_min && val(xi) < xi_max) {
        const double u_r = val(r) / h;
        int j = (int)floor(u_r);
        j = j < 0 ? 0 : (j > n_r - 1 ? n_r - 1 : j);
        const S tr = r / S(h) - S((double)j);
        const S u = (xi - S(xi_min)) / S(dxi);
        int k = (int)floor(val(u));
        if (k > n_xi - 1) k = n_xi - 1;
        const S tk = u - S((double)k);
        const int k1 = k + 1 < n_xi ? k + 1 : k;
        const S tk1 = k + 1 < n_xi ? tk : S(0.0);
        const S one(1.0);
        const S w00 = (one - tr) * (one - tk1), w01 = tr * (one - tk1);
        const S w10 = (one - tr) * tk1, w11 = tr * tk1;
        const int64_t o0 = (int64_t)k * N1 + j, o1 = (int64_t)k1 * N1 + j;
        ez = w00 * S((double)fez[o0]) + w01 * S((double)fez[o0 + 1]) + w10 * S((double)fez[o1]) +
             w11 * S((double)fez[o1 + 1]);
        bt = w00 * S((double)fb[o0]) + w01 * S((double)fb[o0 + 1]) + w10 * S((double)fb[o1]) +
             w11 * S((double)fb[o1 + 1]);
        wv = w00 * S((double)fw[o0]) + w01 * S((double)fw[o0 + 1]) + w10 * S((double)fw[o1]) +
             w11 * S((double)fw[o1 + 1]);
        cell.inside = true;
        cell.j = j;
        cell.k = k;
        cell.k1 = k1;
    }
    if (seed) {
        // gathered field values as independent inputs (zero outside)
        if constexpr (sizeof(S) > sizeof(double)) {
            ez.d[6] += 1.0;
            bt.d[7] += 1.0;
            wv.d[8] += 1.0;
        }
    }
    const S er = wv + bt;
    S ux, uy;
    if (geom == WK_CYL) {
        ux = val(r) > 0.0 ? x / r : S(0.0);
        uy = val(r) > 0.0 ? y / r : S(0.0);
    } else {
        ux = S(val(x) < 0.0 ? -1.0 : 1.0);
        uy = S(0.0);
    }
    const S Ex = er * ux, Ey = er * uy, Ez = ez;
    const S Bx = -(bt * uy), By = bt * ux;
    const S q(qh);
    const S mx = px + q * Ex, my = py + q * Ey, mz = pz + q * Ez;
    const S gm = dsqrt(S(1.0) + mx * mx + my * my + mz * mz);
    const S tx = q * Bx / gm, ty = q * By / gm;
    const S t2 = tx * tx + ty * ty;
    const S qx = mx - mz * ty;
    const S qy = my + mz * tx;
    const S qz = mz + (mx * ty - my * tx);
    const S den = S(1.0) + t2;
    const S sx = S(2.0) * tx / den, sy = S(2.0) * ty / den;
    const S nx = mx - qz * sy;
    const S ny = my + qz * sx;
    const S nz = mz + (qx * sy - qy * sx);
    px = nx + q * Ex;
    py = ny + q * Ey;
    pz = nz + q * Ez;
    const S pp2 = px * px + py * py;
    const S gam = dsqrt(S(1.0) + pp2 + pz * pz);
    const S D(dt);
    x = x + D * px / gam;
    y = y + D * py / gam;
    xi = xi + D * (S(1.0) + pp2) / (gam * (gam + pz));
    return cell;
}

}  // namespace adj
}  // namespace wk
