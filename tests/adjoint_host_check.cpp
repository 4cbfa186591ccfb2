// Host-side check of the per-particle vector-Jacobian products of the
// adjoint against central finite differences of the forward functions they
// differentiate (random states, rows and adjoint seeds).  Prints one line per
// check: "<name> <max relative error>".
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_1411_3246_amd/csrc/wk_adjoint_dev.h"

using namespace wk::adj;

static std::mt19937_64 rng(12345);
static double U(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static double rel(double a, double b) { return std::fabs(a - b) / std::max(1e-12, std::max(std::fabs(a), std::fabs(b))); }

struct Rows {
    std::vector<double> psi, dpsi, bt;
};

static Rows random_rows(int N)
{
    Rows r;
    for (int j = 0; j <= N; ++j) {
        r.psi.push_back(U(-0.4, 0.4));
        r.dpsi.push_back(U(-1.0, 1.0));
        r.bt.push_back(U(-0.5, 0.5));
    }
    return r;
}

// a random state away from node boundaries, the axis and the wall by margin
template <int GEOM, bool WARM>
static St random_state(const Grid& G, bool beyond_wall)
{
    for (;;) {
        St s;
        double r = beyond_wall ? U(G.rmax + 0.05 * G.h, G.rmax + 0.9 * G.h) : U(0.3 * G.h, G.rmax - 0.3 * G.h);
        const double th = U(0.0, 6.28318530718);
        if (GEOM == WK_CYL && WARM) {
            s.x = r * std::cos(th);
            s.y = r * std::sin(th);
        } else {
            s.x = (GEOM == WK_SLAB && U(0, 1) < 0.5) ? -r : r;
            s.y = 0.0;
        }
        s.px = U(-0.3, 0.3);
        s.py = WARM ? U(-0.3, 0.3) : 0.0;
        const Geo g = geo_of<GEOM, WARM>(s, G);
        if (g.t > 0.02 && g.t < 0.98) return s;
    }
}

static double get(const St& s, int i) { return i == 0 ? s.x : i == 1 ? s.y : i == 2 ? s.px : s.py; }
static void add(St& s, int i, double v)
{
    if (i == 0) s.x += v;
    else if (i == 1) s.y += v;
    else if (i == 2) s.px += v;
    else s.py += v;
}

template <int GEOM, bool WARM>
static void check(const char* name)
{
    const Grid G{16, 0.375, 6.0, 0.05};
    double e_der = 0, e_mom = 0, e_s = 0, e_ref = 0;
    const int nvar = (GEOM == WK_CYL && WARM) ? 4 : (WARM ? 4 : 3);
    for (int trial = 0; trial < 200; ++trial) {
        Rows R = random_rows(G.N);
        const St s = random_state<GEOM, WARM>(G, false);
        const double d0 = U(0.8, 1.2), w = U(0.1, 1.0);
        const double eps = 1e-6;
        // derivative
        Der fb{U(-1, 1), U(-1, 1), U(-1, 1), U(-1, 1)};
        if (!(GEOM == WK_CYL && WARM)) fb.fy = 0.0;
        if (!WARM || GEOM == WK_SLAB) fb.fpy = 0.0;
        St sb{0, 0, 0, 0};
        double d0b = 0;
        derivative_vjp<GEOM, WARM>(s, d0, R.psi.data(), R.dpsi.data(), R.bt.data(), G, fb, sb, d0b);
        auto Jf = [&](const St& q, double dd0) {
            Der f = derivative<GEOM, WARM>(q, dd0, R.psi.data(), R.dpsi.data(), R.bt.data(), G);
            return fb.fx * f.fx + fb.fy * f.fy + fb.fpx * f.fpx + fb.fpy * f.fpy;
        };
        for (int i = 0; i < 4; ++i) {
            if (i == 1 && !(GEOM == WK_CYL && WARM)) continue;
            if (i == 3 && !WARM) continue;
            St a = s, b = s;
            add(a, i, eps);
            add(b, i, -eps);
            const double fd = (Jf(a, d0) - Jf(b, d0)) / (2 * eps);
            e_der = std::max(e_der, rel(fd, get(sb, i)));
        }
        e_der = std::max(e_der, rel((Jf(s, d0 + eps) - Jf(s, d0 - eps)) / (2 * eps), d0b));
        // the gathered-row adjoints: perturb one node of each row
        {
            DerAdj o = derivative_vjp<GEOM, WARM>(s, d0, R.psi.data(), R.dpsi.data(), R.bt.data(), G, fb, sb, d0b);
            Rows Rp = R, Rm = R;
            Rp.dpsi[o.j] += eps;
            Rm.dpsi[o.j] -= eps;
            const double fd = (fb.fpx * (derivative<GEOM, WARM>(s, d0, Rp.psi.data(), Rp.dpsi.data(), Rp.bt.data(), G).fpx -
                                         derivative<GEOM, WARM>(s, d0, Rm.psi.data(), Rm.dpsi.data(), Rm.bt.data(), G).fpx) +
                               fb.fpy * (derivative<GEOM, WARM>(s, d0, Rp.psi.data(), Rp.dpsi.data(), Rp.bt.data(), G).fpy -
                                         derivative<GEOM, WARM>(s, d0, Rm.psi.data(), Rm.dpsi.data(), Rm.bt.data(), G).fpy)) /
                              (2 * eps);
            e_der = std::max(e_der, rel(fd, o.gdpsi * (1.0 - o.t)));
        }
        (void)nvar;
        // moment terms
        double gr[7], dr[7];
        std::vector<std::vector<double>> grow(7, std::vector<double>(G.N + 1));
        for (int r = 0; r < 7; ++r)
            for (int j = 0; j <= G.N; ++j) grow[r][j] = U(-1, 1);
        const Geo g = geo_of<GEOM, WARM>(s, G);
        for (int r = 0; r < 7; ++r) {
            gr[r] = (1 - g.t) * grow[r][g.j] + g.t * grow[r][g.j + 1];
            dr[r] = grow[r][g.j + 1] - grow[r][g.j];
        }
        auto Jm = [&](const St& q, double dd0, double ww) {
            double c[7];
            const Geo gg = moment_terms<GEOM, WARM>(q, dd0, ww, R.psi.data(), G, c);
            double v = 0;
            for (int r = 0; r < 7; ++r) v += c[r] * ((1 - gg.t) * grow[r][gg.j] + gg.t * grow[r][gg.j + 1]);
            return v;
        };
        St mb{0, 0, 0, 0};
        double md0 = 0, mw = 0;
        moment_terms_vjp<GEOM, WARM>(s, d0, w, R.psi.data(), G, gr, dr, mb, md0, mw);
        for (int i = 0; i < 4; ++i) {
            if (i == 1 && !(GEOM == WK_CYL && WARM)) continue;
            if (i == 3 && !WARM) continue;
            St a = s, b = s;
            add(a, i, eps);
            add(b, i, -eps);
            e_mom = std::max(e_mom, rel((Jm(a, d0, w) - Jm(b, d0, w)) / (2 * eps), get(mb, i)));
        }
        e_mom = std::max(e_mom, rel((Jm(s, d0 + eps, w) - Jm(s, d0 - eps, w)) / (2 * eps), md0));
        e_mom = std::max(e_mom, rel((Jm(s, d0, w + eps) - Jm(s, d0, w - eps)) / (2 * eps), mw));
        // S term
        std::vector<double> sbar(G.N + 1);
        for (auto& v : sbar) v = U(-1, 1);
        auto Js = [&](const St& q, double ww) {
            const Geo gg = geo_of<GEOM, WARM>(q, G);
            return ww * ((1 - gg.t) * sbar[gg.j] + gg.t * sbar[gg.j + 1]);
        };
        St ssb{0, 0, 0, 0};
        double swb = 0;
        s_term_vjp<GEOM, WARM>(s, w, G, sbar.data(), ssb, swb);
        for (int i = 0; i < 2; ++i) {
            if (i == 1 && !(GEOM == WK_CYL && WARM)) continue;
            St a = s, b = s;
            add(a, i, eps);
            add(b, i, -eps);
            e_s = std::max(e_s, rel((Js(a, w) - Js(b, w)) / (2 * eps), get(ssb, i)));
        }
        e_s = std::max(e_s, rel((Js(s, w + eps) - Js(s, w - eps)) / (2 * eps), swb));
        // reflection
        const St o = random_state<GEOM, WARM>(G, true);
        St rb{U(-1, 1), (GEOM == WK_CYL && WARM) ? U(-1, 1) : 0.0, U(-1, 1), WARM && GEOM == WK_CYL ? U(-1, 1) : 0.0};
        auto Jr = [&](St q) {
            reflect<GEOM, WARM>(q, G.rmax);
            return rb.x * q.x + rb.y * q.y + rb.px * q.px + rb.py * q.py;
        };
        St ob = rb;
        reflect_vjp<GEOM, WARM>(o, G.rmax, ob);
        for (int i = 0; i < 4; ++i) {
            if (i == 1 && !(GEOM == WK_CYL && WARM)) continue;
            if (i == 3 && !(GEOM == WK_CYL && WARM)) continue;
            St a = o, b = o;
            add(a, i, eps);
            add(b, i, -eps);
            e_ref = std::max(e_ref, rel((Jr(a) - Jr(b)) / (2 * eps), get(ob, i)));
        }
    }
    std::printf("%s_derivative %.3e\n%s_moments %.3e\n%s_s_term %.3e\n%s_reflect %.3e\n", name, e_der, name, e_mom,
                name, e_s, name, e_ref);
}

static void check_boris()
{
    const int n_r = 8, n_xi = 12;
    const double r_max = 2.0, h = r_max / n_r, xi_min = 0.0, dxi = 0.25, dt = 40.0;
    std::vector<double> f(3 * n_xi * (n_r + 1));
    for (auto& v : f) v = U(-0.3, 0.3);
    const double* fez = f.data();
    const double* fb = fez + n_xi * (n_r + 1);
    const double* fw = fb + n_xi * (n_r + 1);
    double e = 0;
    for (int geom = 0; geom < 2; ++geom) {
        for (int trial = 0; trial < 200; ++trial) {
            double s0[6] = {U(-1.2, 1.2), geom == WK_CYL ? U(-1.2, 1.2) : 0.0, U(0.2, 2.6), U(-3, 3),
                            geom == WK_CYL ? U(-3, 3) : 0.0, 4.0e4 * (1 + U(-0.01, 0.01))};
            Dual d[6];
            for (int i = 0; i < 6; ++i) {
                d[i] = Dual(s0[i]);
                d[i].d[i] = 1.0;
            }
            boris_step<Dual>(geom, n_r, n_xi, r_max, h, xi_min, dxi, fez, fb, fw, d[0], d[1], d[2], d[3], d[4], d[5],
                             dt, false);
            for (int i = 0; i < 6; ++i) {
                if (geom == WK_SLAB && (i == 1 || i == 4)) continue;
                const double eps = (i == 5) ? 1e-2 : 1e-7;
                double a[6], b[6];
                for (int m = 0; m < 6; ++m) a[m] = b[m] = s0[m];
                a[i] += eps;
                b[i] -= eps;
                boris_step<double>(geom, n_r, n_xi, r_max, h, xi_min, dxi, fez, fb, fw, a[0], a[1], a[2], a[3], a[4],
                                   a[5], dt, false);
                boris_step<double>(geom, n_r, n_xi, r_max, h, xi_min, dxi, fez, fb, fw, b[0], b[1], b[2], b[3], b[4],
                                   b[5], dt, false);
                for (int o = 0; o < 6; ++o) {
                    const double fd = (a[o] - b[o]) / (2 * eps);
                    const double scale = std::max(1.0, std::fabs(fd));
                    e = std::max(e, std::fabs(fd - d[o].d[i]) / scale);
                }
            }
        }
    }
    std::printf("boris_step %.3e\n", e);
}

int main()
{
    check<WK_CYL, true>("cyl_warm");
    check<WK_CYL, false>("cyl_cold");
    check<WK_SLAB, true>("slab_warm");
    check<WK_SLAB, false>("slab_cold");
    check_boris();
    return 0;
}
