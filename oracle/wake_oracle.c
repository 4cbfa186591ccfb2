/*
 * Serial FP64 CPU oracle for the quasi-static plasma response of the WAKE
 * paper (arXiv:1411.3246).  TEST INFRASTRUCTURE ONLY: the product path never
 * links or calls this file.  Every function below states the passage of the
 * paper it follows; where the paper gives no discretization, the reading
 * taken is written next to the code.
 *
 * Model (Section II A):
 *   invariant    gamma - p_z + psi = gamma0 - p_z0 =: D0           Eq. (1), q = -1
 *   gamma, p_z   from D = D0 + psi                                Eqs. (2)-(3)
 *   radial EOM   dp_r/dxi = (gamma/D) dpsi/dr + l^2/(D r^3) - B    Eq. (4)
 *                dr/dxi   = p_r / D                                Eq. (5)
 *   fields       (1/r) d_r (r B) = d_xi^2 psi + J_z                Eq. (6)
 *                d_xi d_r psi   = J_r                              Eq. (7)
 *   beam         Eqs. (8)-(11), density Eq. (12).
 *
 * Readings where the paper is silent:
 *   - The transverse motion of each ring electron is integrated in the
 *     Cartesian transverse plane (x, y, p_x, p_y); the ring radius is
 *     r = |(x, y)|, p_r and l_z = x p_y - y p_x follow, and Eqs. (4)-(5) are
 *     this motion written in polar form.  This avoids the coordinate
 *     singularity of l_z^2/r^3 on the axis; for l_z = 0 it reduces exactly to
 *     the mirror-extended polar form.  Slab: x with mirror symmetry, p_y is a
 *     conserved canonical momentum.
 *   - psi from the transverse Poisson equation lap_perp psi = S - n_ion with
 *     S = n (1 - v_z) (Gauss's law minus Eq. (6)), psi(r_max) = 0.
 *   - E_z = -int_r^{r_max} J_r dr' (Eq. (7), E_z(r_max) = 0).
 *   - B_theta from Eq. (6) differentiated in r with d_xi J_r eliminated
 *     through Eqs. (1)-(5) and particle continuity, which gives the
 *     tridiagonal Helmholtz problem
 *        d_r[(1/r) d_r(r B)] - M1 B = d_r J_z - M2 psi' - M3 + M4 E_z
 *                                     + (1/r) d_r (r M5).
 *   - Linear hat shape in r for deposit and gather; node volumes are the
 *     integrals of the hats; Heun (RK2) integration in xi.
 */
#include "wake_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

typedef struct {
    const or_problem* p;
    int N;           /* radial cells */
    double h;        /* radial cell size */
    double alpha;    /* 1 cylindrical, 0 slab */
    double dxi;      /* slice spacing */
    double* V;       /* node volumes (N+1) */
    double* rn;      /* node radii (N+1) */
} grid_t;

static int check_problem(const or_problem* p)
{
    if (!p) return -1;
    if (p->geom != OR_CYL && p->geom != OR_SLAB) return -1;
    if (p->n_r < 2 || p->n_xi < 1 || p->ppc < 1) return -1;
    if (!(p->r_max > 0.0) || !(p->xi_max > p->xi_min)) return -1;
    if (p->u_th < 0.0 || (p->u_th > 0.0 && (p->ppc % 2) != 0)) return -1;
    if (p->n_bunch < 0 || p->n_bunch > 2) return -1;
    if (!(p->d_min > 0.0)) return -1;
    return 0;
}

/* Node volume V_j = integral of the hat function of node j times the
 * transverse measure (2 pi r dr in cylindrical, dx in slab) over [0, r_max]. */
static double node_volume(const or_problem* p, int j)
{
    const int N = p->n_r;
    const double h = p->r_max / N;
    if (p->geom == OR_CYL) {
        if (j == 0) return OR_PI * h * h / 3.0;
        if (j == N) return OR_PI * h * h * ((double)N - 1.0 / 3.0);
        return 2.0 * OR_PI * (double)j * h * h;
    }
    if (j == 0 || j == N) return 0.5 * h;
    return h;
}

static int grid_init(const or_problem* p, grid_t* g)
{
    g->p = p;
    g->N = p->n_r;
    g->h = p->r_max / p->n_r;
    g->alpha = (p->geom == OR_CYL) ? 1.0 : 0.0;
    g->dxi = (p->xi_max - p->xi_min) / p->n_xi;
    g->V = (double*)malloc(sizeof(double) * (g->N + 1));
    g->rn = (double*)malloc(sizeof(double) * (g->N + 1));
    if (!g->V || !g->rn) return -2;
    for (int j = 0; j <= g->N; ++j) {
        g->V[j] = node_volume(p, j);
        g->rn[j] = j * g->h;
    }
    return 0;
}

static void grid_free(grid_t* g)
{
    free(g->V);
    free(g->rn);
}

/* Transverse radius of a particle (cylindrical |(x,y)|, slab |x|). */
static double radius_of(const grid_t* g, double x, double y)
{
    if (g->p->geom == OR_CYL) return sqrt(x * x + y * y);
    return fabs(x);
}

/* Position used for deposit and gather.  A predictor state beyond the outer
 * wall is folded back as its specular image (rho = 2 r_max - r) and the sign
 * of radial vector quantities flips (*wall_sign = -1). */
static double fold_radius(const grid_t* g, double r, double* wall_sign)
{
    const double rmax = g->p->r_max;
    *wall_sign = 1.0;
    if (r > rmax) {
        *wall_sign = -1.0;
        r = 2.0 * rmax - r;
        if (r < 0.0) r = 0.0;
    }
    return r;
}

/* Linear hat weights: node j gets (1-t), node j+1 gets t. */
static void hat(const grid_t* g, double rho, int* j, double* t)
{
    double u = rho / g->h;
    int jj = (int)floor(u);
    if (jj < 0) jj = 0;
    if (jj > g->N - 1) jj = g->N - 1;
    *j = jj;
    *t = u - (double)jj;
}

int or_thomas(int64_t n, const double* a, const double* b, const double* c,
              const double* d, double* x)
{
    if (n < 1) return -1;
    double* cp = (double*)malloc(sizeof(double) * n);
    double* dp = (double*)malloc(sizeof(double) * n);
    if (!cp || !dp) { free(cp); free(dp); return -2; }
    double den = b[0];
    cp[0] = (n > 1) ? c[0] / den : 0.0;
    dp[0] = d[0] / den;
    for (int64_t i = 1; i < n; ++i) {
        den = b[i] - a[i] * cp[i - 1];
        cp[i] = (i < n - 1) ? c[i] / den : 0.0;
        dp[i] = (d[i] - a[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int64_t i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    free(cp);
    free(dp);
    return 0;
}

int64_t or_plasma_count(const or_problem* p)
{
    if (check_problem(p)) return -1;
    return (int64_t)p->n_r * p->ppc;
}

/*
 * Plasma loader.  The paper takes the constant of motion D0 = gamma0 - p_z0
 * of each particle from its thermal momentum (Section II A, after Eq. (1)) and
 * uses a fixed number of particles per cell (Section III).  Reading: ring
 * particles at cell-uniform radii; warm plasma is loaded in mirrored pairs
 * (p0, -p0) with p0 = u_th * eps, and each member carries the flux weight
 * a * D0/gamma0 (the xi-flux n(1 - v_z) of its share a of the sub-annulus), so
 * that the flux density, J_r and J_z vanish in the unperturbed plasma.  The
 * immobile ion density is the deposit of the initial areas.
 */
int or_load_plasma(const or_problem* p, const double* eps,
                   double* x, double* y, double* px, double* py,
                   double* d0, double* w, double* nion)
{
    if (check_problem(p)) return -1;
    grid_t g;
    if (grid_init(p, &g)) { grid_free(&g); return -2; }
    const int N = g.N;
    const int warm = p->u_th > 0.0;
    const int npos = warm ? p->ppc / 2 : p->ppc;   /* radii per cell */
    if (warm && !eps) { grid_free(&g); return -1; }
    for (int j = 0; j <= N; ++j) nion[j] = 0.0;

    int64_t i = 0;
    for (int c = 0; c < N; ++c) {
        for (int m = 0; m < npos; ++m) {
            const double rlo = (c + (double)m / npos) * g.h;
            const double rhi = (c + (double)(m + 1) / npos) * g.h;
            const double r0 = (c + (m + 0.5) / npos) * g.h;
            double area;
            if (p->geom == OR_CYL) area = p->n0 * OR_PI * (rhi * rhi - rlo * rlo);
            else area = p->n0 * (rhi - rlo);

            int jj; double t;
            hat(&g, r0, &jj, &t);
            nion[jj] += area * (1.0 - t);
            nion[jj + 1] += area * t;

            if (!warm) {
                x[i] = r0; y[i] = 0.0; px[i] = 0.0; py[i] = 0.0;
                d0[i] = 1.0; w[i] = area;
                ++i;
                continue;
            }
            const int64_t q = (int64_t)c * npos + m;
            const double pr0 = p->u_th * eps[3 * q + 0];
            const double pt0 = p->u_th * eps[3 * q + 1];
            const double pz0 = p->u_th * eps[3 * q + 2];
            const double g0 = sqrt(1.0 + pr0 * pr0 + pt0 * pt0 + pz0 * pz0);
            const double half = 0.5 * area;
            for (int s = 0; s < 2; ++s) {
                const double sg = s == 0 ? 1.0 : -1.0;
                const double dd = g0 - sg * pz0;
                x[i] = r0; y[i] = 0.0;
                px[i] = sg * pr0; py[i] = sg * pt0;
                d0[i] = dd;
                w[i] = half * dd / g0;
                ++i;
            }
        }
    }
    for (int j = 0; j <= N; ++j) nion[j] /= g.V[j];
    grid_free(&g);
    return 0;
}

/* Beam density of Eq. (12) at (r, xi). */
static double beam_density(const or_problem* p, double r, double xi)
{
    double s = 0.0;
    for (int b = 0; b < p->n_bunch; ++b) {
        const double u = (xi - p->xi_c[b]) / p->sigma_z[b];
        s += p->n_peak[b] * exp(-0.5 * u * u);
    }
    const double v = r / p->sigma_r;
    return exp(-0.5 * v * v) * s;
}

/* Fixed-beam current: the beam moves at v_z = c, so J_bz = -n_b (Eq. (12)
 * and the total current of Section II A). */
int or_beam_current_analytic(const or_problem* p, double* jb)
{
    if (check_problem(p)) return -1;
    const int N = p->n_r;
    const double h = p->r_max / N;
    const double dxi = (p->xi_max - p->xi_min) / p->n_xi;
    for (int k = 0; k < p->n_xi; ++k) {
        const double xi = p->xi_min + k * dxi;
        for (int j = 0; j <= N; ++j)
            jb[(int64_t)k * (N + 1) + j] = -beam_density(p, j * h, xi);
    }
    return 0;
}

/* Charge of bunch b of Eq. (12) over the half domain represented by the grid
 * (full plane in cylindrical geometry, x >= 0 in slab geometry). */
static double bunch_charge(const or_problem* p, int b)
{
    const double sz = sqrt(2.0 * OR_PI) * p->sigma_z[b];
    double sperp;
    if (p->geom == OR_CYL) sperp = 2.0 * OR_PI * p->sigma_r * p->sigma_r;
    else sperp = sqrt(0.5 * OR_PI) * p->sigma_r;
    return p->n_peak[b] * sz * sperp;
}

/*
 * Beam macroparticles sampling Eq. (12): Gaussian in x, y (common sigma_r)
 * and in xi about each bunch centre, zero emittance (Section III: the
 * initial beam emittance is zero), energy spread about gamma0.
 */
int or_load_beam(const or_problem* p, int64_t n_beam, int64_t n_drive,
                 double gamma0, double rel_spread, const double* eps,
                 double* bx, double* by, double* bpx, double* bpy, double* bpz,
                 double* bxi, double* bw, int32_t* tag)
{
    if (check_problem(p) || n_beam < 0 || n_drive < 0 || n_drive > n_beam) return -1;
    if (p->n_bunch < 1 || (p->n_bunch == 1 && n_drive != n_beam)) return -1;
    if (p->n_bunch == 2 && (n_drive == 0 || n_drive == n_beam)) return -1;
    const double wd = bunch_charge(p, 0) / (double)n_drive;
    const double ww = (p->n_bunch == 2) ? bunch_charge(p, 1) / (double)(n_beam - n_drive) : 0.0;
    for (int64_t i = 0; i < n_beam; ++i) {
        const int b = (i < n_drive) ? 0 : 1;
        const double* e = eps + 4 * i;
        bx[i] = p->sigma_r * e[0];
        by[i] = (p->geom == OR_CYL) ? p->sigma_r * e[1] : 0.0;
        bxi[i] = p->xi_c[b] + p->sigma_z[b] * e[2];
        const double gam = gamma0 * (1.0 + rel_spread * e[3]);
        bpx[i] = 0.0;
        bpy[i] = 0.0;
        bpz[i] = sqrt(gam * gam - 1.0);
        bw[i] = b == 0 ? wd : ww;
        tag[i] = b;
    }
    return 0;
}

/* J_bz = -(sum of W hat_j(r) hat_k(xi)) / (V_j dxi): the macroparticle form
 * of the beam current (v_z = c). */
int or_beam_current_macro(const or_problem* p, int64_t n_beam,
                          const double* bx, const double* by, const double* bxi,
                          const double* bw, double* jb, int64_t* n_out)
{
    if (check_problem(p)) return -1;
    grid_t g;
    if (grid_init(p, &g)) { grid_free(&g); return -2; }
    const int N = g.N;
    const int64_t tot = (int64_t)p->n_xi * (N + 1);
    for (int64_t q = 0; q < tot; ++q) jb[q] = 0.0;
    int64_t out = 0;
    for (int64_t i = 0; i < n_beam; ++i) {
        const double r = radius_of(&g, bx[i], by[i]);
        const double xi = bxi[i];
        if (r > p->r_max || xi < p->xi_min || xi >= p->xi_max) { ++out; continue; }
        int j; double tr;
        hat(&g, r, &j, &tr);
        const double u = (xi - p->xi_min) / g.dxi;
        int k = (int)floor(u);
        if (k > p->n_xi - 1) k = p->n_xi - 1;
        const double tk = u - k;
        double* row0 = jb + (int64_t)k * (N + 1);
        row0[j] += bw[i] * (1.0 - tr) * (1.0 - tk);
        row0[j + 1] += bw[i] * tr * (1.0 - tk);
        if (k + 1 < p->n_xi) {
            double* row1 = row0 + (N + 1);
            row1[j] += bw[i] * (1.0 - tr) * tk;
            row1[j + 1] += bw[i] * tr * tk;
        }
    }
    for (int k = 0; k < p->n_xi; ++k)
        for (int j = 0; j <= N; ++j)
            jb[(int64_t)k * (N + 1) + j] = -jb[(int64_t)k * (N + 1) + j] / (g.V[j] * g.dxi);
    if (n_out) *n_out = out;
    grid_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Stage evaluation                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *S, *psi, *dpsi, *Jr, *Jz, *M1, *M2, *M3, *M4, *M5, *Ez, *B, *Q;
    double *ta, *tb, *tc, *td, *tx;
    double *D, *gam;
} scratch_t;

static int scratch_init(scratch_t* s, int N, int64_t np)
{
    memset(s, 0, sizeof(*s));
    const size_t n1 = (size_t)(N + 1);
    double** rows[] = {&s->S, &s->psi, &s->dpsi, &s->Jr, &s->Jz, &s->M1, &s->M2,
                       &s->M3, &s->M4, &s->M5, &s->Ez, &s->B, &s->Q,
                       &s->ta, &s->tb, &s->tc, &s->td, &s->tx};
    for (size_t q = 0; q < sizeof(rows) / sizeof(rows[0]); ++q) {
        *rows[q] = (double*)calloc(n1, sizeof(double));
        if (!*rows[q]) return -2;
    }
    s->D = (double*)calloc((size_t)(np > 0 ? np : 1), sizeof(double));
    s->gam = (double*)calloc((size_t)(np > 0 ? np : 1), sizeof(double));
    if (!s->D || !s->gam) return -2;
    return 0;
}

static void scratch_free(scratch_t* s)
{
    double* rows[] = {s->S, s->psi, s->dpsi, s->Jr, s->Jz, s->M1, s->M2, s->M3,
                      s->M4, s->M5, s->Ez, s->B, s->Q, s->ta, s->tb, s->tc,
                      s->td, s->tx, s->D, s->gam};
    for (size_t q = 0; q < sizeof(rows) / sizeof(rows[0]); ++q) free(rows[q]);
}

/* Add v * hat weights of rho into row. */
static void deposit(const grid_t* g, double* row, double rho, double v)
{
    int j; double t;
    hat(g, rho, &j, &t);
    row[j] += v * (1.0 - t);
    row[j + 1] += v * t;
}

static double gather(const grid_t* g, const double* row, double rho)
{
    int j; double t;
    hat(g, rho, &j, &t);
    return (1.0 - t) * row[j] + t * row[j + 1];
}

/* Transverse Poisson problem for psi, conservative (finite-volume) form:
 *   [r_{j+1/2}^a (psi_{j+1}-psi_j) - r_{j-1/2}^a (psi_j-psi_{j-1})]/(r_j^a h^2)
 *       = S_j - n_ion_j,                     j = 1..N-1
 *   (2+2a)(psi_1 - psi_0)/h^2 = S_0 - n_ion_0,  psi_N = 0. */
static void solve_psi(const grid_t* g, scratch_t* s, const double* nion)
{
    const int N = g->N;
    const double h = g->h, a = g->alpha, h2 = h * h;
    s->ta[0] = 0.0;
    s->tb[0] = -(2.0 + 2.0 * a) / h2;
    s->tc[0] = (2.0 + 2.0 * a) / h2;
    s->td[0] = s->S[0] - nion[0];
    for (int j = 1; j < N; ++j) {
        const double rj = pow(g->rn[j], a);
        const double rm = pow(g->rn[j] - 0.5 * h, a);
        const double rp = pow(g->rn[j] + 0.5 * h, a);
        s->ta[j] = rm / (rj * h2);
        s->tc[j] = rp / (rj * h2);
        s->tb[j] = -(rm + rp) / (rj * h2);
        s->td[j] = s->S[j] - nion[j];
    }
    or_thomas(N, s->ta, s->tb, s->tc, s->td, s->psi);
    s->psi[N] = 0.0;
    /* node derivative psi' */
    s->dpsi[0] = 0.0;
    for (int j = 1; j < N; ++j) s->dpsi[j] = (s->psi[j + 1] - s->psi[j - 1]) / (2.0 * h);
    s->dpsi[N] = (s->psi[N] - s->psi[N - 1]) / h;
}

/* Radial components of the particle state used for deposits. */
typedef struct {
    double rho;    /* folded radius */
    double sw;     /* wall sign */
    double sg;     /* total parity of radial vectors (slab: sign(x) * sw) */
    double r;      /* unfolded radius */
    double pr;     /* physical radial momentum at rho */
    double l2;     /* l_z^2 (cylindrical) */
} radial_t;

static radial_t radial_of(const grid_t* g, double x, double y, double px, double py)
{
    radial_t q;
    q.r = radius_of(g, x, y);
    q.rho = fold_radius(g, q.r, &q.sw);
    if (g->p->geom == OR_CYL) {
        q.sg = q.sw;
        q.pr = q.r > 0.0 ? q.sw * (x * px + y * py) / q.r : 0.0;
        const double l = x * py - y * px;
        q.l2 = l * l;
    } else {
        q.sg = (x < 0.0 ? -1.0 : 1.0) * q.sw;
        q.pr = q.sg * px;
        q.l2 = 0.0;
    }
    return q;
}

static int eval_core_b(const grid_t* g, scratch_t* s, int64_t np,
                       const double* x, const double* y, const double* px, const double* py,
                       const double* d0, const double* w, const double* nion,
                       const double* jb_row, double* fx, double* fy, double* fpx, double* fpy,
                       int64_t* clamps, const double* b_given);

static int eval_core(const grid_t* g, scratch_t* s, int64_t np,
                     const double* x, const double* y, const double* px, const double* py,
                     const double* d0, const double* w, const double* nion,
                     const double* jb_row, double* fx, double* fy, double* fpx, double* fpy,
                     int64_t* clamps)
{
    return eval_core_b(g, s, np, x, y, px, py, d0, w, nion, jb_row, fx, fy, fpx, fpy, clamps, NULL);
}

/* The stage evaluation; with b_given != NULL, B_theta is taken from it
 * instead of the Helmholtz solve of step 7 (the Eq. (6)-direct march). */
static int eval_core_b(const grid_t* g, scratch_t* s, int64_t np,
                       const double* x, const double* y, const double* px, const double* py,
                       const double* d0, const double* w, const double* nion,
                       const double* jb_row, double* fx, double* fy, double* fpx, double* fpy,
                       int64_t* clamps, const double* b_given)
{
    const int N = g->N;
    const double h = g->h, a = g->alpha;
    const or_problem* p = g->p;

    /* 1. flux density S = n (1 - v_z) */
    memset(s->S, 0, sizeof(double) * (N + 1));
    for (int64_t i = 0; i < np; ++i) {
        radial_t q = radial_of(g, x[i], y[i], px[i], py[i]);
        deposit(g, s->S, q.rho, w[i]);
    }
    for (int j = 0; j <= N; ++j) s->S[j] /= g->V[j];

    /* 2. psi and node psi' */
    solve_psi(g, s, nion);

    /* 3-5. gather psi -> D, gamma, p_z (Eqs. (1)-(3)); deposit currents and
     * the moments of d_xi J_r. */
    double* rows[7] = {s->Jr, s->Jz, s->M1, s->M2, s->M3, s->M4, s->M5};
    for (int m = 0; m < 7; ++m) memset(rows[m], 0, sizeof(double) * (N + 1));
    for (int64_t i = 0; i < np; ++i) {
        radial_t q = radial_of(g, x[i], y[i], px[i], py[i]);
        double D = d0[i] + gather(g, s->psi, q.rho);
        if (D < p->d_min) { D = p->d_min; ++*clamps; }
        const double p2 = px[i] * px[i] + py[i] * py[i];
        const double gam = (1.0 + p2 + D * D) / (2.0 * D);
        const double pz = (1.0 + p2 - D * D) / (2.0 * D);
        s->D[i] = D;
        s->gam[i] = gam;
        const double wi = w[i];
        deposit(g, s->Jr, q.rho, -wi * q.pr / D);
        deposit(g, s->Jz, q.rho, -wi * pz / D);
        deposit(g, s->M1, q.rho, wi / D);
        deposit(g, s->M2, q.rho, wi * (gam / (D * D) - q.pr * q.pr / (D * D * D)));
        if (p->geom == OR_CYL && q.rho > 0.0)
            deposit(g, s->M3, q.rho, wi * q.l2 / (D * D * q.rho * q.rho * q.rho));
        deposit(g, s->M4, q.rho, wi * q.pr / (D * D));
        deposit(g, s->M5, q.rho, wi * q.pr * q.pr / (D * D));
    }
    for (int m = 0; m < 7; ++m)
        for (int j = 0; j <= N; ++j) rows[m][j] /= g->V[j];
    for (int j = 0; j <= N; ++j) s->Jz[j] += jb_row[j];

    /* 6. E_z from Eq. (7): d_r E_z = J_r, E_z(r_max) = 0 (trapezoid rule) */
    s->Ez[N] = 0.0;
    for (int j = N - 1; j >= 0; --j) s->Ez[j] = s->Ez[j + 1] - 0.5 * h * (s->Jr[j] + s->Jr[j + 1]);

    /* 7. B_theta: Eq. (6) differentiated in r (Helmholtz form) on nodes
     * 1..N-1, B_0 = 0.  At the wall E_z = 0 for every xi, so Eq. (6) there
     * reads (1/r) d_r (r B) = J_z; it closes the system at node N
     * (discretized at r_{N-1/2}). */
    if (b_given) {
        memcpy(s->B, b_given, sizeof(double) * (N + 1));
        goto derivative;
    }
    const double h2 = h * h;
    for (int j = 1; j < N; ++j) {
        const double rj = g->rn[j];
        const double ra = pow(rj, a);
        s->ta[j - 1] = 1.0 / h2 - a / (2.0 * rj * h);
        s->tb[j - 1] = -2.0 / h2 - a / (rj * rj) - s->M1[j];
        s->tc[j - 1] = 1.0 / h2 + a / (2.0 * rj * h);
        const double m5flux = (pow(g->rn[j + 1], a) * s->M5[j + 1]
                               - pow(g->rn[j - 1], a) * s->M5[j - 1]) / (2.0 * h * ra);
        s->Q[j] = (s->Jz[j + 1] - s->Jz[j - 1]) / (2.0 * h) - s->M2[j] * s->dpsi[j]
                  - a * s->M3[j] + s->M4[j] * s->Ez[j] + m5flux;
        s->td[j - 1] = s->Q[j];
    }
    {
        const double rhalf = pow(g->rn[N] - 0.5 * h, a);
        s->ta[N - 1] = -pow(g->rn[N - 1], a) / (h * rhalf);
        s->tb[N - 1] = pow(g->rn[N], a) / (h * rhalf);
        s->tc[N - 1] = 0.0;
        s->td[N - 1] = 0.5 * (s->Jz[N] + s->Jz[N - 1]);
    }
    s->Q[0] = 0.0;
    s->Q[N] = s->td[N - 1];
    or_thomas(N, s->ta, s->tb, s->tc, s->td, s->tx);
    s->B[0] = 0.0;
    for (int j = 1; j <= N; ++j) s->B[j] = s->tx[j - 1];
derivative:

    /* 8. xi-derivatives of the particle state: Eq. (5) and Eq. (4) (the
     * centrifugal term of Eq. (4) is the polar form of free Cartesian
     * motion). */
    if (fx) {
        for (int64_t i = 0; i < np; ++i) {
            radial_t q = radial_of(g, x[i], y[i], px[i], py[i]);
            const double D = s->D[i];
            const double F = (s->gam[i] / D) * gather(g, s->dpsi, q.rho) - gather(g, s->B, q.rho);
            fx[i] = px[i] / D;
            if (p->geom == OR_CYL) {
                fy[i] = py[i] / D;
                if (q.r > 0.0) {
                    fpx[i] = q.sw * F * x[i] / q.r;
                    fpy[i] = q.sw * F * y[i] / q.r;
                } else {
                    fpx[i] = 0.0;
                    fpy[i] = 0.0;
                }
            } else {
                fy[i] = 0.0;
                fpx[i] = q.sg * F;
                fpy[i] = 0.0;
            }
        }
    }
    return 0;
}

static int64_t count_nonfinite(const double* v, int64_t n)
{
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i) c += !isfinite(v[i]);
    return c;
}

static void store_fields(const grid_t* g, const scratch_t* s, double* psi, double* ez,
                         double* b, double* wfield)
{
    for (int j = 0; j <= g->N; ++j) {
        psi[j] = s->psi[j];
        ez[j] = s->Ez[j];
        b[j] = s->B[j];
        wfield[j] = -s->dpsi[j];   /* E_r - B_theta = -d psi/dr */
    }
}

int or_eval(const or_problem* p, int64_t np,
            const double* x, const double* y, const double* px, const double* py,
            const double* d0, const double* w, const double* nion,
            const double* jb_row, double* f, double* fields, double* mom,
            double* part, int64_t* counters)
{
    if (check_problem(p) || np < 0) return -1;
    grid_t g;
    scratch_t s;
    int rc = grid_init(p, &g);
    if (!rc) rc = scratch_init(&s, g.N, np);
    if (rc) { grid_free(&g); return -2; }
    const int N1 = g.N + 1;
    int64_t clamps = 0;
    double *fx = NULL, *fy = NULL, *fpx = NULL, *fpy = NULL;
    if (f) { fx = f; fy = f + np; fpx = f + 2 * np; fpy = f + 3 * np; }
    eval_core(&g, &s, np, x, y, px, py, d0, w, nion, jb_row, fx, fy, fpx, fpy, &clamps);
    if (fields) store_fields(&g, &s, fields, fields + N1, fields + 2 * N1, fields + 3 * N1);
    if (mom) {
        const double* rows[9] = {s.S, s.Jr, s.Jz, s.M1, s.M2, s.M3, s.M4, s.M5, s.Q};
        for (int m = 0; m < 9; ++m) memcpy(mom + (int64_t)m * N1, rows[m], sizeof(double) * N1);
    }
    if (part) {
        for (int64_t i = 0; i < np; ++i) {
            const double D = s.D[i];
            part[i] = D;
            part[np + i] = s.gam[i];
            const double p2 = px[i] * px[i] + py[i] * py[i];
            part[2 * np + i] = (1.0 + p2 - D * D) / (2.0 * D);
        }
    }
    if (counters) {
        counters[0] = clamps;
        counters[1] = 0;
        counters[2] = count_nonfinite(s.psi, N1) + count_nonfinite(s.Ez, N1) + count_nonfinite(s.B, N1);
    }
    scratch_free(&s);
    grid_free(&g);
    return 0;
}

/* Specular reflection at the outer wall (reading: the paper states no
 * boundary; particles leaving r_max are reflected and counted). */
static int64_t reflect_wall(const grid_t* g, int64_t np, double* x, double* y,
                            double* px, double* py)
{
    const double rmax = g->p->r_max;
    int64_t n = 0;
    for (int64_t i = 0; i < np; ++i) {
        if (g->p->geom == OR_CYL) {
            const double r = sqrt(x[i] * x[i] + y[i] * y[i]);
            if (r > rmax) {
                double rn = 2.0 * rmax - r;
                if (rn < 0.0) rn = 0.0;
                const double ux = x[i] / r, uy = y[i] / r;
                const double pr = ux * px[i] + uy * py[i];
                x[i] = rn * ux;
                y[i] = rn * uy;
                px[i] -= 2.0 * pr * ux;
                py[i] -= 2.0 * pr * uy;
                ++n;
            }
        } else {
            const double ax = fabs(x[i]);
            if (ax > rmax) {
                double xn = 2.0 * rmax - ax;
                if (xn < 0.0) xn = 0.0;
                x[i] = x[i] < 0.0 ? -xn : xn;
                px[i] = -px[i];
                ++n;
            }
        }
    }
    return n;
}

/*
 * Plasma response for a fixed beam current (Section II A: the plasma
 * equations are solved in the r-xi window for a frozen beam).  Reading: Heun
 * (RK2) steps in xi; the fields stored at slice k are those of the state at
 * xi_k; the plasma ahead of the beam (slice 0) is unperturbed.
 */
static int march_impl(const or_problem* p, int64_t np,
                      double* x, double* y, double* px, double* py,
                      const double* d0, const double* w, const double* nion,
                      const double* jb, double* fields, double* diag, int64_t* counters,
                      int32_t stride, double* traj)
{
    if (check_problem(p) || np < 0 || !fields) return -1;
    grid_t g;
    scratch_t s;
    int rc = grid_init(p, &g);
    if (!rc) rc = scratch_init(&s, g.N, np);
    if (rc) { grid_free(&g); return -2; }
    const int N1 = g.N + 1;
    const int64_t plane = (int64_t)p->n_xi * N1;
    const int64_t n4 = np > 0 ? np : 1;
    double* f0 = (double*)malloc(sizeof(double) * 4 * n4);
    double* f1 = (double*)malloc(sizeof(double) * 4 * n4);
    double* ys = (double*)malloc(sizeof(double) * 4 * n4);
    if (!f0 || !f1 || !ys) { free(f0); free(f1); free(ys); scratch_free(&s); grid_free(&g); return -2; }
    int64_t clamps = 0, walls = 0;
    const double dxi = g.dxi;

    const int64_t n_traj = stride > 0 ? (np + stride - 1) / stride : 0;
    for (int k = 0; k < p->n_xi; ++k) {
        /* trajectories: the radius of every stride-th particle at xi_k */
        for (int64_t q = 0; q < n_traj; ++q) {
            const int64_t i = q * stride;
            traj[(int64_t)k * n_traj + q] = radius_of(&g, x[i], y[i]);
        }
        eval_core(&g, &s, np, x, y, px, py, d0, w, nion, jb + (int64_t)k * N1,
                  f0, f0 + n4, f0 + 2 * n4, f0 + 3 * n4, &clamps);
        store_fields(&g, &s, fields + (int64_t)k * N1, fields + plane + (int64_t)k * N1,
                     fields + 2 * plane + (int64_t)k * N1, fields + 3 * plane + (int64_t)k * N1);
        if (diag) {
            memcpy(diag + (int64_t)k * N1, s.S, sizeof(double) * N1);
            memcpy(diag + plane + (int64_t)k * N1, s.Jr, sizeof(double) * N1);
            memcpy(diag + 2 * plane + (int64_t)k * N1, s.Jz, sizeof(double) * N1);
        }
        if (k == p->n_xi - 1) break;
        /* predictor */
        for (int64_t i = 0; i < np; ++i) {
            ys[i] = x[i] + dxi * f0[i];
            ys[n4 + i] = y[i] + dxi * f0[n4 + i];
            ys[2 * n4 + i] = px[i] + dxi * f0[2 * n4 + i];
            ys[3 * n4 + i] = py[i] + dxi * f0[3 * n4 + i];
        }
        eval_core(&g, &s, np, ys, ys + n4, ys + 2 * n4, ys + 3 * n4, d0, w, nion,
                  jb + (int64_t)(k + 1) * N1, f1, f1 + n4, f1 + 2 * n4, f1 + 3 * n4, &clamps);
        /* corrector */
        const double hd = 0.5 * dxi;
        for (int64_t i = 0; i < np; ++i) {
            x[i] = x[i] + hd * (f0[i] + f1[i]);
            y[i] = y[i] + hd * (f0[n4 + i] + f1[n4 + i]);
            px[i] = px[i] + hd * (f0[2 * n4 + i] + f1[2 * n4 + i]);
            py[i] = py[i] + hd * (f0[3 * n4 + i] + f1[3 * n4 + i]);
        }
        walls += reflect_wall(&g, np, x, y, px, py);
    }
    if (counters) {
        counters[0] = clamps;
        counters[1] = walls;
        counters[2] = count_nonfinite(fields, 4 * plane);
    }
    free(f0); free(f1); free(ys);
    scratch_free(&s);
    grid_free(&g);
    return 0;
}

int or_march(const or_problem* p, int64_t np,
             double* x, double* y, double* px, double* py,
             const double* d0, const double* w, const double* nion,
             const double* jb, double* fields, double* diag, int64_t* counters)
{
    return march_impl(p, np, x, y, px, py, d0, w, nion, jb, fields, diag, counters, 0, NULL);
}

int or_march_traj(const or_problem* p, int64_t np,
                  double* x, double* y, double* px, double* py,
                  const double* d0, const double* w, const double* nion,
                  const double* jb, double* fields, int64_t* counters,
                  int32_t stride, double* traj)
{
    if (stride < 1 || !traj) return -1;
    return march_impl(p, np, x, y, px, py, d0, w, nion, jb, fields, NULL, counters, stride, traj);
}

/*
 * B_theta from Eq. (6) as written: (1/r) d_r (r B) = d_xi E_z + J_z, with
 * d_xi E_z = d^2 psi / d xi^2 (Eq. (7) fixes E_z = d_xi psi in the gauge of
 * the psi solve), integrated from the axis by the trapezoid rule:
 * r_j B_j = r_{j-1} B_{j-1} + h/2 (r_{j-1} q_{j-1} + r_j q_j), B_0 = 0
 * (slab: without the r weights).
 */
static void b_direct(const grid_t* g, const double* dez, const double* jz, double* b)
{
    const int N = g->N;
    const double h = g->h;
    b[0] = 0.0;
    if (g->p->geom == OR_CYL) {
        double rb = 0.0;
        for (int j = 1; j <= N; ++j) {
            rb += 0.5 * h * (g->rn[j - 1] * (dez[j - 1] + jz[j - 1]) + g->rn[j] * (dez[j] + jz[j]));
            b[j] = rb / g->rn[j];
        }
    } else {
        for (int j = 1; j <= N; ++j) b[j] = b[j - 1] + 0.5 * h * ((dez[j - 1] + jz[j - 1]) + (dez[j] + jz[j]));
    }
}

/* Workspace of the Eq. (6)-direct march. */
typedef struct {
    const grid_t* g;
    scratch_t* s;
    int64_t np, n4;
    const double *x, *y, *px, *py, *d0, *w, *nion, *jb_k, *jb_n;
    const double *ez_prev, *ez_k, *jz_k;
    double *f0, *f1, *ys, *yn, *dez, *bstar;
    int last;
    int64_t scratch_clamps;
} direct_t;

/* One trial step of slice k with B_k = b: the Heun step from Y_k (stage-2 B
 * at the predicted state from Eq. (6) with the one-sided d_xi E_z), E_z of
 * the stepped state, and the B_k that Eq. (6) gives with
 * d_xi E_z = (E_z,k+1 - E_z,k) / dxi (the last slice: (E_z,k - E_z,k-1) /
 * dxi); written to out.  The stepped state is left in yn. */
static void direct_phi(direct_t* c, const double* b, double* out)
{
    const grid_t* g = c->g;
    scratch_t* s = c->s;
    const int N = g->N;
    const int64_t np = c->np, n4 = c->n4;
    const double dxi = g->dxi, hd = 0.5 * dxi;
    double *f0 = c->f0, *f1 = c->f1, *ys = c->ys, *yn = c->yn;
    eval_core_b(g, s, np, c->x, c->y, c->px, c->py, c->d0, c->w, c->nion, c->jb_k, f0, f0 + n4, f0 + 2 * n4,
                f0 + 3 * n4, &c->scratch_clamps, b);
    for (int64_t i = 0; i < np; ++i) {
        ys[i] = c->x[i] + dxi * f0[i];
        ys[n4 + i] = c->y[i] + dxi * f0[n4 + i];
        ys[2 * n4 + i] = c->px[i] + dxi * f0[2 * n4 + i];
        ys[3 * n4 + i] = c->py[i] + dxi * f0[3 * n4 + i];
    }
    eval_core_b(g, s, np, ys, ys + n4, ys + 2 * n4, ys + 3 * n4, c->d0, c->w, c->nion, c->jb_n, NULL, NULL, NULL,
                NULL, &c->scratch_clamps, b);
    for (int j = 0; j <= N; ++j) c->dez[j] = (s->Ez[j] - c->ez_k[j]) / dxi;
    b_direct(g, c->dez, s->Jz, c->bstar);
    eval_core_b(g, s, np, ys, ys + n4, ys + 2 * n4, ys + 3 * n4, c->d0, c->w, c->nion, c->jb_n, f1, f1 + n4,
                f1 + 2 * n4, f1 + 3 * n4, &c->scratch_clamps, c->bstar);
    for (int64_t i = 0; i < np; ++i) {
        yn[i] = c->x[i] + hd * (f0[i] + f1[i]);
        yn[n4 + i] = c->y[i] + hd * (f0[n4 + i] + f1[n4 + i]);
        yn[2 * n4 + i] = c->px[i] + hd * (f0[2 * n4 + i] + f1[2 * n4 + i]);
        yn[3 * n4 + i] = c->py[i] + hd * (f0[3 * n4 + i] + f1[3 * n4 + i]);
    }
    if (c->last) {
        for (int j = 0; j <= N; ++j) c->dez[j] = (c->ez_k[j] - c->ez_prev[j]) / dxi;
    } else {
        eval_core_b(g, s, np, yn, yn + n4, yn + 2 * n4, yn + 3 * n4, c->d0, c->w, c->nion, c->jb_n, NULL, NULL,
                    NULL, NULL, &c->scratch_clamps, b);
        for (int j = 0; j <= N; ++j) c->dez[j] = (s->Ez[j] - c->ez_k[j]) / dxi;
    }
    b_direct(g, c->dez, c->jz_k, out);
}

/*
 * The plasma response with B_theta from Eq. (6) directly instead of the
 * Helmholtz form.  d_xi E_z at slice k is taken implicitly, (E_z,k+1 -
 * E_z,k) / dxi, and E_z of slice k + 1 depends on B_k through the step, so
 * B_k solves B = Phi(B) with Phi the trial step of direct_phi.
 * * Plain iteration of Phi diverges: a change of B bends the orbits by
 *   B dxi and moves E_z,k+1 by about B dxi r_max, which the difference
 *   divides by dxi, a gain of order r_max for any dxi.  So the fixed point
 *   is found by Newton steps on B - Phi(B) = 0, each solving its linear
 *   system by GMRES (Saad and Schultz 1986) with the Jacobian applied by a
 *   finite difference of Phi: at most `iters` Newton steps, until the
 *   residual is at most tol of max |B|.
 * * The centred difference (E_z,k+1 - E_z,k-1) / (2 dxi) couples alternate
 *   slices and grows an odd-even mode from slice to slice; the one-sided
 *   implicit difference is stable and first order in dxi.
 * Slice 0 (unperturbed plasma ahead of the beam) starts from B = 0.
 * iterations[k] receives the Newton steps used.
 */
#define DIRECT_KRYLOV 40

static double vnorm(const double* v, int n)
{
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) s2 += v[i] * v[i];
    return sqrt(s2);
}

/* Solve (I - J) dx = r with J v = (Phi(b + eps v) - phi_b) / eps by GMRES;
 * V: (m + 1) n, H: (m + 1) m. */
static void direct_gmres(direct_t* c, const double* b, const double* phi_b, const double* r, double* dx, int n,
                         double* V, double* H, double* work, double* tmp)
{
    const int m = DIRECT_KRYLOV;
    double cs[DIRECT_KRYLOV], sn[DIRECT_KRYLOV], gv[DIRECT_KRYLOV + 1], yv[DIRECT_KRYLOV];
    for (int i = 0; i < n; ++i) dx[i] = 0.0;
    const double beta = vnorm(r, n);
    if (beta == 0.0) return;
    for (int i = 0; i < n; ++i) V[i] = r[i] / beta;
    for (int i = 0; i <= m; ++i) gv[i] = 0.0;
    gv[0] = beta;
    const double bn = vnorm(b, n);
    int k_used = 0;
    for (int k = 0; k < m; ++k) {
        double* vk = V + (int64_t)k * n;
        double* w = V + (int64_t)(k + 1) * n;
        /* w = (I - J) v_k */
        const double eps = 1e-7 * (1.0 + bn);
        for (int i = 0; i < n; ++i) tmp[i] = b[i] + eps * vk[i];
        direct_phi(c, tmp, work);
        for (int i = 0; i < n; ++i) w[i] = vk[i] - (work[i] - phi_b[i]) / eps;
        for (int q = 0; q <= k; ++q) {
            const double* vq = V + (int64_t)q * n;
            double hq = 0.0;
            for (int i = 0; i < n; ++i) hq += w[i] * vq[i];
            H[q * m + k] = hq;
            for (int i = 0; i < n; ++i) w[i] -= hq * vq[i];
        }
        const double hn = vnorm(w, n);
        H[(k + 1) * m + k] = hn;
        if (hn > 0.0)
            for (int i = 0; i < n; ++i) w[i] /= hn;
        for (int q = 0; q < k; ++q) {
            const double a0 = H[q * m + k], a1 = H[(q + 1) * m + k];
            H[q * m + k] = cs[q] * a0 + sn[q] * a1;
            H[(q + 1) * m + k] = -sn[q] * a0 + cs[q] * a1;
        }
        const double a0 = H[k * m + k], a1 = H[(k + 1) * m + k];
        const double den = sqrt(a0 * a0 + a1 * a1);
        cs[k] = den > 0.0 ? a0 / den : 1.0;
        sn[k] = den > 0.0 ? a1 / den : 0.0;
        H[k * m + k] = den;
        H[(k + 1) * m + k] = 0.0;
        gv[k + 1] = -sn[k] * gv[k];
        gv[k] = cs[k] * gv[k];
        k_used = k + 1;
        if (fabs(gv[k + 1]) <= 1e-13 * beta || hn == 0.0) break;
    }
    for (int k = k_used - 1; k >= 0; --k) {
        double t = gv[k];
        for (int q = k + 1; q < k_used; ++q) t -= H[k * m + q] * yv[q];
        yv[k] = t / H[k * m + k];
    }
    for (int k = 0; k < k_used; ++k)
        for (int i = 0; i < n; ++i) dx[i] += yv[k] * V[(int64_t)k * n + i];
}

int or_march_direct(const or_problem* p, int64_t np,
                    double* x, double* y, double* px, double* py,
                    const double* d0, const double* w, const double* nion,
                    const double* jb, double* fields, int64_t* counters,
                    int32_t iters, double tol, int32_t* iterations)
{
    if (check_problem(p) || np < 0 || !fields || iters < 1) return -1;
    grid_t g;
    scratch_t s;
    int rc = grid_init(p, &g);
    if (!rc) rc = scratch_init(&s, g.N, np);
    if (rc) { grid_free(&g); return -2; }
    const int N = g.N, N1 = N + 1;
    const int64_t plane = (int64_t)p->n_xi * N1;
    const int64_t n4 = np > 0 ? np : 1;
    const int m = DIRECT_KRYLOV;
    double* f0 = (double*)malloc(sizeof(double) * 4 * n4);
    double* f1 = (double*)malloc(sizeof(double) * 4 * n4);
    double* ys = (double*)malloc(sizeof(double) * 4 * n4);
    double* yn = (double*)malloc(sizeof(double) * 4 * n4);
    double* rows = (double*)malloc(sizeof(double) * 12 * N1);
    double* V = (double*)malloc(sizeof(double) * (m + 1) * N1);
    double* H = (double*)malloc(sizeof(double) * (m + 1) * m);
    if (!f0 || !f1 || !ys || !yn || !rows || !V || !H) {
        free(f0); free(f1); free(ys); free(yn); free(rows); free(V); free(H);
        scratch_free(&s); grid_free(&g);
        return -2;
    }
    double* ez_prev = rows;
    double* ez_k = rows + N1;
    double* jz_k = rows + 2 * N1;
    double* bk = rows + 3 * N1;
    double* phi = rows + 4 * N1;
    double* res = rows + 5 * N1;
    double* dx = rows + 6 * N1;
    double* work = rows + 7 * N1;
    double* tmp = rows + 8 * N1;
    double* dez = rows + 9 * N1;
    double* bstar = rows + 10 * N1;
    double* psi_k = rows + 11 * N1;
    for (int j = 0; j <= N; ++j) { ez_prev[j] = 0.0; bk[j] = 0.0; }
    direct_t c = {&g, &s, np, n4, x, y, px, py, d0, w, nion, NULL, NULL, ez_prev, ez_k, jz_k,
                  f0, f1, ys, yn, dez, bstar, 0, 0};
    int64_t clamps = 0, walls = 0;

    for (int k = 0; k < p->n_xi; ++k) {
        c.jb_k = jb + (int64_t)k * N1;
        c.jb_n = jb + (int64_t)(k + 1 < p->n_xi ? k + 1 : k) * N1;
        c.last = k + 1 >= p->n_xi;
        /* the B-independent fields of slice k */
        eval_core_b(&g, &s, np, x, y, px, py, d0, w, nion, c.jb_k, NULL, NULL, NULL, NULL, &c.scratch_clamps, bk);
        for (int j = 0; j <= N; ++j) {
            ez_k[j] = s.Ez[j];
            jz_k[j] = s.Jz[j];
            psi_k[j] = s.psi[j];
            fields[3 * plane + (int64_t)k * N1 + j] = -s.dpsi[j];
        }
        int it = 0;
        for (;;) {
            direct_phi(&c, bk, phi);
            double rmax = 0.0, bmax = 0.0;
            for (int j = 0; j <= N; ++j) {
                res[j] = phi[j] - bk[j];
                rmax = fmax(rmax, fabs(res[j]));
                bmax = fmax(bmax, fabs(phi[j]));
            }
            if (rmax <= tol * bmax || it >= iters) break;
            ++it;
            direct_gmres(&c, bk, phi, res, dx, N1, V, H, work, tmp);
            for (int j = 0; j <= N; ++j) bk[j] += dx[j];
        }
        if (iterations) iterations[k] = it;
        for (int j = 0; j <= N; ++j) {
            fields[(int64_t)k * N1 + j] = psi_k[j];
            fields[plane + (int64_t)k * N1 + j] = ez_k[j];
            fields[2 * plane + (int64_t)k * N1 + j] = bk[j];
        }
        if (k == p->n_xi - 1) break;
        /* accept the step with the converged B_k (its clamps count) */
        c.scratch_clamps = 0;
        direct_phi(&c, bk, phi);
        clamps += c.scratch_clamps;
        for (int64_t i = 0; i < np; ++i) {
            x[i] = yn[i];
            y[i] = yn[n4 + i];
            px[i] = yn[2 * n4 + i];
            py[i] = yn[3 * n4 + i];
        }
        walls += reflect_wall(&g, np, x, y, px, py);
        for (int j = 0; j <= N; ++j) ez_prev[j] = ez_k[j];
    }
    if (counters) {
        counters[0] = clamps;
        counters[1] = walls;
        counters[2] = count_nonfinite(fields, 4 * plane);
    }
    free(f0); free(f1); free(ys); free(yn); free(rows); free(V); free(H);
    scratch_free(&s);
    grid_free(&g);
    return 0;
}

/*
 * Beam push over n_steps of dt in frozen fields: Eqs. (8)-(11) for electrons
 * (q_b = -1), written with E = (E_r x/r, E_r y/r, E_z), B = B_theta e_theta,
 * E_r = W + B_theta and advanced with the Boris rotation (published method,
 * Boris 1970).  dxi_b/dt = 1 - v_z = (1 + p_perp^2)/(gamma (gamma + p_z)),
 * the cancellation-free form of Eq. (11).  Fields are bilinear in (r, xi).
 */
int or_beam_push(const or_problem* p, int64_t n_beam,
                 double* bx, double* by, double* bpx, double* bpy, double* bpz,
                 double* bxi, const double* fields, int32_t n_steps, double dt,
                 int64_t* n_out)
{
    if (check_problem(p) || n_steps < 0) return -1;
    grid_t g;
    if (grid_init(p, &g)) { grid_free(&g); return -2; }
    const int N1 = g.N + 1;
    const int64_t plane = (int64_t)p->n_xi * N1;
    const double* fez = fields + plane;
    const double* fb = fields + 2 * plane;
    const double* fw = fields + 3 * plane;
    int64_t out = 0;
    const double qh = -0.5 * dt;   /* q dt / 2 with q = -1 */
    for (int64_t i = 0; i < n_beam; ++i) {
        for (int st = 0; st < n_steps; ++st) {
            const double x = bx[i], y = by[i], xi = bxi[i];
            const double r = radius_of(&g, x, y);
            double ez = 0.0, bt = 0.0, wv = 0.0;
            if (r <= p->r_max && xi >= p->xi_min && xi < p->xi_max) {
                int j; double tr;
                hat(&g, r, &j, &tr);
                const double u = (xi - p->xi_min) / g.dxi;
                int k = (int)floor(u);
                if (k > p->n_xi - 1) k = p->n_xi - 1;
                const double tk = u - k;
                const int k1 = (k + 1 < p->n_xi) ? k + 1 : k;
                const double tk1 = (k + 1 < p->n_xi) ? tk : 0.0;
                const double w00 = (1.0 - tr) * (1.0 - tk1), w01 = tr * (1.0 - tk1);
                const double w10 = (1.0 - tr) * tk1, w11 = tr * tk1;
                const int64_t o0 = (int64_t)k * N1 + j, o1 = (int64_t)k1 * N1 + j;
                ez = w00 * fez[o0] + w01 * fez[o0 + 1] + w10 * fez[o1] + w11 * fez[o1 + 1];
                bt = w00 * fb[o0] + w01 * fb[o0 + 1] + w10 * fb[o1] + w11 * fb[o1 + 1];
                wv = w00 * fw[o0] + w01 * fw[o0 + 1] + w10 * fw[o1] + w11 * fw[o1 + 1];
            } else {
                ++out;
            }
            const double er = wv + bt;
            double ux, uy;
            if (p->geom == OR_CYL) {
                ux = r > 0.0 ? x / r : 0.0;
                uy = r > 0.0 ? y / r : 0.0;
            } else {
                ux = x < 0.0 ? -1.0 : 1.0;
                uy = 0.0;
            }
            const double Ex = er * ux, Ey = er * uy, Ez = ez;
            const double Bx = -bt * uy, By = bt * ux, Bz = 0.0;
            /* half electric kick */
            double mx = bpx[i] + qh * Ex, my = bpy[i] + qh * Ey, mz = bpz[i] + qh * Ez;
            const double gm = sqrt(1.0 + mx * mx + my * my + mz * mz);
            /* magnetic rotation */
            const double tx = qh * Bx / gm, ty = qh * By / gm, tz = qh * Bz / gm;
            const double t2 = tx * tx + ty * ty + tz * tz;
            const double qx = mx + (my * tz - mz * ty);
            const double qy = my + (mz * tx - mx * tz);
            const double qz = mz + (mx * ty - my * tx);
            const double sx = 2.0 * tx / (1.0 + t2), sy = 2.0 * ty / (1.0 + t2), sz = 2.0 * tz / (1.0 + t2);
            const double nx = mx + (qy * sz - qz * sy);
            const double ny = my + (qz * sx - qx * sz);
            const double nz = mz + (qx * sy - qy * sx);
            /* half electric kick */
            bpx[i] = nx + qh * Ex;
            bpy[i] = ny + qh * Ey;
            bpz[i] = nz + qh * Ez;
            const double pp2 = bpx[i] * bpx[i] + bpy[i] * bpy[i];
            const double gam = sqrt(1.0 + pp2 + bpz[i] * bpz[i]);
            bx[i] = x + dt * bpx[i] / gam;
            by[i] = y + dt * bpy[i] / gam;
            bxi[i] = xi + dt * (1.0 + pp2) / (gam * (gam + bpz[i]));
        }
    }
    if (n_out) *n_out = out;
    grid_free(&g);
    return 0;
}

double or_mean_gain(int64_t n_beam, const int32_t* tag, int32_t which,
                    const double* bw, const double* gamma_before,
                    const double* bpx, const double* bpy, const double* bpz)
{
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < n_beam; ++i) {
        if (tag[i] != which) continue;
        const double gam = sqrt(1.0 + bpx[i] * bpx[i] + bpy[i] * bpy[i] + bpz[i] * bpz[i]);
        num += bw[i] * (gam - gamma_before[i]);
        den += bw[i];
    }
    return den > 0.0 ? num / den : 0.0;
}

/*
 * Energy spectrum (Section III, witness spectra): counts of the gain
 * gamma - gamma_init in n_bins equal bins of [lo, hi), with [0] below lo and
 * [n_bins + 1] at or above hi.  Bin k holds lo + k (hi - lo)/n_bins <= gain <
 * lo + (k + 1)(hi - lo)/n_bins, decided as floor(n_bins (gain - lo)/(hi - lo)).
 */
int or_gain_histogram(int64_t n_beam, const int32_t* tag, int32_t which,
                      const double* bpx, const double* bpy, const double* bpz,
                      const double* gamma_before, int32_t n_bins, double lo, double hi,
                      uint64_t* hist)
{
    if (n_bins < 1 || !(hi > lo) || !hist) return -1;
    for (int32_t q = 0; q < n_bins + 2; ++q) hist[q] = 0;
    for (int64_t i = 0; i < n_beam; ++i) {
        if (which >= 0 && tag[i] != which) continue;
        const double px2 = bpx[i] * bpx[i], py2 = bpy[i] * bpy[i], pz2 = bpz[i] * bpz[i];
        const double gain = sqrt(((1.0 + px2) + py2) + pz2) - gamma_before[i];
        if (!(gain >= lo)) {
            ++hist[0];
        } else if (gain >= hi) {
            ++hist[n_bins + 1];
        } else {
            int k = (int)floor((gain - lo) / (hi - lo) * (double)n_bins);
            if (k < 0) k = 0;
            if (k > n_bins - 1) k = n_bins - 1;
            ++hist[1 + k];
        }
    }
    return 0;
}

double or_ez_peak(const or_problem* p, const double* fields, double xi_from)
{
    const int N1 = p->n_r + 1;
    const int64_t plane = (int64_t)p->n_xi * N1;
    const double dxi = (p->xi_max - p->xi_min) / p->n_xi;
    double m = 0.0;
    int first = 1;
    for (int k = 0; k < p->n_xi; ++k) {
        const double xi = p->xi_min + k * dxi;
        if (xi < xi_from) continue;
        const double v = fields[plane + (int64_t)k * N1];
        if (first || v < m) { m = v; first = 0; }
    }
    return m;
}
