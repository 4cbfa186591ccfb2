/*
 * Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle: every entry point on small cylindrical and slab problems (cold and
 * warm plasma, macroparticle beam, a driver strong enough to reach the wall
 * and the D floor), so that an out-of-bounds index, a use of freed scratch or
 * an undefined operation anywhere in the oracle ends the run with an error.
 * Exits 0 when every call returned its success code.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "wake_oracle.h"

static double normal(unsigned* s)
{
    /* Box-Muller on a small LCG: the values only need to be finite and spread */
    *s = *s * 1664525u + 1013904223u;
    const double u1 = ((*s >> 8) + 1.0) / 16777217.0;
    *s = *s * 1664525u + 1013904223u;
    const double u2 = (*s >> 8) / 16777216.0;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * 3.141592653589793 * u2);
}

static int run(int geom, double u_th, double n_peak, int ppc)
{
    or_problem p;
    memset(&p, 0, sizeof(p));
    p.geom = geom;
    p.n_r = 24;
    p.r_max = 3.0;
    p.n_xi = 40;
    p.xi_min = 0.0;
    p.xi_max = 8.0;
    p.ppc = ppc;
    p.u_th = u_th;
    p.n0 = 1.0;
    p.sigma_r = 0.3;
    p.n_bunch = 2;
    p.n_peak[0] = n_peak;
    p.n_peak[1] = 0.3 * n_peak;
    p.sigma_z[0] = 0.7;
    p.sigma_z[1] = 0.5;
    p.xi_c[0] = 2.0;
    p.xi_c[1] = 6.0;
    p.d_min = 0.05;
    const int64_t np = or_plasma_count(&p);
    const int N1 = p.n_r + 1;
    if (np <= 0) return 1;
    unsigned seed = 12345u + (unsigned)geom * 7u + (unsigned)ppc;
    double* eps = malloc(sizeof(double) * 3 * (size_t)np);
    for (int64_t i = 0; i < 3 * np; ++i) eps[i] = normal(&seed);
    double *x = malloc(sizeof(double) * np), *y = malloc(sizeof(double) * np);
    double *px = malloc(sizeof(double) * np), *py = malloc(sizeof(double) * np);
    double *d0 = malloc(sizeof(double) * np), *w = malloc(sizeof(double) * np);
    double* nion = malloc(sizeof(double) * N1);
    double* jb = malloc(sizeof(double) * (size_t)p.n_xi * N1);
    double* fields = malloc(sizeof(double) * 4 * (size_t)p.n_xi * N1);
    double* diag = malloc(sizeof(double) * 3 * (size_t)p.n_xi * N1);
    int64_t cnt[3] = {0, 0, 0};
    int rc = 0;
    rc |= or_load_plasma(&p, u_th > 0.0 ? eps : NULL, x, y, px, py, d0, w, nion);

    /* one stage evaluation, every output */
    double* f = malloc(sizeof(double) * 4 * np);
    double* fr = malloc(sizeof(double) * 4 * N1);
    double* mom = malloc(sizeof(double) * 9 * N1);
    double* part = malloc(sizeof(double) * 3 * np);
    rc |= or_beam_current_analytic(&p, jb);
    rc |= or_eval(&p, np, x, y, px, py, d0, w, nion, jb + 10 * N1, f, fr, mom, part, cnt);

    /* macroparticle beam, its current, the march, the push and the diagnostics */
    const int64_t nb = 600, nd = 400;
    double* beps = malloc(sizeof(double) * 4 * nb);
    for (int64_t i = 0; i < 4 * nb; ++i) {
        double v = normal(&seed);
        beps[i] = v > 3.0 ? 3.0 : (v < -3.0 ? -3.0 : v);
    }
    double *bx = malloc(sizeof(double) * nb), *by = malloc(sizeof(double) * nb);
    double *bpx = malloc(sizeof(double) * nb), *bpy = malloc(sizeof(double) * nb);
    double *bpz = malloc(sizeof(double) * nb), *bxi = malloc(sizeof(double) * nb);
    double *bw = malloc(sizeof(double) * nb), *g0 = malloc(sizeof(double) * nb);
    int32_t* tag = malloc(sizeof(int32_t) * nb);
    int64_t nout = 0;
    rc |= or_load_beam(&p, nb, nd, 4.0e4, 1e-3, beps, bx, by, bpx, bpy, bpz, bxi, bw, tag);
    for (int64_t i = 0; i < nb; ++i) g0[i] = sqrt(1.0 + bpx[i] * bpx[i] + bpy[i] * bpy[i] + bpz[i] * bpz[i]);
    rc |= or_beam_current_macro(&p, nb, bx, by, bxi, bw, jb, &nout);
    rc |= or_march(&p, np, x, y, px, py, d0, w, nion, jb, fields, diag, cnt);
    rc |= or_beam_push(&p, nb, bx, by, bpx, bpy, bpz, bxi, fields, 5, 40.0, &nout);
    const double gain = or_mean_gain(nb, tag, 1, bw, g0, bpx, bpy, bpz);
    const double peak = or_ez_peak(&p, fields, 3.0);
    if (!isfinite(gain) || !isfinite(peak)) rc |= 1;
    printf("geom %d u_th %g n_peak %g ppc %d: clamps %lld walls %lld nonfinite %lld gain %.6g peak %.6g rc %d\n",
           geom, u_th, n_peak, ppc, (long long)cnt[0], (long long)cnt[1], (long long)cnt[2], gain, peak, rc);

    free(eps); free(x); free(y); free(px); free(py); free(d0); free(w); free(nion); free(jb);
    free(fields); free(diag); free(f); free(fr); free(mom); free(part); free(beps);
    free(bx); free(by); free(bpx); free(bpy); free(bpz); free(bxi); free(bw); free(g0); free(tag);
    return rc;
}

int main(void)
{
    /* Thomas on a small diagonally dominant system */
    double a[5] = {0, 1, 1, 1, 1}, b[5] = {4, 4, 4, 4, 4}, c[5] = {1, 1, 1, 1, 0}, d[5] = {1, 2, 3, 4, 5}, xs[5];
    int rc = or_thomas(5, a, b, c, d, xs);
    rc |= run(OR_CYL, 0.0, 0.5, 2);
    rc |= run(OR_CYL, 0.05, 8.0, 4);
    rc |= run(OR_SLAB, 0.02, 8.0, 4);
    rc |= run(OR_CYL, 0.0, 60.0, 2);   /* strong driver: wall reflections and D floor */
    return rc != 0;
}
