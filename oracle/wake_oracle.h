/*
 * Serial FP64 CPU oracle for the quasi-static plasma response of
 * Jain, Palastro, Antonsen, Mori and An, "Plasma wakefield acceleration
 * studies using the quasi-static code WAKE" (arXiv:1411.3246), Section II.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or constant with
 * the HIP library.
 *
 * Units: lengths in k_p^-1, time in omega_p^-1, momenta in m_e c, potentials
 * in m_e c^2/e, fields in m_e c omega_p/e, densities in n_p, currents in
 * e n_p c.  Plasma electrons have charge q = -1; ions are an immobile
 * background.  xi = c t - z grows from the head of the beam backwards.
 */
#ifndef WAKE_ORACLE_H
#define WAKE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_CYL = 0, OR_SLAB = 1 };

typedef struct {
    int32_t geom;        /* OR_CYL (r-xi) or OR_SLAB (x-xi, half domain x>=0) */
    int32_t n_r;         /* radial cells; nodes j = 0..n_r                   */
    double  r_max;       /* outer radius (x_max in slab)                     */
    int32_t n_xi;        /* stored slices k = 0..n_xi-1                      */
    double  xi_min, xi_max;
    int32_t ppc;         /* plasma macroparticles per radial cell            */
    double  u_th;        /* thermal momentum spread per component (0: cold)  */
    double  n0;          /* plasma density (1 in normalized units)           */
    double  sigma_r;     /* common radial rms size of both bunches, Eq. (12) */
    int32_t n_bunch;     /* 1: single bunch, 2: drive + witness              */
    double  n_peak[2];   /* peak densities n_d, n_w                          */
    double  sigma_z[2];  /* rms lengths sigma_zd, sigma_zw                   */
    double  xi_c[2];     /* centres xi_d, xi_w                               */
    double  d_min;       /* floor applied to D = gamma - p_z                 */
} or_problem;

/* Number of plasma macroparticles in one slice (n_r * ppc). */
int64_t or_plasma_count(const or_problem* p);

/* Warm or cold plasma loader.  eps: 3 standard normals per particle pair
 * (n_r*ppc/2 pairs), ignored when u_th == 0.  Outputs have or_plasma_count
 * entries (nion has n_r+1).  Returns 0 or a negative error code. */
int or_load_plasma(const or_problem* p, const double* eps,
                   double* x, double* y, double* px, double* py,
                   double* d0, double* w, double* nion);

/* Beam current J_bz on the nodes from the analytic density of Eq. (12):
 * jb[k*(n_r+1)+j] = -n_b(r_j, xi_k). */
int or_beam_current_analytic(const or_problem* p, double* jb);

/* Macroparticle beam loader (Eq. (12) sampled with the given draws).
 * eps: 4 truncated standard normals per particle (x, y, xi, energy).
 * Particles [0, n_drive) belong to bunch 0, the rest to bunch 1. */
int or_load_beam(const or_problem* p, int64_t n_beam, int64_t n_drive,
                 double gamma0, double rel_spread, const double* eps,
                 double* bx, double* by, double* bpx, double* bpy, double* bpz,
                 double* bxi, double* bw, int32_t* tag);

/* J_bz from macroparticles (bilinear in r and xi). n_out counts particles
 * outside the window. */
int or_beam_current_macro(const or_problem* p, int64_t n_beam,
                          const double* bx, const double* by, const double* bxi,
                          const double* bw, double* jb, int64_t* n_out);

/* One field evaluation for a given particle state at one slice (the stage
 * evaluation of the xi integrator).  Any output pointer may be NULL.
 *   f      : 4*np   (dx, dy, dpx, dpy per unit xi; blocks of np)
 *   fields : 4*(n_r+1)  psi, E_z, B_theta, W = E_r - B_theta
 *   mom    : 9*(n_r+1)  S, J_r, J_z(plasma+beam), M1..M5, Q
 *   part   : 3*np   D, gamma, p_z
 * counters: [0] D clamps, [1] wall reflections (unused here), [2] nonfinite. */
int or_eval(const or_problem* p, int64_t np,
            const double* x, const double* y, const double* px, const double* py,
            const double* d0, const double* w, const double* nion,
            const double* jb_row, double* f, double* fields, double* mom,
            double* part, int64_t* counters);

/* Full plasma response: xi march over all slices with Heun (RK2) steps.
 * The particle state (x, y, px, py) is advanced in place to the last slice.
 *   fields : 4*n_xi*(n_r+1)  [psi | E_z | B_theta | W], slice-major rows
 *   diag   : NULL or 3*n_xi*(n_r+1)  [S | J_r | J_z] of each stored slice
 *   counters (>= 3 entries): D clamps, wall reflections, nonfinite values. */
int or_march(const or_problem* p, int64_t np,
             double* x, double* y, double* px, double* py,
             const double* d0, const double* w, const double* nion,
             const double* jb, double* fields, double* diag, int64_t* counters);

/* or_march that also records, at every slice k (before its fields are
 * computed), the radius of particles 0, stride, 2 stride, ...:
 * traj[k * n_traj + q], n_traj = ceil(np / stride). */
int or_march_traj(const or_problem* p, int64_t np,
                  double* x, double* y, double* px, double* py,
                  const double* d0, const double* w, const double* nion,
                  const double* jb, double* fields, int64_t* counters,
                  int32_t stride, double* traj);

/* The plasma response with B_theta from Eq. (6) directly,
 * (1/r) d_r (r B) = d_xi E_z + J_z, with d_xi E_z = d^2 psi / d xi^2 taken
 * implicitly, (E_z,k+1 - E_z,k) / dxi, and solved per slice by Newton steps
 * (GMRES for each; at most iters steps, until the residual is at most tol of
 * max |B|).  First order in dxi.  Same outputs as or_march (no diag);
 * iterations (n_xi entries, may be NULL) receives the Newton steps used. */
int or_march_direct(const or_problem* p, int64_t np,
                    double* x, double* y, double* px, double* py,
                    const double* d0, const double* w, const double* nion,
                    const double* jb, double* fields, int64_t* counters,
                    int32_t iters, double tol, int32_t* iterations);

/* Beam advance in time with frozen fields, Eqs. (8)-(11), Boris rotation.
 * n_out counts particle-steps that sampled no field (outside the window). */
int or_beam_push(const or_problem* p, int64_t n_beam,
                 double* bx, double* by, double* bpx, double* bpy, double* bpz,
                 double* bxi, const double* fields, int32_t n_steps, double dt,
                 int64_t* n_out);

/* Charge-weighted mean energy gain of particles with tag == which. */
double or_mean_gain(int64_t n_beam, const int32_t* tag, int32_t which,
                    const double* bw, const double* gamma_before,
                    const double* bpx, const double* bpy, const double* bpz);

/* Counts of gamma - gamma_before (tag == which; all if which < 0) in n_bins
 * equal bins of [lo, hi); hist has n_bins + 2 entries: [0] below lo,
 * [n_bins + 1] at or above hi. */
int or_gain_histogram(int64_t n_beam, const int32_t* tag, int32_t which,
                      const double* bpx, const double* bpy, const double* bpz,
                      const double* gamma_before, int32_t n_bins, double lo, double hi,
                      uint64_t* hist);

/* Most negative on-axis E_z over slices with xi_k >= xi_from. */
double or_ez_peak(const or_problem* p, const double* fields, double xi_from);

/* Plain Thomas algorithm for a tridiagonal system (a: sub, b: diag, c: super). */
int or_thomas(int64_t n, const double* a, const double* b, const double* c,
              const double* d, double* x);

#ifdef __cplusplus
}
#endif
#endif
