/*
 * wake.h -- C ABI of the MI355X (gfx950) quasi-static plasma-response library.
 *
 * The library computes the hot path of the quasi-static method of
 * Jain, Palastro, Antonsen, Mori and An, "Plasma wakefield acceleration
 * studies using the quasi-static code WAKE" (arXiv:1411.3246):
 *   - the plasma response to a frozen beam, marched slice by slice in
 *     xi = c t - z over an r-xi (cylindrical) or x-xi (slab) grid
 *     (Section II A, Eqs. (1)-(7));
 *   - the beam current from Eq. (12) or from beam macroparticles;
 *   - the beam advance over the long time step in the frozen fields
 *     (Section II A, Eqs. (8)-(11); plasma first, then beam).
 *
 * Units are normalized: lengths k_p^-1, time omega_p^-1, momenta m_e c,
 * potentials m_e c^2/e, fields m_e c omega_p/e, densities n_p, currents
 * e n_p c.  Plasma and beam particles are electrons (q = -1).
 *
 * Conventions for every call:
 *   - All buffers are caller-owned.  Pointers named d_* are device pointers
 *     (HIP device memory on the current device); h_* are host pointers.
 *     The library never allocates or frees device memory; its one static
 *     device array (see wk_plasma_response_noalloc) comes with its code.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Work is enqueued asynchronously; argument errors are reported
 *     synchronously by the return value, device-side numeric events through
 *     the caller's counter array (see wk_counter_index).
 *   - A plan is host-only, immutable after creation and may be shared by
 *     calls on different streams; it is not thread-safe to destroy while in
 *     use.
 *   - Layouts are structure-of-arrays.  Node arrays have n_r + 1 entries
 *     (node j at r_j = j r_max / n_r); slice-node arrays are slice-major
 *     [n_xi][n_r + 1] (slice k at xi_k = xi_min + k (xi_max - xi_min)/n_xi).
 *   - "real" below means double for WK_FP64 plans and float for WK_MIXED
 *     plans.
 */
#ifndef WAKE_H
#define WAKE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WK_OK = 0,
    WK_ERR_INVALID_ARG = -1,   /* bad problem field, size or null pointer */
    WK_ERR_UNSUPPORTED = -2,   /* valid but outside what this build handles */
    WK_ERR_BUFFER = -3,        /* misaligned or missing buffer */
    WK_ERR_HIP = -4,           /* a HIP runtime call failed */
    WK_ERR_NUMERIC = -5        /* non-finite field values were produced */
} wk_status;

typedef enum { WK_CYL = 0, WK_SLAB = 1 } wk_geom;
/* WK_FP64: every operation in double.  WK_MIXED: per-particle arithmetic in
 * float; particle positions and momenta, deposit accumulation, the radial
 * field solves and the xi integration stay double. */
typedef enum { WK_FP64 = 0, WK_MIXED = 1 } wk_prec;

/* One Gaussian bunch of Eq. (12): peak density (units of n_p), rms length
 * sigma_z and centre xi_c (both in k_p^-1). */
typedef struct {
    double n_peak;
    double sigma_z;
    double xi_c;
} wk_bunch;

/* The problem statement of Section II: uniform plasma of density n0 and
 * thermal momentum spread u_th (per component, units of m_e c); an r-xi
 * window [0, r_max] x [xi_min, xi_max) with n_r cells and n_xi slices;
 * ppc ring macroparticles per radial cell (even when u_th > 0: mirrored
 * pairs); the two-bunch beam of Eq. (12) with common radial size sigma_r
 * (n_bunch = 1 gives the single-bunch driver, n_w = 0).  With n_beam > 0 the
 * beam is represented by macroparticles (first n_drive in bunch 0), energy
 * gamma0 (1 + rel_spread eps), zero emittance.  d_min floors D = gamma - p_z
 * (Eqs. (2)-(3)); floored evaluations are counted. */
typedef struct {
    int32_t geom;          /* wk_geom */
    int32_t n_r;           /* radial cells, 2 .. 2048 */
    double r_max;
    int32_t n_xi;          /* slices, >= 1 */
    double xi_min, xi_max;
    int32_t ppc;           /* macroparticles per cell, 1 .. 128 */
    double u_th;           /* >= 0 */
    double n0;             /* plasma density (1 in normalized units) */
    double sigma_r;
    int32_t n_bunch;       /* 0, 1 or 2 */
    wk_bunch bunch[2];
    int64_t n_beam;        /* beam macroparticles (0: analytic Eq. (12) current) */
    int64_t n_drive;       /* macroparticles of bunch 0 */
    double gamma0, rel_spread;
    int32_t prec;          /* wk_prec */
    double d_min;          /* > 0 */
} wk_problem;

typedef struct wk_plan wk_plan;

/* Byte sizes of every caller buffer of a plan (all multiples of 256). */
typedef struct {
    int64_t n_plasma;         /* plasma macroparticles in one slice = n_r * ppc */
    int64_t n_nodes;          /* n_r + 1 */
    size_t plasma_state;      /* one of x, y, px, py: n_plasma doubles */
    size_t plasma_const;      /* one of d0, w: n_plasma reals */
    size_t plasma_draws;      /* 3 doubles per particle pair */
    size_t nion;              /* n_nodes doubles */
    size_t beam_current;      /* n_xi * n_nodes doubles */
    size_t fields;            /* 4 * n_xi * n_nodes reals: psi, E_z, B_theta, W */
    size_t beam_state;        /* one of x, y, px, py, pz, xi, w, gamma_init: n_beam doubles */
    size_t beam_tag;          /* n_beam int32 */
    size_t beam_draws;        /* 4 doubles per beam macroparticle */
    size_t workspace;         /* scratch for wk_plasma_response / beam calls */
    size_t counters;          /* WK_NCOUNTERS uint64 */
} wk_sizes;

/* Plasma macroparticles of one slice: transverse Cartesian position and
 * momentum of each ring's electron (cylindrical: ring radius |(x, y)|;
 * slab: x, with py the conserved canonical momentum p_y, y unused), the
 * invariant D0 = gamma0 - p_z0 of Eq. (1), the flux weight w, and the ion
 * density n_ion on the nodes. */
typedef struct {
    double* d_x;
    double* d_y;
    double* d_px;
    double* d_py;
    void* d_d0;     /* real[n_plasma] */
    void* d_w;      /* real[n_plasma] */
    double* d_nion; /* double[n_nodes] */
} wk_plasma_bufs;

/* Beam macroparticles (lab-frame transverse position, momentum, xi, charge
 * weight, initial gamma for gain diagnostics, bunch tag 0/1). */
typedef struct {
    double* d_x;
    double* d_y;
    double* d_px;
    double* d_py;
    double* d_pz;
    double* d_xi;
    double* d_w;
    double* d_gamma_init;
    int32_t* d_tag;
} wk_beam_bufs;

enum wk_counter_index {
    WK_CNT_D_CLAMP = 0,        /* stage evaluations with D floored to d_min */
    WK_CNT_WALL = 1,           /* plasma reflections at r_max */
    WK_CNT_NONFINITE = 2,      /* non-finite stored field values */
    WK_CNT_BEAM_OUT_DEPOSIT = 3,  /* beam particles outside the window (deposit) */
    WK_CNT_BEAM_OUT_PUSH = 4,  /* beam particle-steps outside the window (push) */
    WK_CNT_BEAM_BIN = 5,       /* beam particles that left their xi bin */
    WK_CNT_PIPELINE_ABORT = 6, /* nonzero: a wait between workgroups gave up (results invalid) */
    WK_CNT_BEAM_ORDER = 7,     /* nonzero: a pipelined cycle lost beam particles from its xi bins
                                  (results invalid) */
    WK_NCOUNTERS = 8
};

const char* wk_version(void);
const char* wk_status_string(wk_status s);

/* Validate a problem and create a host-only plan (no device work, no
 * allocation on the device).  The plan also holds the launch shape chosen
 * for this problem size.  Returns WK_ERR_INVALID_ARG with a message in
 * wk_last_error() when a field is out of range. */
wk_status wk_plan_create(const wk_problem* problem, wk_plan** out);
void wk_plan_destroy(wk_plan* plan);
wk_status wk_plan_sizes(const wk_plan* plan, wk_sizes* out);
/* Message of the last failed call on this thread ("" if none). */
const char* wk_last_error(void);

/* Zero a caller counter array (WK_NCOUNTERS uint64 on the device) with a
 * kernel (safe under stream capture). */
wk_status wk_counters_zero(uint64_t* d_counters, void* stream);

/* Copy the counter array to h_out (WK_NCOUNTERS uint64, host memory),
 * waiting for `stream`.  Returns WK_ERR_NUMERIC when non-finite field values
 * were stored, a wait between workgroups gave up or a pipelined cycle lost
 * beam particles from its bins (the results are then invalid), WK_OK
 * otherwise; the other counters are informational. */
wk_status wk_counters_read(const uint64_t* d_counters, uint64_t* h_out, void* stream);

/* Plasma loader: ring macroparticles at cell-uniform radii; with u_th > 0,
 * mirrored pairs with momenta u_th * draws (d_draws: 3 standard normals per
 * pair, pair q = cell * ppc/2 + sub-radius) and flux weights a D0/gamma0;
 * n_ion = deposit of the initial areas (Section II A, Eq. (1) and the
 * thermal loading it implies).  d_draws may be NULL when u_th == 0. */
wk_status wk_init_plasma(const wk_plan* plan, const wk_plasma_bufs* plasma,
                         const double* d_draws, void* stream);

/* Beam loader: macroparticles sampling Eq. (12) from d_draws (4 standard
 * normals per particle: x, y, xi, energy), charge weight Q_bunch / N_bunch. */
wk_status wk_init_beam(const wk_plan* plan, const wk_beam_bufs* beam,
                       const double* d_draws, void* stream);

/* Beam current, analytic: J_bz = -n_b(r_j, xi_k) from Eq. (12) (fixed beam). */
wk_status wk_beam_current_analytic(const wk_plan* plan, double* d_jb, void* stream);

/* Beam current, macroparticles: J_bz = -sum W hat_j(r) hat_k(xi) / (V_j dxi) with
 * v_z = c (Section II A: the total current includes the beam current).
 * Uses the workspace for the xi binning of the beam; counts particles
 * outside the window.  The result depends on the beam alone: each xi cell's
 * particles are summed in index order, so repeated calls give the same rows
 * bit for bit. */
wk_status wk_beam_current(const wk_plan* plan, const wk_beam_bufs* beam, double* d_jb,
                          void* d_workspace, uint64_t* d_counters, void* stream);

/* One plasma response.  Marches the plasma state of `plasma` from
 * slice 0 (unperturbed, as loaded) to slice n_xi - 1 with Heun steps,
 * solving psi, E_z and B_theta on every slice and storing
 * d_fields = real[4][n_xi][n_nodes] = psi, E_z, B_theta, W = E_r - B_theta.
 * d_jb: double[n_xi][n_nodes] beam current.  The plasma state is advanced in
 * place (load it again before the next response).  Beyond about 1070
 * cells the march keeps its field and solver rows in the plan workspace. */
wk_status wk_plasma_response(const wk_plan* plan, const wk_plasma_bufs* plasma,
                             const double* d_jb, void* d_fields, void* d_workspace,
                             uint64_t* d_counters, void* stream);

/* wk_plasma_response that also records plasma electron trajectories (the
 * particle radius r = |(x, y)|, slab |x|, of every stride-th macroparticle,
 * i = 0, stride, 2 stride, ... of the loaded order, at every slice k: the
 * state the slice's fields are computed from), for the discussion of the
 * trajectories behind the driver in Section III.  FP64 plans only
 * (WK_ERR_UNSUPPORTED otherwise).  d_traj: double[n_xi][ceil(n_plasma /
 * stride)], written entirely; the other arguments as for wk_plasma_response. */
wk_status wk_plasma_response_traj(const wk_plan* plan, const wk_plasma_bufs* plasma,
                                  const double* d_jb, void* d_fields, void* d_workspace,
                                  int32_t stride, double* d_traj, uint64_t* d_counters,
                                  void* stream);

/* The plasma response with B_theta from Eq. (6) as written, (1/r) d_r (r B)
 * = d_xi E_z + J_z (slab: d_x B = d_xi E_z + J_z), integrated from the axis
 * by the trapezoid rule, instead of its Helmholtz form: the cross-check of
 * that reading (Section II A, Eqs. (6)-(7)).  d_xi E_z at slice k is the
 * implicit one-sided (E_z,k+1 - E_z,k) / dxi (the last slice: the backward
 * difference), and E_z,k+1 depends on B_k through the Heun step, so B_k is
 * found by at most `iters` (1..64) Newton steps per slice on the fixed point
 * of that step, each solved by GMRES (at most 40 Krylov vectors) with a
 * finite-difference Jacobian, until max |Phi(B) - B| <= tol max |Phi(B)|
 * (tol > 0).  First order in dxi.  FP64 plans, n_r up to 512 (its rows are
 * kept in LDS), one workgroup per call (WK_ERR_UNSUPPORTED otherwise).
 * d_workspace: wk_direct_workspace_size(plan) bytes, 8-byte aligned.
 * d_iterations: optional int32[n_xi] of Newton steps used per slice.  The
 * other arguments as for wk_plasma_response. */
size_t wk_direct_workspace_size(const wk_plan* plan);
wk_status wk_plasma_response_direct(const wk_plan* plan, const wk_plasma_bufs* plasma,
                                    const double* d_jb, void* d_fields, void* d_workspace,
                                    size_t workspace_bytes, int32_t iters, double tol,
                                    int32_t* d_iterations, uint64_t* d_counters, void* stream);

/* Bytes of the library's static device scratch array (one per device). */
#define WK_NOALLOC_SCRATCH_BYTES (8u << 20)

/* wk_plasma_response for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same march, with the exchange rows between workgroups,
 * the group counter and the large-grid node rows in a static array of
 * WK_NOALLOC_SCRATCH_BYTES bytes that every device the library runs on holds
 * until the process ends, instead of a caller workspace.  It calls no
 * allocator; the caller passes the inputs and outputs as for
 * wk_plasma_response.  The call runs on the current device, and `stream`
 * must belong to it.  The array holds the march region of every plan that
 * wk_plan_create accepts (n_r <= 2048, up to 16 workgroups: about 7.1 MB);
 * a response that needed more would return WK_ERR_UNSUPPORTED before
 * anything is launched.  Every call on one device shares that
 * device's array, which keeps the last call's contents (each call clears
 * what must start at zero): calls that overlap on one device race, so
 * serialise them (one stream, or events between streams). */
wk_status wk_plasma_response_noalloc(const wk_plan* plan, const wk_plasma_bufs* plasma,
                                     const double* d_jb, void* d_fields,
                                     uint64_t* d_counters, void* stream);

/* Launch shape: smallest workgroup size of the march kernel (256, 512 or
 * 1024; the launch may use a larger one to keep the particles in
 * registers).  The plan picks one from the problem size; an autotuner may
 * override it before the plan is first used. */
wk_status wk_plan_set_threads(wk_plan* plan, int32_t threads);
int32_t wk_plan_threads(const wk_plan* plan);

/* Workgroups that march one response together (1..16, at most n_r; 0 = chosen
 * per call).  The response's plasma cells are split into `group` contiguous
 * bands, one per workgroup; the deposits of the bands (S, the currents and
 * the moments, Section II A) are summed between the workgroups in a fixed
 * order through device memory four times per slice, and every workgroup
 * solves the field equations on the identical sums.  Results do not depend
 * on the group beyond the summation order of the deposits.  All workgroups
 * of a group must run at once; the library sizes its launches so that they
 * do, and a wait that exceeds 20 s sets WK_CNT_PIPELINE_ABORT instead of
 * hanging.  wk_plan_group returns the group a single response uses: the
 * plan's, else 1 up to 1024 macroparticles per slice and max(8, n_p / 1024)
 * above, at most 16 and n_r. */
wk_status wk_plan_set_group(wk_plan* plan, int32_t group);
int32_t wk_plan_group(const wk_plan* plan);

/* Batched responses (a parameter scan of independent instances, any mix of
 * sizes, all with the same geometry, precision and temperature class):
 *   1. wk_batch_describe fills a host blob of wk_batch_desc_bytes(n) bytes
 *      with one descriptor per instance (device pointers of its buffers and
 *      its slice of the workspace), longest instances first;
 *   2. the caller copies the blob to device memory;
 *   3. wk_batch_response marches every instance in one persistent launch:
 *      each instance by a group of workgroups (enough to hold its particles
 *      in registers and to bring its cost, weighted by n_r over the batch's
 *      largest n_r, near the per-compute-unit average
 *      of the batch, at most 16), the workgroups taking tickets (one member
 *      of one instance's group) from a queue in the workspace, longest
 *      instances first.
 * h_* arrays have n entries; d_workspace has wk_batch_workspace_size bytes;
 * a plan's group (wk_plan_set_group) overrides the choice for its instance. */
size_t wk_batch_desc_bytes(int32_t n);
size_t wk_batch_workspace_size(int32_t n, const wk_plan* const* h_plans);
/* Workgroups that march instance i (0-based, in the order of h_plans) under
 * the batch's schedule; 0 for a bad argument. */
int32_t wk_batch_group(int32_t n, const wk_plan* const* h_plans, int32_t i);
wk_status wk_batch_describe(int32_t n, const wk_plan* const* h_plans,
                            const wk_plasma_bufs* h_plasma, const double* const* h_jb,
                            void* const* h_fields, void* d_workspace, size_t workspace_bytes,
                            uint64_t* d_counters, void* h_desc);
wk_status wk_batch_response(int32_t n, const wk_plan* const* h_plans, const void* d_desc,
                            void* d_workspace, size_t workspace_bytes, void* stream);
/* The same launch with an explicit shape: threads per workgroup (256, 512 or
 * 1024; 0 = the largest of the plans' choices) and workgroups per compute
 * unit (1..8, clamped to what LDS and the 2048-thread limit allow; 0 =
 * default).  Used by the autotuner; the results do not depend on the shape
 * beyond the summation order of the deposits. */
wk_status wk_batch_response_shape(int32_t n, const wk_plan* const* h_plans, const void* d_desc,
                                  void* d_workspace, size_t workspace_bytes, int32_t threads,
                                  int32_t wg_per_cu, void* stream);

/* The quasi-static cycle, n_steps times: beam current from the macroparticles
 * -> plasma response -> beam advance by dt (Section II A: the plasma responds
 * to the frozen beam, then the beam is advanced in t).  The responses of
 * successive steps run concurrently on separate groups of workgroups
 * (wk_cycle_group; each member of a group owns a band of the plasma cells
 * and a contiguous subset of the beam): response n marches slice k once
 * response n-1 has stored the slices up to k + 2, and advances the beam
 * particles of each xi bin just before it deposits them.
 * The result equals n_steps sequential calls of wk_beam_current,
 * wk_plasma_response (from the same loaded plasma) and wk_beam_push(1 step)
 * up to the summation order of the deposits.
 *   plasma:   loaded by wk_init_plasma; read only (each response starts from it)
 *   d_ring:   2 * sizes.fields bytes; the fields of response n are in slot
 *             n % 2, so the last response is in slot (n_steps - 1) % 2
 *   workspace: wk_cycle_workspace_size(plan, n_steps) bytes.
 * Any n_r up to 2048: beyond about 880 cells the field and solver node rows
 * live in the workspace and the beam current is deposited straight into the
 * LDS current row instead of an LDS ring of rows.  Counter
 * WK_CNT_PIPELINE_ABORT is set if a workgroup waited too long for another
 * (then the results are invalid); WK_CNT_BEAM_BIN counts particles whose xi
 * moved by more than a slice during the run (or that were found ahead of the
 * window); WK_CNT_BEAM_ORDER is set if a subset's bins lost particles. */
size_t wk_cycle_workspace_size(const wk_plan* plan, int32_t n_steps);
/* Workgroups per response that wk_cycle uses for n_steps steps on the
 * current device: the plan's group when set, else the largest group for
 * which all responses are resident at once. */
int32_t wk_cycle_group(const wk_plan* plan, int32_t n_steps);
wk_status wk_cycle(const wk_plan* plan, const wk_plasma_bufs* plasma, const wk_beam_bufs* beam,
                   int32_t n_steps, double dt, void* d_ring, void* d_workspace,
                   size_t workspace_bytes, uint64_t* d_counters, void* stream);

/* Beam push: advance the beam n_steps times by dt in the frozen fields d_fields
 * (Eqs. (8)-(11), Boris rotation, cancellation-free d xi/dt). */
wk_status wk_beam_push(const wk_plan* plan, const wk_beam_bufs* beam, const void* d_fields,
                       int32_t n_steps, double dt, uint64_t* d_counters, void* stream);

/* Diagnostic: charge-weighted mean gamma gain of the particles with tag == which,
 * written to d_out[0] (deterministic two-level reduction in the
 * workspace). */
wk_status wk_mean_gain(const wk_plan* plan, const wk_beam_bufs* beam, int32_t which,
                       double* d_out, void* d_workspace, void* stream);
/* Diagnostic: energy spectrum of the beam (Section III, the witness energy
 * spectra): counts of the gain gamma - gamma_init of the particles with
 * tag == which (all particles when which < 0) in n_bins (1..4096) equal bins
 * of [lo, hi).  d_hist: uint64[n_bins + 2], written entirely: [0] below lo,
 * [1..n_bins] the bins, [n_bins + 1] at or above hi.  Each particle's bin is
 * decided in double with every operation rounded separately, so the counts
 * are exact and independent of scheduling. */
wk_status wk_gain_histogram(const wk_plan* plan, const wk_beam_bufs* beam, int32_t which,
                            int32_t n_bins, double lo, double hi, uint64_t* d_hist,
                            void* stream);
/* Diagnostic: most negative on-axis E_z over slices with xi_k >= xi_from, written
 * to d_out[0] as double. */
wk_status wk_ez_peak(const wk_plan* plan, const void* d_fields, double xi_from,
                     double* d_out, void* stream);

/* Gradient of the witness energy gain (reverse mode, FP64 or WK_MIXED plans
 * with a two-bunch macroparticle beam; in a mixed plan the recorded march
 * and the per-particle arithmetic of the reverse pass are float, as in
 * wk_plasma_response, while the recorded rows, particle states, adjoint
 * accumulators and the solves stay double).  The objective G is the charge-weighted mean
 * gamma gain of the witness after one plasma response to the loaded beam and
 * n_steps beam advances by dt in that response's frozen fields (Section II A:
 * plasma response for the frozen beam, then the beam advanced over the long
 * step).  Its parameters theta are, in this order: the drive peak density
 * bunch[0].n_peak, the common sigma_r, the drive length bunch[0].sigma_z, the
 * witness separation bunch[1].xi_c - bunch[0].xi_c, and the thermal spread
 * u_th (Eq. (12) beam, thermal plasma loading); the random draws of both
 * loaders are held fixed.  The u_th component is defined for warm plans
 * (u_th > 0) and is 0 otherwise.
 *
 * wk_gradient_forward loads the beam and the plasma from the draws, computes
 * the beam current, marches the plasma (storing d_fields as
 * wk_plasma_response does) while recording what the reverse pass needs in
 * the workspace: per slice and Heun stage the node rows psi, psi', E_z,
 * B_theta, J_r, J_z, M1..M5, and the particle state every `every` slices
 * (the reverse pass recomputes the states in between); then advances the
 * beam n_steps times, recording each step, and writes G to d_out[0].
 * wk_gradient_backward, called after it with the same buffers and
 * workspace, writes d_grad[0..4] = d_gbar[0] * dG/dtheta.  The workspace has
 * wk_gradient_workspace_size bytes (0: the plan or arguments are not
 * supported; the reason is in wk_last_error()) and depends on the plan's
 * workgroup size (wk_plan_set_threads), which the reverse march also uses.
 * The recording march runs on the group of a plain response
 * (wk_plan_group) and uses the exchange rows of the plan workspace inside
 * the gradient workspace.
 * The reverse march needs n_r <= 740 (LDS).  It runs on a group of up to 8
 * workgroups, each with a share of the particles, that sum their deposited
 * node adjoints through the workspace: the plan's group
 * (wk_plan_set_group, capped at 8), else about one particle per thread.
 * All members must run at once; a member that waits more than 20 s for the
 * others gives up, and the gradient is then NaN. */
size_t wk_gradient_workspace_size(const wk_plan* plan, int32_t n_steps, int32_t every);
wk_status wk_gradient_forward(const wk_plan* plan, const wk_plasma_bufs* plasma, const double* d_plasma_draws,
                              const wk_beam_bufs* beam, const double* d_beam_draws, int32_t n_steps, double dt,
                              int32_t every, void* d_fields, double* d_out, void* d_workspace,
                              size_t workspace_bytes, uint64_t* d_counters, void* stream);
wk_status wk_gradient_backward(const wk_plan* plan, const wk_plasma_bufs* plasma, const double* d_plasma_draws,
                               const wk_beam_bufs* beam, const double* d_beam_draws, int32_t n_steps, double dt,
                               int32_t every, const void* d_fields, const double* d_gbar, double* d_grad,
                               void* d_workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* WAKE_H */
