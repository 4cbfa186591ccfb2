// C ABI of libwake: problem validation, plans, buffer sizes and launches.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "wk_direct.h"
#include "wk_internal.h"

struct wk_plan {
    wk_problem p;
    int32_t N;        // cells
    int32_t N1;       // nodes
    int64_t np;       // plasma macroparticles per slice
    double h, dxi;
    int32_t threads;  // preferred workgroup size (256, 512 or 1024)
    int32_t group;    // workgroups per response (0: chosen per call)
    wk_sizes sizes;
    size_t ws_beam_off;
    bool big;   // node rows beyond LDS: the march keeps its field rows in the workspace
};

namespace {

// Compute units of the current device (queried once per device).
int device_cus()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev >= 0 && dev < 64 && cache[dev].load() > 0) return cache[dev].load();
    int cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    if (dev >= 0 && dev < 64) cache[dev].store(cus);
    return cus;
}

thread_local std::string g_err;

wk_status fail(wk_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
wk_status fail(wk_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

wk_status hip_status(hipError_t e, const char* what)
{
    if (e == hipSuccess) return WK_OK;
    return fail(WK_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t real_size(const wk_problem& p) { return p.prec == WK_FP64 ? sizeof(double) : sizeof(float); }

wk::GridDesc grid_of(const wk_plan* pl)
{
    wk::GridDesc g;
    g.geom = pl->p.geom;
    g.n_r = pl->N;
    g.n_xi = pl->p.n_xi;
    g.r_max = pl->p.r_max;
    g.h = pl->h;
    g.xi_min = pl->p.xi_min;
    g.dxi = pl->dxi;
    return g;
}

int default_threads(int64_t np)
{
    if (np <= 2048) return 256;
    if (np <= 8192) return 512;
    return 1024;
}

// Workgroups per response of a single march: the plan's choice, else one
// for up to 1024 particles and otherwise max(8, n_p / 1024), at most
// kMaxGroup and the number of cells.  Two or four members are slower than
// one or eight at 2048-4096 particles: they add the exchanges without
// shortening a slice enough.
int single_group(const wk_plan* pl)
{
    int G = pl->group;
    if (G <= 0)
        G = pl->np <= 1024 ? 1 : (int)std::min<int64_t>(wk::kMaxGroup, std::max<int64_t>(8, pl->np / 1024));
    return std::max(1, std::min(G, pl->N));
}

// Particles of the largest workgroup share when G workgroups march a response.
int64_t member_np(const wk_plan* pl, int G) { return (int64_t)((pl->N + G - 1) / G) * pl->p.ppc; }

// March region at the start of a plan workspace: the large-grid node rows of
// up to kMaxGroup workgroups, the group's partial rows and its counter.
// exchange rows of a group: two slots of G partials of kXRows node rows
size_t march_xbuf_bytes(int N1, int G)
{
    return a256((size_t)2 * G * wk::kXRows * wk::lds_stride(N1) * sizeof(double));
}
// Layout of a march region for `G` workgroups: the large-grid node rows, the
// exchange rows, then the group counter.
size_t march_grow_bytes(const wk_plan* pl, int G) { return pl->big ? G * a256(wk::big_rows_bytes(pl->N1)) : 0; }
size_t march_region_bytes(const wk_plan* pl, int G)
{
    return march_grow_bytes(pl, G) + march_xbuf_bytes(pl->N1, G) + 256;
}
size_t march_region_bytes(const wk_plan* pl) { return march_region_bytes(pl, wk::kMaxGroup); }

bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

wk_status check_plasma(const wk_plan* pl, const wk_plasma_bufs* b)
{
    if (!b) return fail(WK_ERR_INVALID_ARG, "plasma buffers are NULL");
    if (!b->d_x || !b->d_px || !b->d_d0 || !b->d_w || !b->d_nion)
        return fail(WK_ERR_BUFFER, "plasma buffer pointer is NULL");
    const bool warm = pl->p.u_th > 0.0;
    if (pl->p.geom == WK_CYL && warm && (!b->d_y || !b->d_py))
        return fail(WK_ERR_BUFFER, "warm cylindrical plasma needs y and py buffers");
    if (pl->p.geom == WK_SLAB && warm && !b->d_py)
        return fail(WK_ERR_BUFFER, "warm slab plasma needs the py buffer");
    if (!aligned8(b->d_x) || !aligned8(b->d_px) || !aligned8(b->d_nion))
        return fail(WK_ERR_BUFFER, "plasma buffers must be 8-byte aligned");
    return WK_OK;
}

wk_status check_beam(const wk_plan* pl, const wk_beam_bufs* b)
{
    if (!b) return fail(WK_ERR_INVALID_ARG, "beam buffers are NULL");
    if (pl->p.n_beam <= 0) return fail(WK_ERR_INVALID_ARG, "plan has no beam macroparticles");
    if (!b->d_x || !b->d_y || !b->d_px || !b->d_py || !b->d_pz || !b->d_xi || !b->d_w ||
        !b->d_gamma_init || !b->d_tag)
        return fail(WK_ERR_BUFFER, "beam buffer pointer is NULL");
    return WK_OK;
}

wk::MarchDesc make_desc(const wk_plan* pl, const wk_plasma_bufs* b, const double* jb, void* fields,
                        uint64_t* counters)
{
    wk::MarchDesc d;
    d.geom = pl->p.geom;
    d.warm = pl->p.u_th > 0.0 ? 1 : 0;
    d.n_r = pl->N;
    d.n_xi = pl->p.n_xi;
    d.np = pl->np;
    d.r_max = pl->p.r_max;
    d.h = pl->h;
    d.dxi = pl->dxi;
    d.d_min = pl->p.d_min;
    d.x = b->d_x;
    d.y = b->d_y;
    d.px = b->d_px;
    d.py = b->d_py;
    d.d0 = b->d_d0;
    d.w = b->d_w;
    d.nion = b->d_nion;
    d.jb = jb;
    d.fields = fields;
    d.counters = (unsigned long long*)counters;
    d.cost = pl->np * (int64_t)pl->p.n_xi;
    d.grow = nullptr;
    d.ppc = pl->p.ppc;
    d.group = 1;
    d.xbuf = nullptr;
    d.gctr = nullptr;
    d.p0 = 0;
    d.traj = nullptr;
    d.traj_n = 0;
    d.traj_stride = 0;
    return d;
}

// One response from a march region at `ws` laid out for `layout_group`
// workgroups (at least the group that marches it).
wk_status response_in(const wk_plan* plan, const wk_plasma_bufs* plasma, const double* d_jb, void* d_fields,
                      char* ws, int layout_group, uint64_t* d_counters, hipStream_t s, double* traj = nullptr,
                      int traj_stride = 0)
{
    const int G = single_group(plan);
    const int shape = wk::pick_shape(member_np(plan, G), plan->threads, plan->N1, plan->p.prec, G);
    wk::MarchLaunch L{};
    L.one = make_desc(plan, plasma, d_jb, d_fields, d_counters);
    L.one.group = G;
    if (traj) {
        L.one.traj = traj;
        L.one.traj_stride = traj_stride;
        L.one.traj_n = (plan->np + traj_stride - 1) / traj_stride;
    }
    L.one.xbuf = (double*)(ws + march_grow_bytes(plan, layout_group));
    L.one.gctr = (unsigned*)(ws + march_grow_bytes(plan, layout_group) + march_xbuf_bytes(plan->N1, layout_group));
    L.grow = plan->big ? (double*)ws : nullptr;
    L.grow_stride = wk::lds_stride(plan->N1);
    // the exchange slots start zeroed (tag 0) for every launch
    hipError_t e = G > 1 ? wk::launch_zero_u32((unsigned*)L.one.xbuf, (int64_t)march_xbuf_bytes(plan->N1, G) / 4, s)
                         : hipSuccess;
    if (e == hipSuccess) e = wk::launch_zero_u32(L.one.gctr, 1, s);
    if (e == hipSuccess)
        e = wk::launch_march(L, plan->p.prec, plan->p.geom, L.one.warm, shape, G, plan->N1, s);
    return hip_status(e, "plasma response");
}

// Scratch of wk_plasma_response_noalloc: the march region of one response,
// resident on every device the library runs on.  Host code reaches it only
// through the per-device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[WK_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
wk_status scratch_address(char** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(WK_ERR_UNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "scratch address");
        if (!ptr) return fail(WK_ERR_HIP, "scratch address is NULL");
        g_scratch[dev] = (char*)ptr;
    }
    *out = g_scratch[dev];
    return WK_OK;
}

}  // namespace

extern "C" {

const char* wk_version(void) { return "wake-mi355x 0.1 (gfx950)"; }

const char* wk_status_string(wk_status s)
{
    switch (s) {
    case WK_OK: return "ok";
    case WK_ERR_INVALID_ARG: return "invalid argument";
    case WK_ERR_UNSUPPORTED: return "unsupported";
    case WK_ERR_BUFFER: return "bad buffer";
    case WK_ERR_HIP: return "HIP runtime error";
    case WK_ERR_NUMERIC: return "non-finite values";
    }
    return "unknown status";
}

const char* wk_last_error(void) { return g_err.c_str(); }

wk_status wk_plan_create(const wk_problem* p, wk_plan** out)
{
    if (!p || !out) return fail(WK_ERR_INVALID_ARG, "NULL problem or output pointer");
    *out = nullptr;
    if (p->geom != WK_CYL && p->geom != WK_SLAB) return fail(WK_ERR_INVALID_ARG, "geom must be WK_CYL or WK_SLAB");
    if (p->n_r < 2 || p->n_r > 2048) return fail(WK_ERR_INVALID_ARG, "n_r must be in [2, 2048] (got %d)", p->n_r);
    if (p->n_xi < 1) return fail(WK_ERR_INVALID_ARG, "n_xi must be >= 1");
    if (!(p->r_max > 0.0) || !std::isfinite(p->r_max)) return fail(WK_ERR_INVALID_ARG, "r_max must be > 0");
    if (!(p->xi_max > p->xi_min) || !std::isfinite(p->xi_max - p->xi_min))
        return fail(WK_ERR_INVALID_ARG, "xi_max must exceed xi_min");
    if (p->ppc < 1 || p->ppc > 128) return fail(WK_ERR_INVALID_ARG, "ppc must be in [1, 128]");
    if (!(p->u_th >= 0.0)) return fail(WK_ERR_INVALID_ARG, "u_th must be >= 0");
    if (p->u_th > 0.0 && (p->ppc % 2)) return fail(WK_ERR_INVALID_ARG, "warm plasma needs an even ppc (mirrored pairs)");
    if (!(p->n0 > 0.0)) return fail(WK_ERR_INVALID_ARG, "n0 must be > 0");
    if (p->n_bunch < 0 || p->n_bunch > 2) return fail(WK_ERR_INVALID_ARG, "n_bunch must be 0, 1 or 2");
    if (p->n_bunch > 0 && !(p->sigma_r > 0.0)) return fail(WK_ERR_INVALID_ARG, "sigma_r must be > 0");
    for (int b = 0; b < p->n_bunch; ++b)
        if (!(p->bunch[b].sigma_z > 0.0)) return fail(WK_ERR_INVALID_ARG, "bunch sigma_z must be > 0");
    if (p->prec != WK_FP64 && p->prec != WK_MIXED) return fail(WK_ERR_INVALID_ARG, "prec must be WK_FP64 or WK_MIXED");
    if (!(p->d_min > 0.0)) return fail(WK_ERR_INVALID_ARG, "d_min must be > 0");
    if (p->n_beam < 0 || p->n_drive < 0 || p->n_drive > p->n_beam)
        return fail(WK_ERR_INVALID_ARG, "need 0 <= n_drive <= n_beam");
    if (p->n_beam > 0) {
        if (p->n_bunch < 1) return fail(WK_ERR_INVALID_ARG, "beam macroparticles need at least one bunch");
        if (p->n_bunch == 1 && p->n_drive != p->n_beam) return fail(WK_ERR_INVALID_ARG, "single bunch: n_drive must equal n_beam");
        if (p->n_bunch == 2 && (p->n_drive == 0 || p->n_drive == p->n_beam))
            return fail(WK_ERR_INVALID_ARG, "two bunches need macroparticles in both");
        if (p->n_beam > (int64_t)0xFFFFFFF0) return fail(WK_ERR_UNSUPPORTED, "n_beam above 2^32 - 16");
        if (!(p->gamma0 > 1.0)) return fail(WK_ERR_INVALID_ARG, "gamma0 must be > 1");
    }
    const int N1 = p->n_r + 1;
    if (wk::big_lds_bytes(N1) > 159 * 1024)
        return fail(WK_ERR_UNSUPPORTED, "n_r = %d needs more LDS than one workgroup has", p->n_r);

    wk_plan* pl = new (std::nothrow) wk_plan;
    if (!pl) return fail(WK_ERR_INVALID_ARG, "out of host memory");
    pl->p = *p;
    pl->N = p->n_r;
    pl->N1 = N1;
    pl->np = (int64_t)p->n_r * p->ppc;
    pl->h = p->r_max / p->n_r;
    pl->dxi = (p->xi_max - p->xi_min) / p->n_xi;
    pl->threads = default_threads(pl->np);
    pl->group = 0;
    const size_t rs = real_size(*p);
    wk_sizes& s = pl->sizes;
    s.n_plasma = pl->np;
    s.n_nodes = N1;
    s.plasma_state = a256(sizeof(double) * pl->np);
    s.plasma_const = a256(rs * pl->np);
    s.plasma_draws = a256(sizeof(double) * 3 * (pl->np / 2 + 1));
    s.nion = a256(sizeof(double) * N1);
    s.beam_current = a256(sizeof(double) * (size_t)p->n_xi * N1);
    s.fields = a256(rs * 4 * (size_t)p->n_xi * N1);
    const int64_t nb = p->n_beam > 0 ? p->n_beam : 1;
    s.beam_state = a256(sizeof(double) * nb);
    s.beam_tag = a256(sizeof(int32_t) * nb);
    s.beam_draws = a256(sizeof(double) * 4 * nb);
    // the march region first (large-grid node rows, group exchange), then
    // the beam binning
    pl->big = wk::march_needs_global_rows(N1);
    pl->ws_beam_off = march_region_bytes(pl);
    s.workspace = pl->ws_beam_off + a256(wk::beam_ws_bytes(p->n_xi, p->n_beam));
    s.counters = a256(sizeof(uint64_t) * WK_NCOUNTERS);
    *out = pl;
    g_err.clear();
    return WK_OK;
}

void wk_plan_destroy(wk_plan* plan) { delete plan; }

wk_status wk_plan_sizes(const wk_plan* plan, wk_sizes* out)
{
    if (!plan || !out) return fail(WK_ERR_INVALID_ARG, "NULL plan or output");
    *out = plan->sizes;
    return WK_OK;
}

wk_status wk_plan_set_threads(wk_plan* plan, int32_t threads)
{
    if (!plan) return fail(WK_ERR_INVALID_ARG, "NULL plan");
    if (threads != 256 && threads != 512 && threads != 1024)
        return fail(WK_ERR_INVALID_ARG, "threads must be 256, 512 or 1024");
    plan->threads = threads;
    return WK_OK;
}

int32_t wk_plan_threads(const wk_plan* plan) { return plan ? plan->threads : 0; }

wk_status wk_plan_set_group(wk_plan* plan, int32_t group)
{
    if (!plan) return fail(WK_ERR_INVALID_ARG, "NULL plan");
    if (group < 0 || group > wk::kMaxGroup) return fail(WK_ERR_INVALID_ARG, "group must be 0..%d", wk::kMaxGroup);
    if (group > plan->N) return fail(WK_ERR_INVALID_ARG, "group %d exceeds the %d cells", group, plan->N);
    plan->group = group;
    return WK_OK;
}

int32_t wk_plan_group(const wk_plan* plan) { return plan ? single_group(plan) : 0; }

wk_status wk_counters_zero(uint64_t* d_counters, void* stream)
{
    if (!d_counters) return fail(WK_ERR_INVALID_ARG, "NULL counters");
    return hip_status(wk::launch_zero_u64((unsigned long long*)d_counters, WK_NCOUNTERS, (hipStream_t)stream),
                      "zero counters");
}

wk_status wk_counters_read(const uint64_t* d_counters, uint64_t* h_out, void* stream)
{
    if (!d_counters || !h_out) return fail(WK_ERR_INVALID_ARG, "NULL counters or output");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(h_out, d_counters, sizeof(uint64_t) * WK_NCOUNTERS, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "read counters");
    if (h_out[WK_CNT_NONFINITE] != 0)
        return fail(WK_ERR_NUMERIC, "%llu non-finite field values", (unsigned long long)h_out[WK_CNT_NONFINITE]);
    if (h_out[WK_CNT_PIPELINE_ABORT] != 0) return fail(WK_ERR_NUMERIC, "a wait between workgroups gave up");
    if (h_out[WK_CNT_BEAM_ORDER] != 0) return fail(WK_ERR_NUMERIC, "a pipelined cycle lost beam particles from its bins");
    return WK_OK;
}

wk_status wk_init_plasma(const wk_plan* plan, const wk_plasma_bufs* plasma, const double* d_draws, void* stream)
{
    if (!plan) return fail(WK_ERR_INVALID_ARG, "NULL plan");
    wk_status st = check_plasma(plan, plasma);
    if (st != WK_OK) return st;
    if (plan->p.u_th > 0.0 && !d_draws) return fail(WK_ERR_INVALID_ARG, "warm plasma needs draws");
    return hip_status(wk::launch_init_plasma(grid_of(plan), plan->p.ppc, plan->p.u_th, plan->p.n0, plan->p.prec,
                                             *plasma, d_draws, (hipStream_t)stream),
                      "init plasma");
}

wk_status wk_init_beam(const wk_plan* plan, const wk_beam_bufs* beam, const double* d_draws, void* stream)
{
    if (!plan) return fail(WK_ERR_INVALID_ARG, "NULL plan");
    wk_status st = check_beam(plan, beam);
    if (st != WK_OK) return st;
    if (!d_draws) return fail(WK_ERR_INVALID_ARG, "beam loader needs draws");
    return hip_status(wk::launch_init_beam(grid_of(plan), plan->p, *beam, d_draws, (hipStream_t)stream), "init beam");
}

wk_status wk_beam_current_analytic(const wk_plan* plan, double* d_jb, void* stream)
{
    if (!plan || !d_jb) return fail(WK_ERR_INVALID_ARG, "NULL plan or jb");
    return hip_status(wk::launch_beam_current_analytic(grid_of(plan), plan->p, d_jb, (hipStream_t)stream),
                      "analytic beam current");
}

wk_status wk_beam_current(const wk_plan* plan, const wk_beam_bufs* beam, double* d_jb, void* d_workspace,
                          uint64_t* d_counters, void* stream)
{
    if (!plan || !d_jb || !d_workspace || !d_counters) return fail(WK_ERR_INVALID_ARG, "NULL argument");
    wk_status st = check_beam(plan, beam);
    if (st != WK_OK) return st;
    return hip_status(wk::launch_beam_current(grid_of(plan), plan->p.n_beam, *beam, d_jb,
                                              (char*)d_workspace + plan->ws_beam_off,
                                              (unsigned long long*)d_counters, (hipStream_t)stream),
                      "beam current");
}

wk_status wk_plasma_response(const wk_plan* plan, const wk_plasma_bufs* plasma, const double* d_jb, void* d_fields,
                             void* d_workspace, uint64_t* d_counters, void* stream)
{
    if (!plan || !d_jb || !d_fields || !d_workspace || !d_counters) return fail(WK_ERR_INVALID_ARG, "NULL argument");
    wk_status st = check_plasma(plan, plasma);
    if (st != WK_OK) return st;
    return response_in(plan, plasma, d_jb, d_fields, (char*)d_workspace, wk::kMaxGroup, d_counters,
                       (hipStream_t)stream);
}

wk_status wk_plasma_response_traj(const wk_plan* plan, const wk_plasma_bufs* plasma, const double* d_jb,
                                  void* d_fields, void* d_workspace, int32_t stride, double* d_traj,
                                  uint64_t* d_counters, void* stream)
{
    if (!plan || !d_jb || !d_fields || !d_workspace || !d_traj || !d_counters)
        return fail(WK_ERR_INVALID_ARG, "NULL argument");
    if (stride < 1) return fail(WK_ERR_INVALID_ARG, "stride must be >= 1 (got %d)", stride);
    if (plan->p.prec != WK_FP64) return fail(WK_ERR_UNSUPPORTED, "trajectories are recorded by FP64 plans only");
    if (!aligned8(d_traj)) return fail(WK_ERR_BUFFER, "trajectory buffer is not 8-byte aligned");
    wk_status st = check_plasma(plan, plasma);
    if (st != WK_OK) return st;
    return response_in(plan, plasma, d_jb, d_fields, (char*)d_workspace, wk::kMaxGroup, d_counters,
                       (hipStream_t)stream, d_traj, stride);
}

size_t wk_direct_workspace_size(const wk_plan* plan)
{
    if (!plan) return 0;
    return a256(wk::direct_ws_doubles(plan->np, plan->N1) * sizeof(double));
}

wk_status wk_plasma_response_direct(const wk_plan* plan, const wk_plasma_bufs* plasma, const double* d_jb,
                                    void* d_fields, void* d_workspace, size_t workspace_bytes, int32_t iters,
                                    double tol, int32_t* d_iterations, uint64_t* d_counters, void* stream)
{
    if (!plan || !d_jb || !d_fields || !d_workspace || !d_counters) return fail(WK_ERR_INVALID_ARG, "NULL argument");
    if (plan->p.prec != WK_FP64) return fail(WK_ERR_UNSUPPORTED, "the Eq. (6)-direct response is FP64 only");
    if (iters < 1 || iters > 64) return fail(WK_ERR_INVALID_ARG, "iters must be 1..64 (got %d)", iters);
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(WK_ERR_INVALID_ARG, "tol must be finite and > 0");
    if (!wk::lds_fits(wk::direct_lds_bytes(plan->N1)))
        return fail(WK_ERR_UNSUPPORTED, "the Eq. (6)-direct response keeps its rows in LDS: n_r = %d is too large",
                    plan->N);
    const size_t need = wk_direct_workspace_size(plan);
    if (workspace_bytes < need) return fail(WK_ERR_BUFFER, "direct workspace needs %zu bytes", need);
    if (!aligned8(d_workspace) || (d_iterations && ((uintptr_t)d_iterations & 3)))
        return fail(WK_ERR_BUFFER, "workspace or iterations buffer misaligned");
    wk_status st = check_plasma(plan, plasma);
    if (st != WK_OK) return st;
    wk::DirectDesc dd{};
    dd.march = make_desc(plan, plasma, d_jb, d_fields, d_counters);
    const int64_t n4 = std::max<int64_t>(plan->np, 1) * 4;
    double* ws = (double*)d_workspace;
    dd.ys = ws;
    dd.yn = ws + n4;
    dd.f0 = ws + 2 * n4;
    dd.V = ws + 3 * n4;
    dd.iters = iters;
    dd.tol = tol;
    dd.iterations = d_iterations;
    return hip_status(wk::launch_march_direct(dd, (hipStream_t)stream), "Eq. (6)-direct response");
}

wk_status wk_plasma_response_noalloc(const wk_plan* plan, const wk_plasma_bufs* plasma, const double* d_jb,
                                     void* d_fields, uint64_t* d_counters, void* stream)
{
    if (!plan || !d_jb || !d_fields || !d_counters) return fail(WK_ERR_INVALID_ARG, "NULL argument");
    wk_status st = check_plasma(plan, plasma);
    if (st != WK_OK) return st;
    const int G = single_group(plan);
    const size_t need = march_region_bytes(plan, G);
    if (need > WK_NOALLOC_SCRATCH_BYTES)
        return fail(WK_ERR_UNSUPPORTED, "response needs %zu bytes of scratch, the static array holds %zu", need,
                    (size_t)WK_NOALLOC_SCRATCH_BYTES);
    char* ws = nullptr;
    st = scratch_address(&ws);
    if (st != WK_OK) return st;
    return response_in(plan, plasma, d_jb, d_fields, ws, G, d_counters, (hipStream_t)stream);
}

size_t wk_batch_desc_bytes(int32_t n)
{
    if (n <= 0) return 0;
    return a256(sizeof(wk::MarchDesc) * (size_t)n) + a256(sizeof(int) * 2 * wk::kMaxGroup * (size_t)n);
}

}  // extern "C"

namespace {

// Work plan of a batch: instances longest first (by particle-slice updates),
// each marched by G_i workgroups: enough to hold its particles in registers
// (8192 per workgroup) and to bring its cost, weighted by n_r / (the batch's
// largest n_r), near the per-compute-unit average of the batch; at most
// kMaxGroup and its number of cells.  The weight: every member repeats the
// grid work of a slice, so an instance with the batch's largest grid has the
// longest slices and sets the longest chain; one with a smaller grid
// finishes within the makespan on fewer members and spends less on repeated
// grid work and exchanges.
struct BatchSchedule {
    std::vector<int> order;     // instance indices, longest first
    std::vector<int> group;     // G of each instance (original index)
    std::vector<size_t> xoff;   // exchange rows of each instance in the workspace (0: none)
    int tickets = 0;
    int64_t max_member = 0;     // particles of the largest workgroup share
    int max_nodes = 0;
    size_t ws = 0;
};

BatchSchedule batch_schedule(int n, const wk_plan* const* plans)
{
    BatchSchedule B;
    B.group.resize(n);
    B.xoff.assign(n, 0);
    double total = 0.0;
    int nr_max = 1;
    for (int i = 0; i < n; ++i) {
        total += (double)plans[i]->np * plans[i]->p.n_xi;
        nr_max = std::max(nr_max, plans[i]->N);
    }
    const double per_cu = total / std::max(1, device_cus());
    for (int i = 0; i < n; ++i) {
        const wk_plan* pl = plans[i];
        const double cost = (double)pl->np * pl->p.n_xi * ((double)pl->N / nr_max);
        int G = pl->group > 0 ? pl->group
                              : (int)std::max<double>(std::ceil((double)pl->np / 8192.0), std::ceil(cost / per_cu));
        G = std::max(1, std::min({G, wk::kMaxGroup, pl->N}));
        B.group[i] = G;
        B.tickets += G;
        B.max_member = std::max(B.max_member, member_np(pl, G));
        B.max_nodes = std::max(B.max_nodes, pl->N1);
    }
    B.order.resize(n);
    for (int i = 0; i < n; ++i) B.order[i] = i;
    std::stable_sort(B.order.begin(), B.order.end(), [&](int a, int b) {
        return (double)plans[a]->np * plans[a]->p.n_xi > (double)plans[b]->np * plans[b]->p.n_xi;
    });
    // workspace: ticket counter, one group counter per instance, exchange rows
    size_t o = 256 + a256((size_t)n * wk::kCtrPad * sizeof(unsigned));
    for (int i = 0; i < n; ++i)
        if (B.group[i] > 1) {
            B.xoff[i] = o;
            o += march_xbuf_bytes(plans[i]->N1, B.group[i]);
        }
    B.ws = o;
    return B;
}

}  // namespace

extern "C" {

size_t wk_batch_workspace_size(int32_t n, const wk_plan* const* h_plans)
{
    if (n <= 0 || !h_plans) return 0;
    for (int i = 0; i < n; ++i)
        if (!h_plans[i]) return 0;
    return batch_schedule(n, h_plans).ws;
}

int32_t wk_batch_group(int32_t n, const wk_plan* const* h_plans, int32_t i)
{
    if (i < 0 || i >= n || wk_batch_workspace_size(n, h_plans) == 0) return 0;
    return batch_schedule(n, h_plans).group[i];
}

wk_status wk_batch_describe(int32_t n, const wk_plan* const* h_plans, const wk_plasma_bufs* h_plasma,
                            const double* const* h_jb, void* const* h_fields, void* d_workspace,
                            size_t workspace_bytes, uint64_t* d_counters, void* h_desc)
{
    if (n <= 0 || !h_plans || !h_plasma || !h_jb || !h_fields || !d_workspace || !d_counters || !h_desc)
        return fail(WK_ERR_INVALID_ARG, "NULL argument or n <= 0");
    const size_t need = wk_batch_workspace_size(n, h_plans);
    if (need == 0) return fail(WK_ERR_INVALID_ARG, "NULL plan in batch");
    if (workspace_bytes < need) return fail(WK_ERR_BUFFER, "batch workspace needs %zu bytes", need);
    const BatchSchedule B = batch_schedule(n, h_plans);
    const wk_plan* p0 = h_plans[0];
    bool any_warm = false;
    for (int i = 0; i < n; ++i) any_warm |= h_plans[i]->p.u_th > 0.0;
    std::vector<wk::MarchDesc> descs((size_t)n);
    char* ws = (char*)d_workspace;
    for (int q = 0; q < n; ++q) {
        const int i = B.order[q];
        const wk_plan* pl = h_plans[i];
        if (pl->p.prec != p0->p.prec || pl->p.geom != p0->p.geom)
            return fail(WK_ERR_UNSUPPORTED, "batch instances must share geometry and precision");
        wk_status st = check_plasma(pl, &h_plasma[i]);
        if (st != WK_OK) return st;
        // a batch with a warm instance runs every instance on the warm path,
        // which reads the transverse momenta of all of them
        if (any_warm && (!h_plasma[i].d_py || (pl->p.geom == WK_CYL && !h_plasma[i].d_y)))
            return fail(WK_ERR_BUFFER, "instance %d: a batch with warm instances needs y and py buffers for every "
                                       "instance", i);
        if (pl->big) return fail(WK_ERR_UNSUPPORTED, "instance %d: n_r = %d is too large for a batch", i, pl->N);
        if (!h_jb[i] || !h_fields[i]) return fail(WK_ERR_INVALID_ARG, "NULL jb or fields for instance %d", i);
        wk::MarchDesc d = make_desc(pl, &h_plasma[i], h_jb[i], h_fields[i], d_counters);
        d.warm = any_warm ? 1 : 0;
        d.group = B.group[i];
        d.gctr = (unsigned*)(ws + 256) + (size_t)i * wk::kCtrPad;
        d.xbuf = B.group[i] > 1 ? (double*)(ws + B.xoff[i]) : nullptr;
        descs[q] = d;
    }
    std::memcpy(h_desc, descs.data(), sizeof(wk::MarchDesc) * (size_t)n);
    int* tk = (int*)((char*)h_desc + a256(sizeof(wk::MarchDesc) * (size_t)n));
    int t = 0;
    for (int q = 0; q < n; ++q)
        for (int r = 0; r < B.group[B.order[q]]; ++r) {
            tk[2 * t] = q;
            tk[2 * t + 1] = r;
            ++t;
        }
    return WK_OK;
}

wk_status wk_batch_response_shape(int32_t n, const wk_plan* const* h_plans, const void* d_desc, void* d_workspace,
                                  size_t workspace_bytes, int32_t threads, int32_t wg_per_cu, void* stream)
{
    if (n <= 0 || !h_plans || !d_desc || !d_workspace) return fail(WK_ERR_INVALID_ARG, "NULL argument or n <= 0");
    const size_t need = wk_batch_workspace_size(n, h_plans);
    if (need == 0 || workspace_bytes < need) return fail(WK_ERR_BUFFER, "batch workspace too small");
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return fail(WK_ERR_INVALID_ARG, "threads must be 0, 256, 512 or 1024 (got %d)", threads);
    if (wg_per_cu < 0 || wg_per_cu > 8) return fail(WK_ERR_INVALID_ARG, "wg_per_cu must be 0..8 (got %d)", wg_per_cu);
    const BatchSchedule B = batch_schedule(n, h_plans);
    bool warm = false;
    for (int i = 0; i < n; ++i) warm |= h_plans[i]->p.u_th > 0.0;
    const int prec = h_plans[0]->p.prec, geom = h_plans[0]->p.geom;
    int gmax = 1;
    for (int i = 0; i < n; ++i) gmax = std::max(gmax, B.group[i]);
    const int shape = wk::pick_shape(B.max_member, threads > 0 ? threads : 512, B.max_nodes, prec, gmax);
    const int occ = wk::march_occupancy(prec, geom, warm ? 1 : 0, shape, B.max_nodes);
    if (occ <= 0) return fail(WK_ERR_UNSUPPORTED, "batch: no resident workgroup fits (%d nodes)", B.max_nodes);
    const int per_cu = wg_per_cu > 0 ? std::min<int>(wg_per_cu, occ) : occ;
    const int grid = std::min(B.tickets, device_cus() * per_cu);
    hipStream_t s = (hipStream_t)stream;
    // ticket counter, group counters and exchange slots start at zero (a
    // kernel: capturable)
    hipError_t e = wk::launch_zero_u32((unsigned*)d_workspace, (int64_t)B.ws / 4, s);
    if (e != hipSuccess) return hip_status(e, "batch queue");
    wk::MarchLaunch L{};
    L.descs = (const wk::MarchDesc*)d_desc;
    L.tickets = (const int*)((const char*)d_desc + a256(sizeof(wk::MarchDesc) * (size_t)n));
    L.n_tickets = B.tickets;
    L.next = (unsigned*)d_workspace;
    return hip_status(wk::launch_march(L, prec, geom, warm ? 1 : 0, shape, grid, B.max_nodes, s), "batch response");
}

wk_status wk_batch_response(int32_t n, const wk_plan* const* h_plans, const void* d_desc, void* d_workspace,
                            size_t workspace_bytes, void* stream)
{
    return wk_batch_response_shape(n, h_plans, d_desc, d_workspace, workspace_bytes, 0, 0, stream);
}

}  // extern "C"

namespace {

// Launch plan and workspace layout of a pipelined cycle.  G workgroups march
// each response: the plan's choice, else the largest G (at most kMaxGroup and
// the number of cells) for which all n_steps + 1 groups are resident at once.
struct CycleLayout {
    int G = 1, shape = 0, grid = 1;
    int64_t np_max = 0;   // particles of the largest workgroup share
    size_t count, start, fill, order, progress, ticket, gctr, zero_end, plasma, big, xbuf, total;
};

CycleLayout cycle_layout(const wk_plan* pl, int32_t n_steps)
{
    CycleLayout L;
    const int prec = pl->p.prec, geom = pl->p.geom, warm = pl->p.u_th > 0.0 ? 1 : 0;
    const int cus = device_cus();
    // beyond 8 workgroups the exchanges cost more than the split saves
    const int gmax = std::min(pl->group > 0 ? wk::kMaxGroup : 8, pl->N);
    bool found = false;
    for (int G = gmax; G >= 1 && !found; --G) {
        if (pl->group > 0 && G != pl->group) continue;
        int shape = wk::pick_shape(member_np(pl, G), pl->threads, pl->N1, prec, G);
        // the ring of beam-current rows may push a grid into the large-grid shapes
        if (!wk::kShapes[shape].big && !wk::lds_fits(wk::cycle_lds_bytes(shape, pl->N1, prec)))
            shape = (prec != WK_FP64 && member_np(pl, G) <= (int64_t)wk::kShapes[wk::SH_BIG_512_8].threads *
                                                              wk::kShapes[wk::SH_BIG_512_8].kp)
                        ? wk::SH_BIG_512_8
                        : wk::SH_BIG_STREAM;
        int occ = wk::cycle_occupancy(prec, geom, warm, shape, pl->N1);
        if (occ <= 0) occ = 1;
        const int cap = (cus * occ / G) * G;
        if (cap < G) continue;
        const int64_t want = (int64_t)(n_steps + 1) * G;
        if (want <= cap || G == 1 || pl->group > 0) {
            L.G = G;
            L.shape = shape;
            L.grid = (int)std::min<int64_t>(want, cap);
            found = true;
        }
    }
    L.np_max = member_np(pl, L.G);
    const int G = L.G;
    const int nb = pl->p.n_xi + 1;
    const bool stream = !wk::kShapes[L.shape].resident;
    const bool big = wk::kShapes[L.shape].big;
    size_t o = 0;
    L.count = o; o += a256(sizeof(unsigned) * (size_t)G * nb);
    L.start = o; o += a256(sizeof(unsigned) * 2 * (size_t)G * (nb + 1));
    L.fill = o; o += a256(sizeof(unsigned) * (size_t)G * nb);
    L.order = o; o += a256(sizeof(unsigned) * 2 * (size_t)std::max<int64_t>(pl->p.n_beam, 1));
    // zeroed before every launch: progress, ticket, group counters
    L.progress = o; o += a256(sizeof(unsigned) * (size_t)std::max(n_steps, 1));
    L.ticket = o; o += 256;
    L.gctr = o; o += a256(sizeof(unsigned) * wk::kCtrPad * (size_t)(n_steps + 1));
    L.zero_end = o;
    L.plasma = o; o += stream ? a256(sizeof(double) * 4 * (size_t)L.np_max * (size_t)L.grid) : 0;
    L.big = o; o += big ? a256(wk::big_rows_bytes(pl->N1) * (size_t)L.grid) : 0;
    L.xbuf = o; o += G > 1 ? (size_t)n_steps * march_xbuf_bytes(pl->N1, G) : 0;
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

size_t wk_cycle_workspace_size(const wk_plan* plan, int32_t n_steps)
{
    if (!plan || n_steps < 1) return 0;
    return cycle_layout(plan, n_steps).total;
}

int32_t wk_cycle_group(const wk_plan* plan, int32_t n_steps)
{
    if (!plan || n_steps < 1) return 0;
    return cycle_layout(plan, n_steps).G;
}

wk_status wk_cycle(const wk_plan* plan, const wk_plasma_bufs* plasma, const wk_beam_bufs* beam, int32_t n_steps,
                   double dt, void* d_ring, void* d_workspace, size_t workspace_bytes, uint64_t* d_counters,
                   void* stream)
{
    if (!plan || !d_ring || !d_workspace || !d_counters) return fail(WK_ERR_INVALID_ARG, "NULL argument");
    if (n_steps < 1 || !std::isfinite(dt)) return fail(WK_ERR_INVALID_ARG, "bad n_steps or dt");
    wk_status st = check_plasma(plan, plasma);
    if (st != WK_OK) return st;
    st = check_beam(plan, beam);
    if (st != WK_OK) return st;
    const CycleLayout L = cycle_layout(plan, n_steps);
    if (workspace_bytes < L.total) return fail(WK_ERR_BUFFER, "cycle workspace needs %zu bytes", L.total);
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_workspace;
    const wk::GridDesc g = grid_of(plan);
    hipError_t e = wk::launch_zero_u32((unsigned*)(ws + L.progress), (int64_t)(L.zero_end - L.progress) / 4, s);
    // the exchange slots start zeroed (tag 0)
    if (e == hipSuccess && L.G > 1) e = wk::launch_zero_u32((unsigned*)(ws + L.xbuf), (int64_t)(L.total - L.xbuf) / 4, s);
    if (e != hipSuccess) return hip_status(e, "cycle init");
    e = wk::launch_beam_bins_split(g, plan->p.n_beam, L.G, *beam, (unsigned*)(ws + L.count), (unsigned*)(ws + L.start),
                                   (unsigned*)(ws + L.fill), (unsigned*)(ws + L.order), s);
    if (e != hipSuccess) return hip_status(e, "cycle binning");
    wk::CycleDesc c;
    c.base = make_desc(plan, plasma, nullptr, nullptr, d_counters);
    c.base.group = L.G;
    c.beam = *beam;
    c.grid = g;
    c.bin_start = (unsigned*)(ws + L.start);
    c.order = (unsigned*)(ws + L.order);
    c.n_beam = plan->p.n_beam;
    c.progress = (unsigned*)(ws + L.progress);
    c.ticket = (unsigned*)(ws + L.ticket);
    c.abort_flag = (unsigned long long*)(d_counters + WK_CNT_PIPELINE_ABORT);
    c.plasma_ws = wk::kShapes[L.shape].resident ? nullptr : (double*)(ws + L.plasma);
    c.big_rows = wk::kShapes[L.shape].big ? (double*)(ws + L.big) : nullptr;
    c.xbuf = L.G > 1 ? (double*)(ws + L.xbuf) : nullptr;
    c.gctr = (unsigned*)(ws + L.gctr);
    c.ring = d_ring;
    c.slot_elems = (int64_t)4 * plan->p.n_xi * plan->N1;
    c.n_steps = n_steps;
    c.dt = dt;
    return hip_status(wk::launch_cycle(c, plan->p.prec, L.shape, L.grid, s), "cycle");
}

wk_status wk_beam_push(const wk_plan* plan, const wk_beam_bufs* beam, const void* d_fields, int32_t n_steps,
                       double dt, uint64_t* d_counters, void* stream)
{
    if (!plan || !d_fields || !d_counters) return fail(WK_ERR_INVALID_ARG, "NULL argument");
    if (n_steps < 0 || !std::isfinite(dt)) return fail(WK_ERR_INVALID_ARG, "bad n_steps or dt");
    wk_status st = check_beam(plan, beam);
    if (st != WK_OK) return st;
    return hip_status(wk::launch_beam_push(grid_of(plan), plan->p.n_beam, *beam, d_fields, plan->p.prec, n_steps, dt,
                                           (unsigned long long*)d_counters, (hipStream_t)stream),
                      "beam push");
}

wk_status wk_mean_gain(const wk_plan* plan, const wk_beam_bufs* beam, int32_t which, double* d_out,
                       void* d_workspace, void* stream)
{
    if (!plan || !d_out || !d_workspace) return fail(WK_ERR_INVALID_ARG, "NULL argument");
    wk_status st = check_beam(plan, beam);
    if (st != WK_OK) return st;
    // the partial sums sit at the end of the beam binning area
    const size_t off = plan->ws_beam_off + wk::beam_ws_bytes(plan->p.n_xi, plan->p.n_beam) - a256(sizeof(double) * 2 * 512);
    return hip_status(wk::launch_mean_gain(plan->p.n_beam, *beam, which, d_out, (char*)d_workspace + off,
                                           (hipStream_t)stream),
                      "mean gain");
}

wk_status wk_gain_histogram(const wk_plan* plan, const wk_beam_bufs* beam, int32_t which, int32_t n_bins,
                            double lo, double hi, uint64_t* d_hist, void* stream)
{
    if (!plan || !d_hist) return fail(WK_ERR_INVALID_ARG, "NULL argument");
    if (n_bins < 1 || n_bins > 4096) return fail(WK_ERR_INVALID_ARG, "n_bins must be in [1, 4096] (got %d)", n_bins);
    if (!(hi > lo) || !std::isfinite(lo) || !std::isfinite(hi))
        return fail(WK_ERR_INVALID_ARG, "the range needs finite lo < hi");
    wk_status st = check_beam(plan, beam);
    if (st != WK_OK) return st;
    return hip_status(wk::launch_gain_hist(plan->p.n_beam, *beam, which, n_bins, lo, hi,
                                           (unsigned long long*)d_hist, (hipStream_t)stream),
                      "gain histogram");
}

wk_status wk_ez_peak(const wk_plan* plan, const void* d_fields, double xi_from, double* d_out, void* stream)
{
    if (!plan || !d_fields || !d_out) return fail(WK_ERR_INVALID_ARG, "NULL argument");
    return hip_status(wk::launch_ez_peak(grid_of(plan), d_fields, plan->p.prec, xi_from, d_out, (hipStream_t)stream),
                      "ez peak");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Gradient of the witness gain (forward with recording, reverse pass)
// ---------------------------------------------------------------------------
namespace {

struct GradLayout {
    size_t plan_ws, jb, tape, ckpt, hist, fbar, jbbar, scratch, ybar, d0bar, wbar, sb0, wbar_beam, wsum, partials,
        d0_f64, w_f64;
    size_t total;
};

wk_status grad_check(const wk_plan* pl, int32_t n_steps, int32_t every)
{
    if (!pl) return fail(WK_ERR_INVALID_ARG, "NULL plan");
    if (pl->p.n_bunch != 2 || pl->p.n_beam <= 0)
        return fail(WK_ERR_UNSUPPORTED, "the gradient needs a two-bunch beam of macroparticles");
    if (n_steps < 0) return fail(WK_ERR_INVALID_ARG, "n_steps must be >= 0");
    if (every < 1) return fail(WK_ERR_INVALID_ARG, "checkpoint interval must be >= 1");
    if (wk::adjoint_lds_bytes(pl->N1) > 159 * 1024)
        return fail(WK_ERR_UNSUPPORTED, "n_r = %d is too large for the reverse march (LDS)", pl->N);
    return WK_OK;
}

GradLayout grad_layout(const wk_plan* pl, int32_t n_steps, int32_t every)
{
    GradLayout L;
    const size_t d = sizeof(double);
    const int64_t np = pl->np, nb = pl->p.n_beam;
    const size_t nxn = (size_t)pl->p.n_xi * pl->N1;
    const int64_t nck = (pl->p.n_xi - 1) / every + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += a256(bytes);
        return at;
    };
    L.plan_ws = take(pl->sizes.workspace);
    L.jb = take(d * nxn);
    L.tape = take(d * wk::adjoint_tape_doubles(pl->p.n_xi, pl->N1));
    L.ckpt = take(d * (size_t)nck * 4 * np);
    L.hist = take(d * (size_t)(n_steps + 1) * 6 * nb);
    L.fbar = take(d * 4 * nxn);
    L.jbbar = take(d * nxn);
    L.scratch = take(d * wk::adjoint_scratch_doubles(np, every, pl->threads));
    L.ybar = take(d * 4 * np);
    L.d0bar = take(d * np);
    L.wbar = take(d * np);
    L.sb0 = take(d * 6 * nb);
    L.wbar_beam = take(d * nb);
    L.wsum = take(d);
    L.partials = take(d * wk::theta_partials_doubles());
    L.d0_f64 = take(pl->p.prec == WK_FP64 ? 0 : d * np);
    L.w_f64 = take(pl->p.prec == WK_FP64 ? 0 : d * np);
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

size_t wk_gradient_workspace_size(const wk_plan* plan, int32_t n_steps, int32_t every)
{
    if (grad_check(plan, n_steps, every) != WK_OK) return 0;
    return grad_layout(plan, n_steps, every).total;
}

wk_status wk_gradient_forward(const wk_plan* plan, const wk_plasma_bufs* plasma, const double* d_plasma_draws,
                              const wk_beam_bufs* beam, const double* d_beam_draws, int32_t n_steps, double dt,
                              int32_t every, void* d_fields, double* d_out, void* d_workspace, size_t workspace_bytes,
                              uint64_t* d_counters, void* stream)
{
    wk_status st = grad_check(plan, n_steps, every);
    if (st != WK_OK) return st;
    if (!d_fields || !d_out || !d_workspace || !d_counters || !d_beam_draws)
        return fail(WK_ERR_INVALID_ARG, "NULL argument");
    if (plan->p.u_th > 0.0 && !d_plasma_draws) return fail(WK_ERR_INVALID_ARG, "warm plasma needs draws");
    if (!std::isfinite(dt)) return fail(WK_ERR_INVALID_ARG, "dt must be finite");
    if ((st = check_plasma(plan, plasma)) != WK_OK) return st;
    if ((st = check_beam(plan, beam)) != WK_OK) return st;
    const GradLayout L = grad_layout(plan, n_steps, every);
    if (workspace_bytes < L.total) return fail(WK_ERR_BUFFER, "gradient workspace needs %zu bytes", L.total);
    char* ws = (char*)d_workspace;
    hipStream_t s = (hipStream_t)stream;
    const wk::GridDesc g = grid_of(plan);
    double* jb = (double*)(ws + L.jb);
    hipError_t e = wk::launch_init_beam(g, plan->p, *beam, d_beam_draws, s);
    if (e == hipSuccess)
        e = wk::launch_beam_current(g, plan->p.n_beam, *beam, jb, ws + L.plan_ws + plan->ws_beam_off,
                                    (unsigned long long*)d_counters, s);
    if (e == hipSuccess)
        e = wk::launch_init_plasma(g, plan->p.ppc, plan->p.u_th, plan->p.n0, plan->p.prec, *plasma, d_plasma_draws, s);
    if (e != hipSuccess) return hip_status(e, "gradient forward (load)");
    // the recording march by a group (the plan's, else the larger of a plain
    // response's and one workgroup per `threads` particles, at most 8: the
    // recording march keeps every moment row, so more members pay off
    // sooner), its exchange rows and counter in the plan workspace's march
    // region (zeroed per launch)
    wk::MarchDesc md = make_desc(plan, plasma, jb, d_fields, d_counters);
    md.group = plan->group > 0
                   ? single_group(plan)
                   : std::max(single_group(plan),
                              (int)std::min<int64_t>({8, (int64_t)plan->N,
                                                      (plan->np + plan->threads - 1) / plan->threads}));
    char* region = ws + L.plan_ws;
    md.xbuf = (double*)(region + march_grow_bytes(plan, wk::kMaxGroup));
    md.gctr = (unsigned*)(region + march_grow_bytes(plan, wk::kMaxGroup) + march_xbuf_bytes(plan->N1, wk::kMaxGroup));
    if (md.group > 1)
        e = wk::launch_zero_u32((unsigned*)md.xbuf, (int64_t)march_xbuf_bytes(plan->N1, md.group) / 4, s);
    if (e == hipSuccess) e = wk::launch_zero_u32(md.gctr, 1, s);
    if (e == hipSuccess)
        e = wk::launch_march_record(md, plan->p.prec, plan->threads, (double*)(ws + L.tape), (double*)(ws + L.ckpt),
                                    every, s);
    if (e != hipSuccess) return hip_status(e, "gradient forward (march)");
    e = wk::launch_push_record(g, plan->p.n_beam, *beam, d_fields, plan->p.prec, n_steps, dt,
                               (double*)(ws + L.hist), (unsigned long long*)d_counters, s);
    const size_t gain_off = L.plan_ws + plan->ws_beam_off + wk::beam_ws_bytes(plan->p.n_xi, plan->p.n_beam) -
                            a256(sizeof(double) * 2 * 512);
    if (e == hipSuccess) e = wk::launch_mean_gain(plan->p.n_beam, *beam, 1, d_out, ws + gain_off, s);
    return hip_status(e, "gradient forward (push)");
}

wk_status wk_gradient_backward(const wk_plan* plan, const wk_plasma_bufs* plasma, const double* d_plasma_draws,
                               const wk_beam_bufs* beam, const double* d_beam_draws, int32_t n_steps, double dt,
                               int32_t every, const void* d_fields, const double* d_gbar, double* d_grad,
                               void* d_workspace, size_t workspace_bytes, void* stream)
{
    wk_status st = grad_check(plan, n_steps, every);
    if (st != WK_OK) return st;
    if (!d_fields || !d_gbar || !d_grad || !d_workspace || !d_beam_draws)
        return fail(WK_ERR_INVALID_ARG, "NULL argument");
    if (plan->p.u_th > 0.0 && !d_plasma_draws) return fail(WK_ERR_INVALID_ARG, "warm plasma needs draws");
    if ((st = check_plasma(plan, plasma)) != WK_OK) return st;
    if ((st = check_beam(plan, beam)) != WK_OK) return st;
    const GradLayout L = grad_layout(plan, n_steps, every);
    if (workspace_bytes < L.total) return fail(WK_ERR_BUFFER, "gradient workspace needs %zu bytes", L.total);
    char* ws = (char*)d_workspace;
    wk::GradDesc gd;
    gd.march = make_desc(plan, plasma, nullptr, nullptr, nullptr);
    gd.march.group = plan->group;   // the reverse march's group (0: chosen from the particle count)
    gd.grid = grid_of(plan);
    gd.beam = *beam;
    gd.n_beam = plan->p.n_beam;
    gd.n_drive = plan->p.n_drive;
    gd.n_steps = n_steps;
    gd.every = every;
    gd.threads = plan->threads;
    gd.dt = dt;
    gd.n_d = plan->p.bunch[0].n_peak;
    gd.sigma_r = plan->p.sigma_r;
    gd.sigma_zd = plan->p.bunch[0].sigma_z;
    gd.u_th = plan->p.u_th;
    gd.prec = plan->p.prec;
    gd.fields = d_fields;
    gd.d0_f64 = (double*)(ws + L.d0_f64);
    gd.w_f64 = (double*)(ws + L.w_f64);
    gd.tape = (const double*)(ws + L.tape);
    gd.ckpt = (const double*)(ws + L.ckpt);
    gd.hist = (const double*)(ws + L.hist);
    gd.fbar = (double*)(ws + L.fbar);
    gd.jbbar = (double*)(ws + L.jbbar);
    gd.scratch = (double*)(ws + L.scratch);
    gd.ybar = (double*)(ws + L.ybar);
    gd.d0bar = (double*)(ws + L.d0bar);
    gd.wbar = (double*)(ws + L.wbar);
    gd.sb0 = (double*)(ws + L.sb0);
    gd.wbar_beam = (double*)(ws + L.wbar_beam);
    gd.wsum = (double*)(ws + L.wsum);
    gd.partials = (double*)(ws + L.partials);
    gd.beam_draws = d_beam_draws;
    gd.plasma_draws = d_plasma_draws;
    gd.gbar = d_gbar;
    gd.grad = d_grad;
    return hip_status(wk::launch_gradient_backward(gd, (hipStream_t)stream), "gradient backward");
}

}  // extern "C"
