// CPU model run of the gradient's plasma part (wk_adjoint.hip): the recording
// forward march, then the reverse march seeded by a given adjoint of the
// stored fields, each by a group of `group` workgroups of 256 threads with
// one OS thread per GPU thread; see hip/hip_runtime.h beside this file.
// Each workgroup of a group > 1 runs in a child process of its own (its own
// LDS and __shared__ arrays), and device memory is one shared mapping that
// all of them see, so the exchanges between the workgroups run as on the
// device.  Built by tests/test_marcher_race_model.py against a copy of the
// kernel sources, with ThreadSanitizer (which checks the threads of each
// workgroup; the exchanges between processes are checked by their results).
//
//   model_adjoint <in.bin> <fbar.bin> <out.bin> <every> [group]
//
// in.bin as for model_main.cpp (FP64 only); fbar.bin: double [4][n_xi][n_r +
// 1].  out.bin: double fields [4][n_xi][n_r + 1] of the forward, jbbar
// [n_xi][n_r + 1], ybar [4][np] (x, y, px, py), d0bar [np], wbar [np].
#include <pthread.h>
#include <sys/mman.h>
#include <sys/wait.h>
#include <unistd.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "wk_adjoint.hip"

namespace {

constexpr int kT = 256;

struct Input {
    int32_t geom, warm, n_r, n_xi, ppc, prec;
    int64_t np;
    double r_max, h, dxi, d_min;
    std::vector<double> x, y, px, py, d0, w, nion, jb;
};

bool read_input(const char* path, Input& in)
{
    FILE* f = fopen(path, "rb");
    if (!f) return false;
    int32_t hdr[6];
    bool ok = fread(hdr, 4, 6, f) == 6 && fread(&in.np, 8, 1, f) == 1;
    double c[4];
    ok = ok && fread(c, 8, 4, f) == 4;
    if (!ok) { fclose(f); return false; }
    in.geom = hdr[0]; in.warm = hdr[1]; in.n_r = hdr[2]; in.n_xi = hdr[3]; in.ppc = hdr[4]; in.prec = hdr[5];
    in.r_max = c[0]; in.h = c[1]; in.dxi = c[2]; in.d_min = c[3];
    auto rd = [&](std::vector<double>& v, size_t n) { v.resize(n); return fread(v.data(), 8, n, f) == n; };
    const size_t np = (size_t)in.np, N1 = (size_t)in.n_r + 1;
    ok = rd(in.x, np) && rd(in.y, np) && rd(in.px, np) && rd(in.py, np) && rd(in.d0, np) && rd(in.w, np) &&
         rd(in.nion, N1) && rd(in.jb, (size_t)in.n_xi * N1);
    fclose(f);
    return ok;
}

// Device memory: one shared anonymous mapping (zero-filled), carved in
// 256-byte aligned pieces.
struct Arena {
    char* base = nullptr;
    size_t size = 0, used = 0;
    bool init(size_t n)
    {
        void* p = mmap(nullptr, n, PROT_READ | PROT_WRITE, MAP_SHARED | MAP_ANONYMOUS, -1, 0);
        if (p == MAP_FAILED) return false;
        base = (char*)p;
        size = n;
        return true;
    }
    template <typename V>
    V* take(size_t count)
    {
        const size_t bytes = (count * sizeof(V) + 255) & ~(size_t)255;
        if (used + bytes > size) abort();
        V* p = (V*)(base + used);
        used += bytes;
        return p;
    }
};

int g_rank = 0, g_group = 1;
wk::MarchDesc g_md;
double* g_tape;
double* g_ckpt;
int g_every;
wk::AdjDesc g_ad;

template <int GEOM, bool WARM>
void* record(void* arg)
{
    threadIdx.x = (unsigned)(long)arg;
    blockDim.x = kT;
    blockIdx.x = (unsigned)g_rank;
    gridDim.x = (unsigned)g_group;
    wk::k_march_record<double, GEOM, WARM, kT, true>(g_md, g_tape, g_ckpt, g_every);
    return nullptr;
}

template <int GEOM, bool WARM>
void* reverse(void* arg)
{
    threadIdx.x = (unsigned)(long)arg;
    blockDim.x = kT;
    blockIdx.x = (unsigned)g_rank;
    gridDim.x = (unsigned)g_group;
    wk::k_adjoint_march<GEOM, WARM, kT, double>(g_ad);
    return nullptr;
}

void run_threads(void* (*fn)(void*))
{
    wk_model::World* world = new wk_model::World();
    world->block.init(kT);
    for (int i = 0; i < kT / 64; ++i) world->wave[i].init(64);
    wk_model::world = world;
    std::vector<pthread_t> th(kT);
    pthread_attr_t attr;
    pthread_attr_init(&attr);
    pthread_attr_setstacksize(&attr, 1 << 20);
    for (long t = 0; t < kT; ++t)
        if (pthread_create(&th[t], &attr, fn, (void*)t) != 0) abort();
    for (int t = 0; t < kT; ++t) pthread_join(th[t], nullptr);
}

// The workgroups of a group at once: in this process for one, else one child
// process per workgroup.  False if a child failed (a race report included).
bool run_group(void* (*fn)(void*))
{
    if (g_group == 1) {
        g_rank = 0;
        run_threads(fn);
        return true;
    }
    fflush(nullptr);
    std::vector<pid_t> kids;
    for (int r = 0; r < g_group; ++r) {
        const pid_t pid = fork();
        if (pid < 0) return false;
        if (pid == 0) {
            g_rank = r;
            run_threads(fn);
            fflush(nullptr);
            _exit(0);
        }
        kids.push_back(pid);
    }
    bool ok = true;
    for (pid_t pid : kids) {
        int status = 0;
        if (waitpid(pid, &status, 0) != pid || !WIFEXITED(status) || WEXITSTATUS(status) != 0) ok = false;
    }
    return ok;
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc != 5 && argc != 6) {
        fprintf(stderr, "usage: model_adjoint <in.bin> <fbar.bin> <out.bin> <every> [group]\n");
        return 1;
    }
    g_group = argc == 6 ? atoi(argv[5]) : 1;
    if (g_group < 1 || g_group > wk::kRevMaxGroup) return 1;
    Input in;
    if (!read_input(argv[1], in) || in.prec != WK_FP64) return 1;
    const int N1 = in.n_r + 1, st = wk::lds_stride(N1), nxi = in.n_xi;
    const int64_t np = in.np;
    const int every = atoi(argv[4]);
    if (np > (int64_t)kT * wk::kRecK || every < 1) return 1;
    std::vector<double> fbar((size_t)4 * nxi * N1);
    {
        FILE* f = fopen(argv[2], "rb");
        if (!f || fread(fbar.data(), 8, fbar.size(), f) != fbar.size()) return 1;
        fclose(f);
    }
    // device memory of both marches
    Arena mem;
    const int nck = (nxi - 1) / every + 1;
    const size_t need = sizeof(double) * (8 * (size_t)np + 5 * (size_t)nxi * N1 + wk::adjoint_tape_doubles(nxi, N1) +
                                          (size_t)nck * 4 * np + wk::adjoint_scratch_doubles(np, every, kT) +
                                          2 * (size_t)wk::kMaxGroup * wk::kXRows * st) +
                        64 * 256 + (1 << 20);
    if (!mem.init(need)) return 1;
    auto copy_in = [&](const std::vector<double>& v) {
        double* p = mem.take<double>(v.size());
        std::copy(v.begin(), v.end(), p);
        return p;
    };
    // recording forward march
    double* x = copy_in(in.x);
    double* y = copy_in(in.y);
    double* px = copy_in(in.px);
    double* py = copy_in(in.py);
    double* fields = mem.take<double>((size_t)4 * nxi * N1);
    double* tape = mem.take<double>(wk::adjoint_tape_doubles(nxi, N1));
    double* ckpt = mem.take<double>((size_t)nck * 4 * np);
    unsigned long long* counters = mem.take<unsigned long long>(WK_NCOUNTERS);
    const int kr = (int)std::min<int64_t>(wk::kRecK, (np + kT - 1) / kT);
    std::vector<double> lds((size_t)wk::NUM_ROWS * st + 2 * (size_t)kT * kr + 64, 0.0);
    wk::MarchDesc& d = g_md;
    memset(&d, 0, sizeof(d));
    d.geom = in.geom;
    d.warm = in.warm;
    d.n_r = in.n_r;
    d.n_xi = nxi;
    d.np = np;
    d.r_max = in.r_max;
    d.h = in.h;
    d.dxi = in.dxi;
    d.d_min = in.d_min;
    d.x = x;
    d.y = y;
    d.px = px;
    d.py = py;
    d.d0 = in.d0.data();
    d.w = in.w.data();
    d.nion = in.nion.data();
    d.jb = in.jb.data();
    d.fields = fields;
    d.counters = counters;
    d.ppc = in.ppc;
    d.group = g_group;
    d.xbuf = mem.take<double>(2 * (size_t)g_group * wk::kXRows * st);
    d.gctr = mem.take<unsigned>(1);
    g_tape = tape;
    g_ckpt = ckpt;
    g_every = every;
    wk_model::dynamic_lds = lds.data();
    const bool cyl = in.geom == WK_CYL;
    if (!run_group(cyl ? (in.warm ? record<WK_CYL, true> : record<WK_CYL, false>)
                       : (in.warm ? record<WK_SLAB, true> : record<WK_SLAB, false>)))
        return 2;
    // reverse march
    wk::AdjDesc& a = g_ad;
    memset(&a, 0, sizeof(a));
    a.n_r = in.n_r;
    a.n_xi = nxi;
    a.every = every;
    a.np = np;
    a.group = g_group;
    a.np_m = (np + g_group - 1) / g_group;
    a.kp = (int)((a.np_m + kT - 1) / kT);
    a.r_max = in.r_max;
    a.h = in.h;
    a.dxi = in.dxi;
    a.d_min = in.d_min;
    a.d0 = in.d0.data();
    a.w = in.w.data();
    a.tape = tape;
    a.ckpt = ckpt;
    a.fbar = fbar.data();
    const size_t njb = (size_t)nxi * N1;
    double* jbbar = mem.take<double>(njb);
    double* ybar = mem.take<double>((size_t)4 * np);
    double* d0bar = mem.take<double>(np);
    double* wbar = mem.take<double>(np);
    a.member_doubles = ((int64_t)every * 4 + 20) * a.kp * kT;
    a.jbbar = jbbar;
    a.scratch = mem.take<double>(wk::adjoint_scratch_doubles(np, every, kT));
    // exchange slots and abort flag after the members' scratch, as the
    // library lays them out
    a.xbuf = a.scratch + (int64_t)a.group * a.member_doubles;
    a.abort = (unsigned long long*)(a.xbuf + 2 * (int64_t)wk::kRevMaxGroup * wk::kRevXRows * wk::kRevXStride);
    a.ybar_out = ybar;
    a.d0bar_out = d0bar;
    a.wbar_out = wbar;
    std::vector<double> lds2(wk::adjoint_lds_bytes(N1) / sizeof(double), 0.0);
    wk_model::dynamic_lds = lds2.data();
    if (!run_group(cyl ? (in.warm ? reverse<WK_CYL, true> : reverse<WK_CYL, false>)
                       : (in.warm ? reverse<WK_SLAB, true> : reverse<WK_SLAB, false>)))
        return 2;
    if (*a.abort || counters[WK_CNT_PIPELINE_ABORT]) return 3;
    FILE* f = fopen(argv[3], "wb");
    if (!f) return 1;
    fwrite(fields, 8, (size_t)4 * nxi * N1, f);
    fwrite(jbbar, 8, njb, f);
    fwrite(ybar, 8, (size_t)4 * np, f);
    fwrite(d0bar, 8, np, f);
    fwrite(wbar, 8, np, f);
    fclose(f);
    return 0;
}
