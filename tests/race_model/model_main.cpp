// CPU model run of one plasma response by the device marcher (dev::Marcher)
// with one OS thread per GPU thread of a workgroup (see hip/hip_runtime.h
// beside this file).  Built by tests/test_marcher_race_model.py against a
// copy of the kernel headers, with ThreadSanitizer.  With group > 1 the
// response is marched by that many workgroups, as the march kernel splits
// it (cells [n_r g / G, n_r (g + 1) / G) to member g), each workgroup a
// child process (its own LDS) over one shared mapping of device memory, so
// that the exchanges between them run as on the device.
//
//   model <in.bin> <out.bin> <shape> [group]
//
// in.bin: int32 geom, warm, n_r, n_xi, ppc, prec; int64 np; double r_max, h,
// dxi, d_min; double x, y, px, py, d0, w [np]; nion [n_r + 1]; jb
// [n_xi][n_r + 1].  out.bin: double fields [4][n_xi][n_r + 1]; uint64
// counters [WK_NCOUNTERS]; uint64 workgroup barriers passed.
#include <pthread.h>
#include <sys/mman.h>
#include <sys/wait.h>
#include <unistd.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "wk_marcher.h"

namespace {

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

// Shared anonymous mapping (zero-filled), carved in 256-byte pieces.
template <typename V>
V* shared_take(char*& at, size_t count)
{
    V* p = (V*)at;
    at += (count * sizeof(V) + 255) & ~(size_t)255;
    return p;
}

template <typename R, int GEOM, bool WARM, int T, int K, bool RES, bool BIG>
struct Run {
    static wk::MarchDesc* desc;
    static double* smem;
    static void* pconst;
    static wk::dev::Group grp;
    static void* body(void* arg)
    {
        const long tid = (long)arg;
        threadIdx.x = (unsigned)tid;
        blockDim.x = T;
        blockIdx.x = (unsigned)grp.g;
        gridDim.x = (unsigned)grp.G;
        wk::dev::Marcher<R, GEOM, WARM, T, K, RES, BIG> m(*desc, smem, pconst, grp, grp.g == 0, true);
        m.run();
        return nullptr;
    }
    // one workgroup's threads; the number of workgroup barriers passed
    static int run_threads(unsigned long long& barriers)
    {
        wk_model::World world;
        world.block.init(T);
        for (int i = 0; i < T / 64; ++i) world.wave[i].init(64);
        wk_model::world = &world;
        std::vector<pthread_t> th(T);
        pthread_attr_t attr;
        pthread_attr_init(&attr);
        pthread_attr_setstacksize(&attr, 1 << 20);
        for (long t = 0; t < T; ++t)
            if (pthread_create(&th[t], &attr, body, (void*)t) != 0) {
                fprintf(stderr, "pthread_create failed at %ld\n", t);
                return 3;
            }
        for (int t = 0; t < T; ++t) pthread_join(th[t], nullptr);
        barriers = world.barriers;
        return 0;
    }
    // the response by G workgroups, one child process each
    static int go_group(const Input& in, int G, std::vector<double>& fields_out, unsigned long long* counters)
    {
        const int N1 = in.n_r + 1, st = wk::lds_stride(N1);
        const size_t np = (size_t)in.np, nf = (size_t)4 * in.n_xi * N1;
        const size_t bytes = (4 * np * 8 + 2 * np * sizeof(R) + nf * sizeof(R) + 8 * (WK_NCOUNTERS + 1) +
                              2 * (size_t)G * wk::kXRows * st * 8 + (size_t)G * wk::BIG_ROWS * st * 8) +
                             16 * 256;
        void* base = mmap(nullptr, bytes, PROT_READ | PROT_WRITE, MAP_SHARED | MAP_ANONYMOUS, -1, 0);
        if (base == MAP_FAILED) return 3;
        char* at = (char*)base;
        double* x = shared_take<double>(at, np);
        double* y = shared_take<double>(at, np);
        double* px = shared_take<double>(at, np);
        double* py = shared_take<double>(at, np);
        R* d0 = shared_take<R>(at, np);
        R* w = shared_take<R>(at, np);
        R* fields = shared_take<R>(at, nf);
        unsigned long long* cnt = shared_take<unsigned long long>(at, WK_NCOUNTERS + 1);
        double* xbuf = shared_take<double>(at, 2 * (size_t)G * wk::kXRows * st);
        unsigned* gctr = shared_take<unsigned>(at, 1);
        double* grow = shared_take<double>(at, (size_t)G * wk::BIG_ROWS * st);
        for (size_t i = 0; i < np; ++i) {
            x[i] = in.x[i];
            y[i] = in.y[i];
            px[i] = in.px[i];
            py[i] = in.py[i];
            d0[i] = (R)in.d0[i];
            w[i] = (R)in.w[i];
        }
        std::vector<double> lds((size_t)wk::NUM_ROWS * st + 2 * (size_t)T * K + 64, 0.0);
        fflush(nullptr);
        std::vector<pid_t> kids;
        for (int g = 0; g < G; ++g) {
            const pid_t pid = fork();
            if (pid < 0) return 3;
            if (pid > 0) {
                kids.push_back(pid);
                continue;
            }
            // member g: the particles of its cells, as the march kernel splits them
            const int c0 = (int)((int64_t)in.n_r * g / G), c1 = (int)((int64_t)in.n_r * (g + 1) / G);
            const int64_t p0 = (int64_t)c0 * in.ppc;
            wk::MarchDesc d;
            memset(&d, 0, sizeof(d));
            d.geom = in.geom;
            d.warm = in.warm;
            d.n_r = in.n_r;
            d.n_xi = in.n_xi;
            d.p0 = p0;
            d.np = (int64_t)(c1 - c0) * in.ppc;
            d.r_max = in.r_max;
            d.h = in.h;
            d.dxi = in.dxi;
            d.d_min = in.d_min;
            d.x = x + p0;
            d.y = y + p0;
            d.px = px + p0;
            d.py = py + p0;
            d.d0 = d0 + p0;
            d.w = w + p0;
            d.nion = in.nion.data();
            d.jb = in.jb.data();
            d.fields = fields;
            d.counters = cnt;
            d.grow = BIG ? grow + (size_t)g * wk::BIG_ROWS * st : nullptr;
            d.ppc = in.ppc;
            d.group = G;
            desc = &d;
            smem = lds.data();
            pconst = BIG ? nullptr : (void*)(lds.data() + (size_t)wk::NUM_ROWS * st);
            grp.G = G;
            grp.g = g;
            grp.xbuf = xbuf;
            grp.ctr = gctr;
            grp.abort = cnt + WK_CNT_PIPELINE_ABORT;
            unsigned long long barriers = 0;
            const int rc = run_threads(barriers);
            if (g == 0) cnt[WK_NCOUNTERS] = barriers;
            fflush(nullptr);
            _exit(rc);
        }
        int bad = 0;
        for (pid_t pid : kids) {
            int status = 0;
            if (waitpid(pid, &status, 0) != pid || !WIFEXITED(status) || WEXITSTATUS(status) != 0) bad = 4;
        }
        if (bad) return bad;
        fields_out.assign(fields, fields + nf);
        for (int i = 0; i <= WK_NCOUNTERS; ++i) counters[i] = cnt[i];
        return cnt[WK_CNT_PIPELINE_ABORT] ? 5 : 0;
    }
    static int go(const Input& in, int G, std::vector<double>& fields_out, unsigned long long* counters)
    {
        if ((in.geom == WK_CYL) != (GEOM == WK_CYL) || (in.warm != 0) != WARM) return 2;
        if ((in.prec == WK_FP64) != (sizeof(R) == 8)) return 2;
        if (G > 1) return go_group(in, G, fields_out, counters);
        const int N1 = in.n_r + 1, st = wk::lds_stride(N1);
        const size_t np = (size_t)in.np;
        std::vector<double> x = in.x, y = in.y, px = in.px, py = in.py;
        std::vector<R> d0(np), w(np);
        for (size_t i = 0; i < np; ++i) {
            d0[i] = (R)in.d0[i];
            w[i] = (R)in.w[i];
        }
        std::vector<R> fields((size_t)4 * in.n_xi * N1, (R)0);
        std::vector<double> lds((size_t)wk::NUM_ROWS * st + 2 * (size_t)T * K + 64, 0.0);
        std::vector<double> grow(BIG ? (size_t)wk::BIG_ROWS * st : 1, 0.0);
        wk::MarchDesc d;
        memset(&d, 0, sizeof(d));
        d.geom = in.geom;
        d.warm = in.warm;
        d.n_r = in.n_r;
        d.n_xi = in.n_xi;
        d.np = in.np;
        d.r_max = in.r_max;
        d.h = in.h;
        d.dxi = in.dxi;
        d.d_min = in.d_min;
        d.x = x.data();
        d.y = y.data();
        d.px = px.data();
        d.py = py.data();
        d.d0 = d0.data();
        d.w = w.data();
        d.nion = in.nion.data();
        d.jb = in.jb.data();
        d.fields = fields.data();
        d.counters = counters;
        d.grow = BIG ? grow.data() : nullptr;
        d.ppc = in.ppc;
        d.group = 1;
        desc = &d;
        smem = lds.data();
        pconst = BIG ? nullptr : (void*)(lds.data() + (size_t)wk::NUM_ROWS * st);
        grp = wk::dev::Group();
        unsigned long long barriers = 0;
        const int rc = run_threads(barriers);
        if (rc != 0) return rc;
        fields_out.assign(fields.begin(), fields.end());
        counters[WK_NCOUNTERS] = barriers;
        return 0;
    }
};
template <typename R, int GEOM, bool WARM, int T, int K, bool RES, bool BIG>
wk::MarchDesc* Run<R, GEOM, WARM, T, K, RES, BIG>::desc = nullptr;
template <typename R, int GEOM, bool WARM, int T, int K, bool RES, bool BIG>
double* Run<R, GEOM, WARM, T, K, RES, BIG>::smem = nullptr;
template <typename R, int GEOM, bool WARM, int T, int K, bool RES, bool BIG>
void* Run<R, GEOM, WARM, T, K, RES, BIG>::pconst = nullptr;
template <typename R, int GEOM, bool WARM, int T, int K, bool RES, bool BIG>
wk::dev::Group Run<R, GEOM, WARM, T, K, RES, BIG>::grp;

typedef int (*RunFn)(const Input&, int, std::vector<double>&, unsigned long long*);
struct Entry {
    const char* name;
    RunFn fn;
};

#define WK_RUN(R, G, W, T, K, RES, BIG) Run<R, G, W, T, K, RES, BIG>::go
const Entry kEntries[] = {
    // 256 threads with one resident particle per thread (32 cells x 8 per
    // cell, warm cylindrical): the configuration in which fields once
    // differed from run to run
    {"f64-cyl-warm-256x4-res", WK_RUN(double, WK_CYL, true, 256, 4, true, false)},
    {"f64-cyl-cold-256x4-res", WK_RUN(double, WK_CYL, false, 256, 4, true, false)},
    {"f64-slab-warm-256x4-res", WK_RUN(double, WK_SLAB, true, 256, 4, true, false)},
    {"f64-cyl-warm-256x4-stream", WK_RUN(double, WK_CYL, true, 256, 4, false, false)},
    {"f64-cyl-warm-512x4-res", WK_RUN(double, WK_CYL, true, 512, 4, true, false)},
    {"f64-cyl-warm-1024x8-res", WK_RUN(double, WK_CYL, true, 1024, 8, true, false)},
    {"f64-cyl-warm-512x8-big-stream", WK_RUN(double, WK_CYL, true, 512, 8, false, true)},
    {"f32-cyl-warm-512x8-res", WK_RUN(float, WK_CYL, true, 512, 8, true, false)},
    {"f32-cyl-warm-512x8-big-res", WK_RUN(float, WK_CYL, true, 512, 8, true, true)},
};

}  // namespace

int main(int argc, char** argv)
{
    if (argc == 2 && std::string(argv[1]) == "--list") {
        for (const Entry& e : kEntries) printf("%s\n", e.name);
        return 0;
    }
    if (argc != 4 && argc != 5) {
        fprintf(stderr, "usage: model <in.bin> <out.bin> <shape> [group] | --list\n");
        return 1;
    }
    const int group = argc == 5 ? atoi(argv[4]) : 1;
    if (group < 1 || group > wk::kMaxGroup) return 1;
    Input in;
    if (!read_input(argv[1], in)) {
        fprintf(stderr, "cannot read %s\n", argv[1]);
        return 1;
    }
    for (const Entry& e : kEntries) {
        if (std::string(e.name) != argv[3]) continue;
        std::vector<double> fields;
        unsigned long long counters[WK_NCOUNTERS + 1] = {0};
        const int rc = e.fn(in, group, fields, counters);
        if (rc != 0) {
            fprintf(stderr, "shape %s does not fit the input (rc %d)\n", e.name, rc);
            return rc;
        }
        FILE* f = fopen(argv[2], "wb");
        if (!f) return 1;
        fwrite(fields.data(), 8, fields.size(), f);
        fwrite(counters, 8, WK_NCOUNTERS + 1, f);
        fclose(f);
        return 0;
    }
    fprintf(stderr, "unknown shape %s\n", argv[3]);
    return 1;
}
