// CPU model run of the gradient's plasma part (wk_adjoint.hip): the recording
// forward march, then the reverse march seeded by a given adjoint of the
// stored fields, each as one workgroup of 256 threads with one OS thread per
// GPU thread; see hip/hip_runtime.h beside this file.  Built by
// tests/test_marcher_race_model.py against a copy of the kernel sources, with
// ThreadSanitizer.
//
//   model_adjoint <in.bin> <fbar.bin> <out.bin> <every>
//
// in.bin as for model_main.cpp (FP64 only); fbar.bin: double [4][n_xi][n_r +
// 1].  out.bin: double fields [4][n_xi][n_r + 1] of the forward, jbbar
// [n_xi][n_r + 1], ybar [4][np] (x, y, px, py), d0bar [np], wbar [np].
#include <pthread.h>

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
    wk::k_march_record<double, GEOM, WARM, kT, true>(g_md, g_tape, g_ckpt, g_every);
    return nullptr;
}

template <int GEOM, bool WARM>
void* reverse(void* arg)
{
    threadIdx.x = (unsigned)(long)arg;
    blockDim.x = kT;
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

}  // namespace

int main(int argc, char** argv)
{
    if (argc != 5) {
        fprintf(stderr, "usage: model_adjoint <in.bin> <fbar.bin> <out.bin> <every>\n");
        return 1;
    }
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
    // recording forward march
    std::vector<double> x = in.x, y = in.y, px = in.px, py = in.py;
    std::vector<double> fields((size_t)4 * nxi * N1, 0.0);
    std::vector<double> tape(wk::adjoint_tape_doubles(nxi, N1), 0.0);
    const int nck = (nxi - 1) / every + 1;
    std::vector<double> ckpt((size_t)nck * 4 * np, 0.0);
    unsigned long long counters[WK_NCOUNTERS] = {0};
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
    d.x = x.data();
    d.y = y.data();
    d.px = px.data();
    d.py = py.data();
    d.d0 = in.d0.data();
    d.w = in.w.data();
    d.nion = in.nion.data();
    d.jb = in.jb.data();
    d.fields = fields.data();
    d.counters = counters;
    d.ppc = in.ppc;
    d.group = 1;
    g_tape = tape.data();
    g_ckpt = ckpt.data();
    g_every = every;
    wk_model::dynamic_lds = lds.data();
    const bool cyl = in.geom == WK_CYL;
    run_threads(cyl ? (in.warm ? record<WK_CYL, true> : record<WK_CYL, false>)
                    : (in.warm ? record<WK_SLAB, true> : record<WK_SLAB, false>));
    // reverse march
    wk::AdjDesc& a = g_ad;
    memset(&a, 0, sizeof(a));
    a.n_r = in.n_r;
    a.n_xi = nxi;
    a.every = every;
    a.np = np;
    a.kp = (int)((np + kT - 1) / kT);
    // one member (the model runs one workgroup): no exchanges
    a.group = 1;
    a.np_m = np;
    a.r_max = in.r_max;
    a.h = in.h;
    a.dxi = in.dxi;
    a.d_min = in.d_min;
    a.d0 = in.d0.data();
    a.w = in.w.data();
    a.tape = tape.data();
    a.ckpt = ckpt.data();
    a.fbar = fbar.data();
    std::vector<double> jbbar((size_t)nxi * N1, 0.0), scratch(wk::adjoint_scratch_doubles(np, every, kT), 0.0);
    std::vector<double> ybar((size_t)4 * np, 0.0), d0bar(np, 0.0), wbar(np, 0.0);
    a.jbbar = jbbar.data();
    a.scratch = scratch.data();
    a.member_doubles = ((int64_t)every * 4 + 20) * a.kp * kT;
    std::vector<unsigned long long> abort_flag(1, 0ull);
    a.xbuf = nullptr;
    a.abort = abort_flag.data();
    a.ybar_out = ybar.data();
    a.d0bar_out = d0bar.data();
    a.wbar_out = wbar.data();
    std::vector<double> lds2(wk::adjoint_lds_bytes(N1) / sizeof(double), 0.0);
    wk_model::dynamic_lds = lds2.data();
    run_threads(cyl ? (in.warm ? reverse<WK_CYL, true> : reverse<WK_CYL, false>)
                    : (in.warm ? reverse<WK_SLAB, true> : reverse<WK_SLAB, false>));
    FILE* f = fopen(argv[3], "wb");
    if (!f) return 1;
    fwrite(fields.data(), 8, fields.size(), f);
    fwrite(jbbar.data(), 8, jbbar.size(), f);
    fwrite(ybar.data(), 8, ybar.size(), f);
    fwrite(d0bar.data(), 8, d0bar.size(), f);
    fwrite(wbar.data(), 8, wbar.size(), f);
    fclose(f);
    return 0;
}
