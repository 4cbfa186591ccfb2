// CPU model run of one Eq. (6)-direct response (wk_direct.hip, one
// workgroup of 256 threads) with one OS thread per GPU thread; see
// hip/hip_runtime.h beside this file.  Built by
// tests/test_marcher_race_model.py against a copy of the kernel sources, with
// ThreadSanitizer.
//
//   model_direct <in.bin> <out.bin> <iters> <tol>
//
// in.bin as for model_main.cpp (FP64 only).  out.bin: double fields
// [4][n_xi][n_r + 1]; uint64 counters [WK_NCOUNTERS]; int32 Newton steps
// [n_xi].
#include <pthread.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "wk_direct.hip"

namespace wk {
bool lds_fits(size_t bytes) { return bytes <= 159 * 1024; }
}  // namespace wk

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

wk::DirectDesc g_dd;

template <int GEOM, bool WARM>
void* body(void* arg)
{
    threadIdx.x = (unsigned)(long)arg;
    blockDim.x = wk::kDirT;
    wk::k_march_direct<GEOM, WARM>(g_dd);
    return nullptr;
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc != 5) {
        fprintf(stderr, "usage: model_direct <in.bin> <out.bin> <iters> <tol>\n");
        return 1;
    }
    Input in;
    if (!read_input(argv[1], in) || in.prec != WK_FP64) {
        fprintf(stderr, "cannot read %s (FP64 input expected)\n", argv[1]);
        return 1;
    }
    const int N1 = in.n_r + 1, st = wk::lds_stride(N1);
    const size_t np = (size_t)in.np;
    std::vector<double> fields((size_t)4 * in.n_xi * N1, 0.0);
    std::vector<double> ws(wk::direct_ws_doubles(in.np, N1), 0.0);
    std::vector<double> lds(wk::direct_lds_bytes(N1) / sizeof(double), 0.0);
    std::vector<int32_t> its(in.n_xi, 0);
    unsigned long long counters[WK_NCOUNTERS] = {0};
    wk::DirectDesc& dd = g_dd;
    memset(&dd, 0, sizeof(dd));
    wk::MarchDesc& d = dd.march;
    d.geom = in.geom;
    d.warm = in.warm;
    d.n_r = in.n_r;
    d.n_xi = in.n_xi;
    d.np = in.np;
    d.r_max = in.r_max;
    d.h = in.h;
    d.dxi = in.dxi;
    d.d_min = in.d_min;
    d.x = in.x.data();
    d.y = in.y.data();
    d.px = in.px.data();
    d.py = in.py.data();
    d.d0 = in.d0.data();
    d.w = in.w.data();
    d.nion = in.nion.data();
    d.jb = in.jb.data();
    d.fields = fields.data();
    d.counters = counters;
    d.ppc = in.ppc;
    d.group = 1;
    const size_t n4 = 4 * (size_t)(np > 0 ? np : 1);
    dd.ys = ws.data();
    dd.yn = ws.data() + n4;
    dd.f0 = ws.data() + 2 * n4;
    dd.V = ws.data() + 3 * n4;
    dd.iters = atoi(argv[3]);
    dd.tol = atof(argv[4]);
    dd.iterations = its.data();
    (void)st;
    wk_model::dynamic_lds = lds.data();
    wk_model::World world;
    world.block.init(wk::kDirT);
    for (int i = 0; i < wk::kDirT / 64; ++i) world.wave[i].init(64);
    wk_model::world = &world;
    void* (*fn)(void*) = in.geom == WK_CYL ? (in.warm ? body<WK_CYL, true> : body<WK_CYL, false>)
                                           : (in.warm ? body<WK_SLAB, true> : body<WK_SLAB, false>);
    std::vector<pthread_t> th(wk::kDirT);
    pthread_attr_t attr;
    pthread_attr_init(&attr);
    pthread_attr_setstacksize(&attr, 1 << 20);
    for (long t = 0; t < wk::kDirT; ++t)
        if (pthread_create(&th[t], &attr, fn, (void*)t) != 0) return 3;
    for (int t = 0; t < wk::kDirT; ++t) pthread_join(th[t], nullptr);
    FILE* f = fopen(argv[2], "wb");
    if (!f) return 1;
    fwrite(fields.data(), 8, fields.size(), f);
    fwrite(counters, 8, WK_NCOUNTERS, f);
    fwrite(its.data(), 4, its.size(), f);
    fclose(f);
    return 0;
}
