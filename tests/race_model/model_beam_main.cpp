// CPU model run of the macroparticle beam current's ordering and row kernels
// (wk_beam.hip: k_bin_sort, one workgroup of 1024 threads per xi cell, and
// k_beam_rows, one workgroup of 256 threads per slice) with one OS thread per
// GPU thread; see hip/hip_runtime.h beside this file.  The binning itself is
// done here on the host, with each cell's slots handed out in reverse index
// order, as a scheduling-dependent scatter might.  Built by
// tests/test_marcher_race_model.py against a copy of the kernel sources, with
// ThreadSanitizer.
//
//   model_beam <in.bin> <out.bin>
//
// in.bin: int32 geom, n_r, n_xi; int64 n; double r_max, h, xi_min, dxi;
// double x, y, xi, w [n].  out.bin: uint32 start [n_xi + 1]; uint32 order
// [start[n_xi]]; double jb [n_xi][n_r + 1].
#include <pthread.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "wk_beam.hip"

namespace {

wk::GridDesc g_grid;
wk_beam_bufs g_beam;
const unsigned* g_start;
unsigned* g_order;
unsigned* g_tmp;
double* g_jb;
int g_block;

void* sort_body(void* arg)
{
    threadIdx.x = (unsigned)(long)arg;
    blockDim.x = wk::kSortT;
    blockIdx.x = (unsigned)g_block;
    wk::k_bin_sort(g_start, g_order, g_tmp);
    return nullptr;
}

void* rows_body(void* arg)
{
    threadIdx.x = (unsigned)(long)arg;
    blockDim.x = wk::kBlock;
    blockIdx.x = (unsigned)g_block;
    wk::k_beam_rows(g_grid, g_beam, g_start, g_order, g_jb);
    return nullptr;
}

void run_block(void* (*fn)(void*), int threads, int block)
{
    g_block = block;
    wk_model::World* world = new wk_model::World();
    world->block.init(threads);
    for (int i = 0; i < threads / 64; ++i) world->wave[i].init(64);
    wk_model::world = world;
    std::vector<pthread_t> th(threads);
    pthread_attr_t attr;
    pthread_attr_init(&attr);
    pthread_attr_setstacksize(&attr, 1 << 20);
    for (long t = 0; t < threads; ++t)
        if (pthread_create(&th[t], &attr, fn, (void*)t) != 0) abort();
    for (int t = 0; t < threads; ++t) pthread_join(th[t], nullptr);
    delete world;
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc != 3) return 1;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 1;
    int32_t hdr[3];
    int64_t n;
    double c[4];
    if (fread(hdr, 4, 3, f) != 3 || fread(&n, 8, 1, f) != 1 || fread(c, 8, 4, f) != 4) return 1;
    std::vector<double> x(n), y(n), xi(n), w(n), zero(n, 0.0);
    if (fread(x.data(), 8, n, f) != (size_t)n || fread(y.data(), 8, n, f) != (size_t)n ||
        fread(xi.data(), 8, n, f) != (size_t)n || fread(w.data(), 8, n, f) != (size_t)n)
        return 1;
    fclose(f);
    wk::GridDesc& g = g_grid;
    g.geom = hdr[0];
    g.n_r = hdr[1];
    g.n_xi = hdr[2];
    g.r_max = c[0];
    g.h = c[1];
    g.xi_min = c[2];
    g.dxi = c[3];
    const int nxi = g.n_xi, N1 = g.n_r + 1;
    // host binning (the cell test of the scatter kernel), slots of a cell in
    // reverse index order
    std::vector<int> cell(n);
    std::vector<unsigned> count(nxi, 0), start(nxi + 1, 0);
    const double xi_max = g.xi_min + nxi * g.dxi;
    for (int64_t i = 0; i < n; ++i) {
        const double r = g.geom == WK_CYL ? std::sqrt(x[i] * x[i] + y[i] * y[i]) : std::fabs(x[i]);
        int k = -1;
        if (!(r > g.r_max || xi[i] < g.xi_min || xi[i] >= xi_max)) {
            k = (int)std::floor((xi[i] - g.xi_min) / g.dxi);
            if (k > nxi - 1) k = nxi - 1;
        }
        cell[i] = k;
        if (k >= 0) ++count[k];
    }
    for (int k = 0; k < nxi; ++k) start[k + 1] = start[k] + count[k];
    std::vector<unsigned> order(start[nxi] > 0 ? start[nxi] : 1), tmp(order.size());
    std::vector<unsigned> fill(start.begin(), start.end() - 1);
    for (int64_t i = n - 1; i >= 0; --i)
        if (cell[i] >= 0) order[fill[cell[i]]++] = (unsigned)i;
    std::vector<double> jb((size_t)nxi * N1, 0.0);
    memset(&g_beam, 0, sizeof(g_beam));
    g_beam.d_x = x.data();
    g_beam.d_y = y.data();
    g_beam.d_xi = xi.data();
    g_beam.d_w = w.data();
    g_beam.d_px = zero.data();
    g_beam.d_py = zero.data();
    g_beam.d_pz = zero.data();
    g_start = start.data();
    g_order = order.data();
    g_tmp = tmp.data();
    g_jb = jb.data();
    for (int k = 0; k < nxi; ++k) run_block(sort_body, wk::kSortT, k);
    const size_t lds = sizeof(double) * (((N1 + 1) & ~1) + 2 * wk::kRowChunk) + sizeof(int) * wk::kRowChunk;
    std::vector<double> ldsbuf(lds / sizeof(double) + 1, 0.0);
    wk_model::dynamic_lds = ldsbuf.data();
    for (int k = 0; k < nxi; ++k) run_block(rows_body, wk::kBlock, k);
    f = fopen(argv[2], "wb");
    if (!f) return 1;
    fwrite(start.data(), 4, start.size(), f);
    fwrite(order.data(), 4, start[nxi], f);
    fwrite(jb.data(), 8, jb.size(), f);
    fclose(f);
    return 0;
}
