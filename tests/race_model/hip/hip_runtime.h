// CPU model of the HIP device environment for the marcher's barrier-schedule
// check (tests/test_marcher_race_model.py): one OS thread per GPU thread of
// one workgroup, workgroup barriers and wavefront-synchronous cross-lane
// operations as thread barriers, LDS and global memory as ordinary shared
// memory.  Run under ThreadSanitizer, any pair of accesses to the same
// address by two threads that no barrier orders (one of them a write) is a
// reported race.  Device code only; nothing here runs on a GPU.
#pragma once

#include <pthread.h>
#include <stdint.h>
#include <string.h>
#include <time.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

using std::isfinite;

// the integer min / max of the device library
template <typename A, typename B>
inline typename std::common_type<A, B>::type min(A a, B b)
{
    return b < a ? b : a;
}
template <typename A, typename B>
inline typename std::common_type<A, B>::type max(A a, B b)
{
    return a < b ? b : a;
}

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static

typedef int hipError_t;
typedef void* hipStream_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };

struct WkModelIdx {
    unsigned x, y, z;
};
inline thread_local WkModelIdx threadIdx = {0, 0, 0};
inline thread_local WkModelIdx blockIdx = {0, 0, 0};
inline thread_local WkModelIdx blockDim = {1, 1, 1};
inline thread_local WkModelIdx gridDim = {1, 1, 1};

#define __HIP_MEMORY_SCOPE_AGENT 3

namespace wk_model {

// Barrier of n threads (a barrier that some thread never reaches leaves the
// run hanging; the test's time limit reports it).
struct Barrier {
    pthread_barrier_t b;
    void init(int n) { pthread_barrier_init(&b, nullptr, (unsigned)n); }
    void wait(const char*) { pthread_barrier_wait(&b); }
};

struct World {
    Barrier block;
    Barrier wave[16];
    int64_t xlane[16][64];      // cross-lane exchange, one slot per lane
    unsigned long long barriers = 0;
};
inline World* world = nullptr;

inline void block_barrier()
{
    world->block.wait("workgroup barrier");
    if (threadIdx.x == 0) __atomic_add_fetch(&world->barriers, 1ull, __ATOMIC_RELAXED);
}

// Every lane of the wavefront publishes v; returns the wavefront's values
// through `out` after all 64 lanes have arrived; a second barrier keeps the
// slots until every lane has read them.
inline int64_t lane_of(int64_t v, int src)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    world->xlane[w][l] = v;
    world->wave[w].wait("cross-lane operation");
    const int64_t r = world->xlane[w][src & 63];
    world->wave[w].wait("cross-lane operation (read)");
    (void)l;
    return r;
}

// DPP row operations of the wavefront prefix sums (row_shr:1,2,4,8 and
// row_bcast:15/31), with the row mask; lanes without a valid source keep
// `old` (bound_ctrl off).
inline int update_dpp(int old, int src, int ctrl, int row_mask, int, bool)
{
    const int l = threadIdx.x & 63, row = l >> 4, inrow = l & 15;
    int from = -1;
    if (ctrl >= 0x111 && ctrl <= 0x11f) {
        const int n = ctrl - 0x110;
        if (inrow >= n) from = l - n;
    } else if (ctrl == 0x142) {
        if (row >= 1) from = (row - 1) * 16 + 15;
    } else if (ctrl == 0x143) {
        if (row >= 2) from = 31;
    } else {
        fprintf(stderr, "MODEL: DPP control 0x%x not modelled\n", ctrl);
        abort();
    }
    const int64_t v = lane_of((int64_t)src, from < 0 ? l : from);
    if (!((row_mask >> row) & 1)) return old;
    return from < 0 ? old : (int)v;
}

inline int ds_bpermute(int addr, int src) { return (int)lane_of((int64_t)src, (addr >> 2) & 63); }

// Dynamic LDS of the modelled workgroup (kernels' extern __shared__ arrays).
inline double* dynamic_lds = nullptr;

inline void wait_vm() {}
inline void wait_lgkm() {}
inline void compiler_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

inline unsigned long long clock64()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (unsigned long long)ts.tv_sec * 100000000ull + (unsigned long long)ts.tv_nsec / 10ull;
}

}  // namespace wk_model

inline void __syncthreads() { wk_model::block_barrier(); }
inline double __shfl_xor(double v, int mask, int = 64)
{
    int64_t u;
    memcpy(&u, &v, 8);
    u = wk_model::lane_of(u, (int)(threadIdx.x & 63) ^ mask);
    double r;
    memcpy(&r, &u, 8);
    return r;
}

template <typename V>
inline V __shfl_up(V v, unsigned delta, int = 64)
{
    static_assert(sizeof(V) <= 8, "shuffled value");
    int64_t u = 0;
    memcpy(&u, &v, sizeof(V));
    const int l = (int)(threadIdx.x & 63);
    u = wk_model::lane_of(u, l >= (int)delta ? l - (int)delta : l);
    V r;
    memcpy(&r, &u, sizeof(V));
    return r;
}

// Host launch interface seen by kernel sources (the model calls the device
// code directly and never launches).
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
enum { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
inline hipError_t hipFuncSetAttribute(const void*, int, int) { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
#define hipLaunchKernelGGL(...) ((void)0)
#define __builtin_amdgcn_s_barrier() wk_model::block_barrier()
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) wk_model::update_dpp(old, src, ctrl, rm, bm, bc)
#define __builtin_amdgcn_ds_bpermute(addr, src) wk_model::ds_bpermute(addr, src)
#define __builtin_amdgcn_s_sleep(n) ((void)0)
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))
#define __builtin_amdgcn_sqrtf(x) std::sqrt((float)(x))
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
inline unsigned long long wall_clock64() { return wk_model::clock64(); }

inline int __double2loint(double v)
{
    uint64_t u;
    memcpy(&u, &v, 8);
    return (int)(uint32_t)u;
}
inline int __double2hiint(double v)
{
    uint64_t u;
    memcpy(&u, &v, 8);
    return (int)(uint32_t)(u >> 32);
}
inline double __hiloint2double(int hi, int lo)
{
    const uint64_t u = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    double v;
    memcpy(&v, &u, 8);
    return v;
}
inline long long __double_as_longlong(double v)
{
    long long u;
    memcpy(&u, &v, 8);
    return u;
}
inline double __longlong_as_double(long long u)
{
    double v;
    memcpy(&v, &u, 8);
    return v;
}

template <typename F>
inline F atomic_add_float(F* p, F v)
{
    F old, want;
    __atomic_load(p, &old, __ATOMIC_RELAXED);
    do {
        want = old + v;
    } while (!__atomic_compare_exchange(p, &old, &want, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED));
    return old;
}
inline double atomicAdd(double* p, double v) { return atomic_add_float(p, v); }
inline float atomicAdd(float* p, float v) { return atomic_add_float(p, v); }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v)
{
    return __atomic_fetch_add(p, v, __ATOMIC_RELAXED);
}
inline unsigned atomicAdd(unsigned* p, unsigned v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }

template <typename V>
inline V __hip_atomic_load(V* p, int order, int)
{
    V v;
    __atomic_load(p, &v, order);
    return v;
}
template <typename V>
inline void __hip_atomic_store(V* p, V v, int order, int)
{
    __atomic_store(p, &v, order);
}
template <typename V>
inline V __hip_atomic_fetch_add(V* p, V v, int order, int)
{
    return __atomic_fetch_add(p, v, order);
}
