// Roofline denominators measured on the device the scan runs on (gfx950):
// the peaks that bound the scan's kernels, taken with the simplest kernels
// that reach them.
//
//   HBM copy / write-only / read-only   bytes per second over a buffer far
//                                        larger than the caches
//   LDS ds_read_b32                      dword reads per second, lanes of a
//                                        wave on distinct banks or on random
//                                        addresses (the scan's table lookups)
//   random gather from L2 / MALL         dword loads per second from random
//                                        addresses of a table of given size
//   dependent-load latency               one chain of loads whose address is
//                                        the previous load's value, in LDS or
//                                        in global memory (a table of given
//                                        size): nanoseconds per step, the
//                                        cost of one step of the scan's walk
//
// Every entry point launches its kernel `reps` times back to back after one
// warm-up launch and returns the mean time per launch from HIP events.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ac_microbench.h"

namespace {

#define MB_OK(x)                       \
    do {                               \
        if ((x) != hipSuccess) {       \
            (void)hipGetLastError();   \
            return ACB_E_HIP;          \
        }                              \
    } while (0)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kThreads = 256;

// HBM kernels: every block moves one contiguous 4 KiB piece (16 bytes per
// thread) and exits, with a grid that covers the buffer.  Short-lived blocks
// that each touch a few KiB reach higher HBM rates on this device than
// persistent waves looping over the buffer (measured: 6.9 against 4.4-5.4
// TB/s for writes).
constexpr uint32_t kPiece = kThreads * 16;

__global__ __launch_bounds__(kThreads) void k_copy(const u32x4 *__restrict__ src,
                                                   u32x4 *__restrict__ dst, uint64_t n16) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ __launch_bounds__(kThreads) void k_write(u32x4 *__restrict__ dst, uint64_t n16,
                                                    uint32_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    const u32x4 x = {v, v + 1, v + 2, (uint32_t)i};
    if (i < n16) *(dst + i) = x;
}

__global__ __launch_bounds__(kThreads) void k_read(const u32x4 *__restrict__ src, uint64_t n16,
                                                   uint32_t *__restrict__ sink) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    u32x4 a = {0, 0, 0, 0};
    if (i < n16) a = __builtin_nontemporal_load(src + i);
    const uint32_t r = a.x ^ a.y ^ a.z ^ a.w;
    if (r == 0x9E3779B9u) sink[0] = r;  // keeps the loads; practically never taken
}

__device__ __forceinline__ uint32_t mix(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

// LDS reads: 1024 threads, a 64 KiB table; per iteration each lane forms one
// address and reads 16 dwords at fixed distances from it (immediate offsets,
// so the address arithmetic is amortised).  Conflict-free: the lanes of a
// wave read 64 consecutive dwords of the wave's slice (a permutation of them
// that changes every iteration), one bank per lane.  Random: the
// base dword is a fresh hash of (thread, iteration), so the 64 lanes hit
// random banks on every read.
constexpr uint32_t kLdsWords = 16384;
constexpr uint32_t kLdsReads = 16;

template <bool RANDOM>
__global__ __launch_bounds__(1024) void k_lds(uint32_t iters, uint32_t *__restrict__ sink) {
    __shared__ uint32_t t[kLdsWords];
    for (uint32_t i = threadIdx.x; i < kLdsWords; i += 1024) t[i] = mix(i);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t acc = 0;
    for (uint32_t it = 0; it < iters; ++it) {
        uint32_t base;
        // the 16 reads span base .. base + 960, inside the table for
        // base <= 15423: the conflict-free base is at most 15 * 1024 + 63, the
        // random one at most 0x3BFF = 15359
        if (RANDOM)
            base = mix(threadIdx.x * 0x10001u + it * 0x9E3779B9u) & 0x3BFFu;
        else
            base = wave * 1024 + (lane ^ (it & 63));
#pragma unroll
        for (uint32_t k = 0; k < kLdsReads; ++k) acc += t[base + 64 * k];
    }
    if (acc == 0x9E3779B9u) sink[0] = acc;
}

// Random gathers: every lane issues 8 independent loads per iteration from
// random dwords of the table (entries a power of two).
constexpr uint32_t kGatherLoads = 8;

__global__ __launch_bounds__(kThreads) void k_gather(const uint32_t *__restrict__ table,
                                                     uint32_t mask, uint32_t iters,
                                                     uint32_t *__restrict__ sink) {
    const uint32_t g = blockIdx.x * kThreads + threadIdx.x;
    uint32_t acc = 0;
    for (uint32_t it = 0; it < iters; ++it) {
        uint32_t v[kGatherLoads];
        const uint32_t h = mix(g * 0x9E3779B9u + it);
#pragma unroll
        for (uint32_t k = 0; k < kGatherLoads; ++k)
            v[k] = table[(h + k * 0x3C6EF372u) * 0x2545F491u >> 3 & mask];
#pragma unroll
        for (uint32_t k = 0; k < kGatherLoads; ++k) acc += v[k];
    }
    if (acc == 0x9E3779B9u) sink[0] = acc;
}

// Dependent loads: one wave; lane l starts at element l of a random cyclic
// permutation and follows it `steps` times.  LDS variant: the permutation
// (at most 16 Ki entries) is first copied into LDS.
__global__ __launch_bounds__(64) void k_chase_global(const uint32_t *__restrict__ next,
                                                     uint32_t steps, uint32_t *__restrict__ sink) {
    uint32_t s = threadIdx.x;
    for (uint32_t i = 0; i < steps; ++i) s = next[s];
    if (s == 0xFFFFFFFFu) sink[0] = s;
}

constexpr uint32_t kChaseLds = 16384;

__global__ __launch_bounds__(64) void k_chase_lds(const uint32_t *__restrict__ next, uint32_t n,
                                                  uint32_t steps, uint32_t *__restrict__ sink) {
    __shared__ uint32_t t[kChaseLds];
    for (uint32_t i = threadIdx.x; i < n; i += 64) t[i] = next[i];
    __syncthreads();
    uint32_t s = threadIdx.x;
    for (uint32_t i = 0; i < steps; ++i) s = t[s];
    if (s == 0xFFFFFFFFu) sink[0] = s;
}

struct Ctx {
    hipStream_t st = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    uint32_t *sink = nullptr;
    uint32_t cus = 0;
};

int ctx_get(Ctx **out) {
    static Ctx c;
    static bool init = false;
    if (!init) {
        int dev = 0, v = 0;
        MB_OK(hipGetDevice(&dev));
        MB_OK(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev));
        c.cus = (uint32_t)v;
        MB_OK(hipStreamCreateWithFlags(&c.st, hipStreamNonBlocking));
        MB_OK(hipEventCreate(&c.a));
        MB_OK(hipEventCreate(&c.b));
        MB_OK(hipMalloc((void **)&c.sink, 256));
        init = true;
    }
    *out = &c;
    return ACB_OK;
}

template <typename F>
int timed(Ctx *c, int reps, F launch, double *ms) {
    if (reps < 1 || !ms) return ACB_E_INVALID;
    launch(c->st);
    MB_OK(hipGetLastError());
    MB_OK(hipEventRecord(c->a, c->st));
    for (int r = 0; r < reps; ++r) launch(c->st);
    MB_OK(hipGetLastError());
    MB_OK(hipEventRecord(c->b, c->st));
    MB_OK(hipEventSynchronize(c->b));
    float t = 0;
    MB_OK(hipEventElapsedTime(&t, c->a, c->b));
    *ms = (double)t / reps;
    return ACB_OK;
}

}  // namespace

extern "C" {

int acb_hbm_copy(void *d_dst, const void *d_src, uint64_t bytes, int reps, double *ms) {
    if (!d_dst || !d_src || bytes % 16 || !bytes || bytes / kPiece >= (1ull << 31))
        return ACB_E_INVALID;
    Ctx *c;
    int rc = ctx_get(&c);
    if (rc) return rc;
    const uint32_t grid = (uint32_t)((bytes + kPiece - 1) / kPiece);
    return timed(c, reps, [&](hipStream_t st) {
        hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kThreads), 0, st, (const u32x4 *)d_src,
                           (u32x4 *)d_dst, bytes / 16);
    }, ms);
}

int acb_hbm_write(void *d_dst, uint64_t bytes, int reps, double *ms) {
    if (!d_dst || bytes % 16 || !bytes || bytes / kPiece >= (1ull << 31)) return ACB_E_INVALID;
    Ctx *c;
    int rc = ctx_get(&c);
    if (rc) return rc;
    const uint32_t grid = (uint32_t)((bytes + kPiece - 1) / kPiece);
    return timed(c, reps, [&](hipStream_t st) {
        hipLaunchKernelGGL(k_write, dim3(grid), dim3(kThreads), 0, st, (u32x4 *)d_dst, bytes / 16,
                           7u);
    }, ms);
}

int acb_hbm_read(const void *d_src, uint64_t bytes, int reps, double *ms) {
    if (!d_src || bytes % 16 || !bytes || bytes / kPiece >= (1ull << 31)) return ACB_E_INVALID;
    Ctx *c;
    int rc = ctx_get(&c);
    if (rc) return rc;
    const uint32_t grid = (uint32_t)((bytes + kPiece - 1) / kPiece);
    return timed(c, reps, [&](hipStream_t st) {
        hipLaunchKernelGGL(k_read, dim3(grid), dim3(kThreads), 0, st, (const u32x4 *)d_src,
                           bytes / 16, c->sink);
    }, ms);
}

int acb_lds_read(int random, uint32_t iters, int reps, double *ms, uint64_t *reads) {
    if (!iters || !reads) return ACB_E_INVALID;
    Ctx *c;
    int rc = ctx_get(&c);
    if (rc) return rc;
    const uint32_t grid = c->cus;  // one 1024-thread block per compute unit
    *reads = (uint64_t)grid * 1024 * iters * kLdsReads;
    return timed(c, reps, [&](hipStream_t st) {
        if (random)
            hipLaunchKernelGGL(k_lds<true>, dim3(grid), dim3(1024), 0, st, iters, c->sink);
        else
            hipLaunchKernelGGL(k_lds<false>, dim3(grid), dim3(1024), 0, st, iters, c->sink);
    }, ms);
}

int acb_gather(const uint32_t *d_table, uint64_t entries, uint32_t iters, int reps, double *ms,
               uint64_t *reads) {
    if (!d_table || !iters || !reads || entries < 64 || entries > (1ull << 31) ||
        (entries & (entries - 1)))
        return ACB_E_INVALID;
    Ctx *c;
    int rc = ctx_get(&c);
    if (rc) return rc;
    const uint32_t grid = c->cus * 8;
    *reads = (uint64_t)grid * kThreads * iters * kGatherLoads;
    return timed(c, reps, [&](hipStream_t st) {
        hipLaunchKernelGGL(k_gather, dim3(grid), dim3(kThreads), 0, st, d_table,
                           (uint32_t)(entries - 1), iters, c->sink);
    }, ms);
}

int acb_chase(const uint32_t *d_next, uint64_t entries, int lds, uint32_t steps, int reps,
              double *ns_per_step) {
    if (!d_next || !steps || !ns_per_step || entries < 64 || entries >= (1ull << 32) ||
        (lds && entries > kChaseLds))
        return ACB_E_INVALID;
    Ctx *c;
    int rc = ctx_get(&c);
    if (rc) return rc;
    double ms = 0;
    rc = timed(c, reps, [&](hipStream_t st) {
        if (lds)
            hipLaunchKernelGGL(k_chase_lds, dim3(1), dim3(64), 0, st, d_next, (uint32_t)entries,
                               steps, c->sink);
        else
            hipLaunchKernelGGL(k_chase_global, dim3(1), dim3(64), 0, st, d_next, steps, c->sink);
    }, &ms);
    if (rc) return rc;
    *ns_per_step = ms * 1e6 / steps;
    return ACB_OK;
}

}  // extern "C"
