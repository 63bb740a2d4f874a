// solve.hip -- gfx950 kernels of the level-scheduled forward substitution
// (arXiv:2103.11445, Sec. II, Algorithm 1) over a possibly rewritten system
// L' x = b + M b (Sec. III, Fig. 3).
//
// Execution model
//   * One persistent grid of independent wave64 workers.  A worker takes the
//     next 64-lane tile from a monotone device counter (tiles are ordered by
//     level of L'), so it only ever waits on rows of tiles that running
//     workers already hold: the grid always drains.
//   * Per-row readiness instead of a barrier per level: x itself is the flag.
//     Before the solve every x_i is set to a signalling-NaN bit pattern that
//     no arithmetic result can carry (results are quiet NaNs at worst).  A
//     lane that needs x_k polls it with device-scope loads until the pattern
//     is gone; the producer publishes x_i with one device-scope 8-byte store.
//     Device (agent) scope keeps the eight XCDs' L2 caches out of the way.
//   * b-terms (the rewritten right-hand side) never wait.
//   * A wait is bounded by the GPU real-time clock; on expiry the worker
//     marks the plan's status word, which makes every other wait give up,
//     and the grid drains with NaNs.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "plan.hpp"

namespace {

constexpr unsigned long long kNotReady = 0x7FF0DEADBEEF0001ull;  // signalling NaN
constexpr int32_t kPad = INT32_MIN;
constexpr int kBlock = 256;  // 4 independent waves per workgroup

struct SolveArgs {
    const int4 *tiles;
    const int32_t *rows;
    const double *diag;
    const int32_t *tcol;
    const double *tval;
    sptrsv::Workspace *ws;
    const double *b;
    double *x;
    long long ntiles;
    unsigned long long base;
    unsigned long long wait_limit;
};

__global__ void fill_not_ready(unsigned long long *__restrict__ x, int32_t n) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        x[i] = kNotReady;
}

__device__ inline unsigned long long load_agent(const double *p) {
    return __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<double *>(p)),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Value of x[k] once it is published (or NaN if the wait gave up).
__device__ __noinline__ double wait_slow(const double *x, int32_t k, sptrsv::Workspace *ws,
                                         unsigned long long limit) {
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (unsigned it = 1;; ++it) {
        __builtin_amdgcn_s_sleep(1);
        const unsigned long long v = load_agent(x + k);
        if (v != kNotReady) return __longlong_as_double((long long)v);
        if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
            __hip_atomic_fetch_or(&ws->status, (unsigned)SPTRSV_ERR_TIMEOUT, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            return __longlong_as_double(0x7FF8000000000000ll);
        }
        if ((it & 15u) == 0 &&
            __hip_atomic_load(&ws->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            return __longlong_as_double(0x7FF8000000000000ll);
    }
}

__device__ inline double gather(const SolveArgs &a, int32_t col) {
    if (col >= 0) {
        const unsigned long long v = load_agent(a.x + col);
        if (v != kNotReady) return __longlong_as_double((long long)v);
        return wait_slow(a.x, col, a.ws, a.wait_limit);
    }
    return a.b[~col];
}

__device__ inline unsigned long long claim(sptrsv::Workspace *ws) {
    unsigned long long t = 0;
    if ((threadIdx.x & 63) == 0) t = atomicAdd(&ws->ticket, 1ull);
    return __shfl(t, 0, 64);
}

__global__ void __launch_bounds__(kBlock) solve_tiles(SolveArgs a) {
    const int lane = threadIdx.x & 63;
    unsigned long long t = claim(a.ws) - a.base;
    while (t < (unsigned long long)a.ntiles) {
        const unsigned long long tn = claim(a.ws) - a.base;  // next tile, fetched early
        const int4 d = a.tiles[t];
        const int lg = d.w & 0xff;
        const int nrows = d.w >> 8;
        const int r = lane >> lg;
        const bool active = r < nrows;
        double acc = 0.0;
        if (active) {
            const int32_t *col = a.tcol + (size_t)d.x * 64 + lane;
            const double *val = a.tval + (size_t)d.x * 64 + lane;
            for (int c = 0; c < d.z; ++c) {
                const int32_t k = col[(size_t)c * 64];
                if (k == kPad) continue;
                acc = fma(val[(size_t)c * 64], gather(a, k), acc);
            }
        }
        for (int off = (1 << lg) >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (active && (lane & ((1 << lg) - 1)) == 0) {
            const int32_t slot = d.y + r;
            const int32_t row = a.rows[slot];
            const double xi = (a.b[row] + acc) / a.diag[slot];
            __hip_atomic_store(reinterpret_cast<unsigned long long *>(a.x) + row,
                               (unsigned long long)__double_as_longlong(xi), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        t = tn;
    }
}

}  // namespace

extern "C" int sptrsv_device_waves(int *waves) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    *waves = cus * 8;  // two 4-wave workgroups per CU
    return 0;
}

extern "C" int sptrsv_launch_solve(const unsigned char *dev, const sptrsv::Layout *lay, int32_t n,
                                   int64_t ntiles, int waves, unsigned long long ticket_base,
                                   uint64_t wait_limit, const double *b, double *x, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int fill_blocks = (int)std::min<int64_t>(2048, ((int64_t)n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(fill_not_ready, dim3(fill_blocks), dim3(kBlock), 0, s,
                       reinterpret_cast<unsigned long long *>(x), n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    SolveArgs a;
    a.tiles = reinterpret_cast<const int4 *>(dev + lay->tiles);
    a.rows = reinterpret_cast<const int32_t *>(dev + lay->rows);
    a.diag = reinterpret_cast<const double *>(dev + lay->diag);
    a.tcol = reinterpret_cast<const int32_t *>(dev + lay->tcol);
    a.tval = reinterpret_cast<const double *>(dev + lay->tval);
    a.ws = reinterpret_cast<sptrsv::Workspace *>(const_cast<unsigned char *>(dev) + lay->workspace);
    a.b = b;
    a.x = x;
    a.ntiles = ntiles;
    a.base = ticket_base;
    a.wait_limit = wait_limit;
    hipLaunchKernelGGL(solve_tiles, dim3(waves / 4), dim3(kBlock), 0, s, a);
    return (int)hipGetLastError();
}
