// solve.hip -- gfx950 kernels of the level-scheduled forward substitution
// (arXiv:2103.11445, Sec. II, Algorithm 1) over a possibly rewritten system
// L' x = b + M b (Sec. III, Fig. 3).
//
// Execution model
//   * One cooperative grid of W single-wave workgroups, all resident at
//     once.  Tiles (64 lanes each) are ordered by level of L'; wave w takes
//     tiles w, w+W, w+2W, ...  A tile only depends on rows of earlier tiles,
//     and the wave holding the lowest unfinished tile has finished all its
//     earlier tiles, so the grid always drains.
//   * Per-row readiness instead of a barrier per level: x itself is the flag.
//     Before the solve every x_i is set to a signalling-NaN bit pattern that
//     no arithmetic result can carry (results are quiet NaNs at worst).  A
//     lane that needs x_k polls it with device-scope loads until the pattern
//     is gone; the producer publishes x_i with one device-scope 8-byte store.
//     Device (agent) scope keeps the eight XCDs' L2 caches out of the way.
//   * Latency hiding: a wave issues every gather of its current tile at once
//     (x polls, b-terms, b_i), then the loads of its next tile's terms, and
//     only then waits for the gathers; the next tile's descriptor is fetched
//     two tiles ahead.
//   * b-terms (the rewritten right-hand side) never wait.
//   * A wait is bounded by the GPU real-time clock; on expiry the worker
//     marks the plan's status word, which makes every other wait give up,
//     and the grid drains with NaNs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "plan.hpp"

namespace {

constexpr unsigned long long kNotReady = 0x7FF0DEADBEEF0001ull;  // signalling NaN
constexpr long long kQuietNaN = 0x7FF8000000000000ll;
constexpr int32_t kPad = INT32_MIN;
constexpr int kRegChunks = 4;  // chunks of a tile held in registers; more are streamed

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
    long long waves;
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

// Bits of x[k] once it is published (a quiet NaN if the wait gave up).
__device__ __noinline__ unsigned long long wait_slow(const double *x, int32_t k, sptrsv::Workspace *ws,
                                                     unsigned long long limit) {
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (unsigned it = 1;; ++it) {
        __builtin_amdgcn_s_sleep(1);
        const unsigned long long v = load_agent(x + k);
        if (v != kNotReady) return v;
        if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
            __hip_atomic_fetch_or(&ws->status, (unsigned)SPTRSV_ERR_TIMEOUT, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            return (unsigned long long)kQuietNaN;
        }
        if ((it & 15u) == 0 &&
            __hip_atomic_load(&ws->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            return (unsigned long long)kQuietNaN;
    }
}

// Registers of one tile as seen by one lane.
struct Tile {
    int4 d;                     // {chunk offset, slot offset, chunks, nrows << 8 | log2 lanes per row}
    int32_t col[kRegChunks];    // term columns of this lane (kPad if none)
    double val[kRegChunks];     // term coefficients (0 for pads)
    int32_t row;                // row finished by this lane, -1 if none
    double diag;
};

__device__ inline void load_tile(const SolveArgs &a, const int4 d, int lane, Tile &T) {
    T.d = d;
    const int lg = d.w & 0xff;
    const bool active = (lane >> lg) < (d.w >> 8);
    const size_t base = (size_t)d.x * 64 + lane;
#pragma unroll
    for (int c = 0; c < kRegChunks; ++c) {
        T.col[c] = kPad;
        T.val[c] = 0.0;
        if (active && c < d.z) {
            T.col[c] = a.tcol[base + (size_t)c * 64];
            T.val[c] = a.tval[base + (size_t)c * 64];
        }
    }
    T.row = -1;
    T.diag = 1.0;
    if (active && (lane & ((1 << lg) - 1)) == 0) {
        const int32_t slot = d.y + (lane >> lg);
        T.row = a.rows[slot];
        T.diag = a.diag[slot];
    }
}

__device__ inline unsigned long long issue_gather(const SolveArgs &a, int32_t k) {
    if (k >= 0) return load_agent(a.x + k);
    if (k != kPad) return (unsigned long long)__double_as_longlong(a.b[~k]);
    return 0ull;
}

__device__ inline unsigned long long resolve(const SolveArgs &a, int32_t k, unsigned long long v) {
    if (k >= 0 && v == kNotReady) v = wait_slow(a.x, k, a.ws, a.wait_limit);
    return v;
}

__global__ void __launch_bounds__(64) solve_tiles(SolveArgs a) {
    const int lane = threadIdx.x;
    long long t = blockIdx.x;
    if (t >= a.ntiles) return;
    Tile cur;
    load_tile(a, a.tiles[t], lane, cur);
    int4 dnext = make_int4(0, 0, 0, 0);
    if (t + a.waves < a.ntiles) dnext = a.tiles[t + a.waves];
    for (;;) {
        const long long tn = t + a.waves, tnn = tn + a.waves;
        // 1. every gather of the current tile in flight
        unsigned long long g[kRegChunks];
#pragma unroll
        for (int c = 0; c < kRegChunks; ++c) g[c] = issue_gather(a, cur.col[c]);
        const double bi = cur.row >= 0 ? a.b[cur.row] : 0.0;
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        // 2. the next tile's terms and the descriptor after it
        Tile nxt;
        int4 dnn = make_int4(0, 0, 0, 0);
        if (tn < a.ntiles) {
            load_tile(a, dnext, lane, nxt);
            if (tnn < a.ntiles) dnn = a.tiles[tnn];
        }
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        // 3. wait for the gathers, accumulate
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kRegChunks; ++c)
            acc = fma(cur.val[c], __longlong_as_double((long long)resolve(a, cur.col[c], g[c])), acc);
        // 4. rows longer than the register chunks: stream the rest
        if (cur.d.z > kRegChunks) {
            const int lg = cur.d.w & 0xff;
            if ((lane >> lg) < (cur.d.w >> 8)) {
                const size_t base = (size_t)cur.d.x * 64 + lane;
                for (int c = kRegChunks; c < cur.d.z; ++c) {
                    const int32_t k = a.tcol[base + (size_t)c * 64];
                    const double v = a.tval[base + (size_t)c * 64];
                    acc = fma(v, __longlong_as_double((long long)resolve(a, k, issue_gather(a, k))), acc);
                }
            }
        }
        // 5. row sums across the row's lanes, then x_i
        const int lg = cur.d.w & 0xff;
        for (int off = (1 << lg) >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (cur.row >= 0) {
            const double xi = (bi + acc) / cur.diag;
            __hip_atomic_store(reinterpret_cast<unsigned long long *>(a.x) + cur.row,
                               (unsigned long long)__double_as_longlong(xi), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tn >= a.ntiles) break;
        cur = nxt;
        dnext = dnn;
        t = tn;
    }
}

}  // namespace

extern "C" int sptrsv_device_limits(int *cus, int *max_waves_per_cu) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    int blocks = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, solve_tiles, 64, 0);
    if (e != hipSuccess) return (int)e;
    *max_waves_per_cu = blocks;
    return 0;
}

extern "C" int sptrsv_launch_solve(const unsigned char *dev, const sptrsv::Layout *lay, int32_t n,
                                   int64_t ntiles, int waves, uint64_t wait_limit, const double *b,
                                   double *x, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int fill_blocks = (int)std::min<int64_t>(2048, ((int64_t)n + 255) / 256);
    hipLaunchKernelGGL(fill_not_ready, dim3(fill_blocks), dim3(256), 0, s,
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
    a.waves = waves;
    a.wait_limit = wait_limit;
    void *args[] = {&a};
    return (int)hipLaunchCooperativeKernel(reinterpret_cast<const void *>(solve_tiles), dim3(waves),
                                           dim3(64), args, 0, s);
}
