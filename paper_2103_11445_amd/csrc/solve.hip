// solve.hip -- gfx950 kernels of the level-scheduled forward substitution
// (arXiv:2103.11445, Sec. II, Algorithm 1) over a possibly rewritten system
// L' x = b + M b (Sec. III, Fig. 3).
//
// Execution model
//   * One cooperative grid of W single-wave workgroups, all resident at
//     once.  Work items (wide tiles of 64 lanes, or segments) are ordered by
//     level of L'; wave w takes items w, w+W, w+2W, ...  An item only depends
//     on rows of earlier items, and the wave holding the lowest unfinished
//     item has finished all its earlier items, so the grid always drains.
//   * Per-row readiness instead of a barrier per level: x itself is the flag.
//     Before the solve every x_i is set to a signalling-NaN bit pattern that
//     no arithmetic result can carry (results are quiet NaNs at worst).  A
//     lane that needs x_k polls it with device-scope loads until the pattern
//     is gone; the producer publishes x_i with one device-scope 8-byte store.
//     Device (agent) scope keeps the eight XCDs' L2 caches out of the way.
//   * Latency hiding in wide tiles: a wave issues every gather of its current
//     tile at once (x polls, b-terms, b_i), then the loads of its next tile's
//     terms, and only then waits for the gathers; the next descriptor is
//     fetched two items ahead.
//   * Segments (runs of narrow levels, e.g. a long serial chain) are one
//     work item executed by one wave tile after tile.  Rows the segment
//     produced recently are read from the wave's LDS ring instead of global
//     memory, and the wave runs a software pipeline: term loads kDepth tiles
//     ahead, b / external-x gathers kDepth/2 tiles ahead, so the critical
//     path waits only on LDS and on loads issued several tiles before.
//   * b-terms (the rewritten right-hand side) never wait.
//   * A wait is bounded by the GPU real-time clock; on expiry the worker
//     marks the plan's status word, which makes every other wait give up,
//     and the grid drains with NaNs.
//
// Loads in this file are issued unconditionally (pads and inactive lanes read
// a valid dummy address and are masked where the value is used), and a
// prefetched register is not touched until its use: the hardware counts
// outstanding loads in issue order, and a load skipped on some paths, or a
// select / copy right after a load, makes the compiler wait for loads still
// in flight (the prefetches) at that point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "plan.hpp"

namespace {

constexpr unsigned long long kNotReady = 0x7FF0DEADBEEF0001ull;  // signalling NaN
constexpr long long kQuietNaN = 0x7FF8000000000000ll;
constexpr int32_t kPad = INT32_MIN;
constexpr int kRegChunks = 4;  // chunks of a wide tile held in registers; more are streamed
constexpr int kDepth = sptrsv::kSegDepth;  // segment pipeline depth (tiles)
constexpr int kSegChunks = sptrsv::kSegChunks;
constexpr int kRing = sptrsv::kRing;

struct SolveArgs {
    const int4 *items;
    const int32_t *rows;
    const double *diag;
    const int32_t *tcol;
    const double *tval;
    const int32_t *scol;
    const double *sval;
    const int2 *srow;
    const double *sdiag;
    sptrsv::Workspace *ws;
    const double *b;
    double *x;
    long long nitems;
    long long waves;
    unsigned long long wait_limit;
    int32_t n;
};

__device__ inline bool is_segment(const int4 d) { return d.w < 0; }

__global__ void fill_not_ready(unsigned long long *__restrict__ x, int32_t n) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        x[i] = kNotReady;
}

__device__ inline unsigned long long load_agent(const double *p) {
    return __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<double *>(p)),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// First attempt at a gather: an ordinary (cached) load.  Stream order makes
// the fill of x visible to this kernel and no cache holds x lines from before
// it, so within the solve a cached copy of x_k is either the not-ready
// pattern or the final value: a stale pattern only sends the lane to the
// device-scope poll, never yields a wrong value.  It lets repeated gathers
// of a published value hit in L2 instead of going to memory each time.
__device__ inline unsigned long long load_cached(const double *p) {
    return *reinterpret_cast<const unsigned long long *>(p);
}

// Bits of x[k] once it is published (a quiet NaN if the wait gave up).
// Only reached behind a wave-uniform branch (see resolve_pending), so the
// call and the waits it implies stay off the path where nothing is pending.
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

// Address a term gathers from: x_k for x-terms (0 <= k < n), b_j for b-terms
// (k = ~j), the dummy b_0 otherwise.
__device__ inline const double *gather_addr(const SolveArgs &a, int32_t k) {
    const double *p = a.b;
    if (k >= 0 && k < a.n) p = a.x + k;
    if (k < 0 && k != kPad) p = a.b + ~k;
    return p;
}

__device__ inline bool pending(const SolveArgs &a, int32_t k, unsigned long long v) {
    return k >= 0 && k < a.n && v == kNotReady;
}

// Waits for every gathered x-term that was not yet published.  The test is a
// wave-wide vote: with a lane-divergent branch the compiler would drain every
// load in flight (the prefetches too) before it on all paths.
//   kElect (wide tiles): while terms are pending, one elected lane polls one
//     of its pending terms; once that value appears every lane re-reads its
//     pending terms once.  The rows a wide tile waits on finish at about the
//     same time, so this costs little latency and keeps the polling traffic
//     to one lane per waiting wave (waves run ahead of the frontier).
//   otherwise (segments, which rarely wait and then on a single row just
//     produced by another wave): every pending lane polls its own term.
template <int kN, bool kElect>
__device__ inline void resolve_pending(const SolveArgs &a, const int32_t *col, unsigned long long *g) {
    bool any = false;
#pragma unroll
    for (int c = 0; c < kN; ++c) any |= pending(a, col[c], g[c]);
    unsigned long long mask = __ballot(any);
    if (!kElect) {
        if (mask) {
#pragma unroll
            for (int c = 0; c < kN; ++c)
                if (pending(a, col[c], g[c])) g[c] = wait_slow(a.x, col[c], a.ws, a.wait_limit);
        }
        return;
    }
    while (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        if ((int)(threadIdx.x & 63) == leader) {
            bool done = false;
#pragma unroll
            for (int c = 0; c < kN; ++c)
                if (!done && pending(a, col[c], g[c])) {
                    g[c] = wait_slow(a.x, col[c], a.ws, a.wait_limit);
                    done = true;
                }
        }
        any = false;
#pragma unroll
        for (int c = 0; c < kN; ++c) {
            if (pending(a, col[c], g[c])) g[c] = load_agent(a.x + col[c]);
            any |= pending(a, col[c], g[c]);
        }
        mask = __ballot(any);
    }
}

// Value of a gathered term (after resolve_pending); 0 for pads.
__device__ inline double term_value(int32_t k, unsigned long long v) {
    return k == kPad ? 0.0 : __longlong_as_double((long long)v);
}

template <int kCtrl>
__device__ inline double dpp_add(double v) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffff), kCtrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), kCtrl, 0xf, 0xf, false);
    return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over aligned groups of 2^lg lanes (every lane of a group gets the sum).
// Groups up to 16 lanes stay in the ALU (DPP quad permutes, then the
// half-row and row mirrors pair the two halves); 32 and 64 use permutes.
__device__ inline double group_sum(double v, int lg) {
    if (lg >= 1) v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
    if (lg >= 2) v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
    if (lg >= 3) v = dpp_add<0x141>(v);  // row_half_mirror
    if (lg >= 4) v = dpp_add<0x140>(v);  // row_mirror
    if (lg >= 5) v += __shfl_xor(v, 16, 64);
    if (lg >= 6) v += __shfl_xor(v, 32, 64);
    return v;
}

// Descriptor of item i, fetched by a vector load (lane q < 4 reads word q)
// so that it never waits behind LDS traffic, and unpacked into scalars only
// when it is needed (one item later).
__device__ inline int load_item(const SolveArgs &a, long long i, int lane) {
    const long long idx = i < a.nitems ? i : 0;
    return reinterpret_cast<const int *>(a.items)[idx * 4 + (lane & 3)];
}
__device__ inline int4 unpack_item(int w) {
    return make_int4(__builtin_amdgcn_readlane(w, 0), __builtin_amdgcn_readlane(w, 1),
                     __builtin_amdgcn_readlane(w, 2), __builtin_amdgcn_readlane(w, 3));
}

// ----------------------------------------------------------- wide tiles --

// Registers of one wide tile as seen by one lane.  They hold loads in
// flight: nothing touches them until the tile is processed, so pads and
// inactive lanes read a dummy address and are masked at use.
struct Tile {
    int4 d;                     // {chunk offset, slot offset, chunks, nrows << 8 | log2 lanes per row}
    int32_t col[kRegChunks];    // term columns of this lane, raw
    double val[kRegChunks];     // term coefficients, raw
    int32_t row;                // row id of the lane's slot, raw
    double diag;
};

__device__ inline bool tile_active(const int4 d, int lane) { return (lane >> (d.w & 0xff)) < (d.w >> 8); }
__device__ inline bool tile_lead(const int4 d, int lane) {
    return tile_active(d, lane) && (lane & ((1 << (d.w & 0xff)) - 1)) == 0;
}
__device__ inline int32_t tile_col(const Tile &T, int c, int lane) {
    return tile_active(T.d, lane) && c < T.d.z ? T.col[c] : kPad;
}
__device__ inline double tile_val(const Tile &T, int c, int lane) {
    return tile_active(T.d, lane) && c < T.d.z ? T.val[c] : 0.0;
}

__device__ inline void load_tile(const SolveArgs &a, const int4 d, int lane, Tile &T) {
    T.d = d;
    const bool active = tile_active(d, lane);
    const size_t base = (size_t)d.x * 64 + lane;
#pragma unroll
    for (int c = 0; c < kRegChunks; ++c) {
        const bool ok = active && c < d.z;
        T.col[c] = *(ok ? a.tcol + base + (size_t)c * 64 : a.rows);
        T.val[c] = *(ok ? a.tval + base + (size_t)c * 64 : a.diag);
    }
    const int32_t slot = tile_lead(d, lane) ? d.y + (lane >> (d.w & 0xff)) : 0;
    T.row = a.rows[slot];
    T.diag = a.diag[slot];
}

// ------------------------------------------------------------- segments --

// One tile of a segment as seen by one lane, from load to finish.  As for
// Tile, the loaded registers are left untouched until they are used.
struct SegSlot {
    int4 col;                          // term columns
    double2 v01, v23;                  // term coefficients
    int2 rm;                           // {row (-1 if the lane finishes none), meta}
    double diag;
    unsigned long long g[kSegChunks];  // gathered b / external x (bits)
    double bi;                         // b of the lane's row (meaningful where rm.x >= 0)
};

__device__ inline int32_t seg_col(const SegSlot &S, int c) {
    return c == 0 ? S.col.x : c == 1 ? S.col.y : c == 2 ? S.col.z : S.col.w;
}
__device__ inline double seg_val(const SegSlot &S, int c) {
    return c == 0 ? S.v01.x : c == 1 ? S.v01.y : c == 2 ? S.v23.x : S.v23.y;
}

__device__ inline void seg_load(const SolveArgs &a, long long st, int lane, SegSlot &S) {
    static_assert(kSegChunks == 4, "segment tiles are fetched as int4 / 2 x double2 per lane");
    const size_t ln = (size_t)st * 64 + lane;
    S.col = reinterpret_cast<const int4 *>(a.scol)[ln];
    S.v01 = reinterpret_cast<const double2 *>(a.sval)[2 * ln];
    S.v23 = reinterpret_cast<const double2 *>(a.sval)[2 * ln + 1];
    S.rm = a.srow[ln];
    S.diag = a.sdiag[ln];
}

__device__ inline void seg_gather(const SolveArgs &a, SegSlot &S) {
#pragma unroll
    for (int c = 0; c < kSegChunks; ++c) S.g[c] = load_cached(gather_addr(a, seg_col(S, c)));
    S.bi = a.b[S.rm.x >= 0 ? S.rm.x : 0];
}

__device__ inline void seg_finish(const SolveArgs &a, SegSlot &S, double *ring) {
    int32_t col[kSegChunks];
#pragma unroll
    for (int c = 0; c < kSegChunks; ++c) col[c] = seg_col(S, c);
    resolve_pending<kSegChunks, false>(a, col, S.g);
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < kSegChunks; ++c) {
        const int32_t k = col[c];
        const double v = k >= a.n ? ring[k - a.n] : term_value(k, S.g[c]);
        acc = fma(seg_val(S, c), v, acc);
    }
    acc = group_sum(acc, __builtin_amdgcn_readfirstlane(S.rm.y) & 0xff);
    if (S.rm.x >= 0) {
        const double xi = (S.bi + acc) / S.diag;
        ring[S.rm.y >> 8] = xi;
        __hip_atomic_store(reinterpret_cast<unsigned long long *>(a.x) + S.rm.x,
                           (unsigned long long)__double_as_longlong(xi), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Tiles [first, first + count) of the segment arrays, in order, by this wave
// (count is a multiple of kDepth: the packer pads segments with empty tiles,
// so the unrolled loop body has no exit and keeps its registers in place).
// Loads of tile t+kDepth and gathers of tile t+kDepth/2 are issued while tile
// t finishes; indices past the end are clamped to the last tile (the extra
// loads are harmless and keep the load count per step fixed).  The compiler
// barriers keep every stage where it is written: left to itself the
// scheduler sinks the prefetch loads down to their use.
__device__ void run_segment(const SolveArgs &a, const int4 d, int lane, double *ring) {
    const long long first = d.x, count = d.y, last = first + count - 1;
    SegSlot S[kDepth];
#pragma unroll
    for (int k = 0; k < kDepth; ++k) seg_load(a, min(first + k, last), lane, S[k]);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kDepth / 2; ++k) seg_gather(a, S[k]);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    for (long long base = 0; base < count; base += kDepth) {
#pragma unroll
        for (int k = 0; k < kDepth; ++k) {
            const long long t = base + k;
            seg_finish(a, S[k], ring);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            seg_gather(a, S[(k + kDepth / 2) % kDepth]);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            seg_load(a, min(first + t + kDepth, last), lane, S[k]);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// ----------------------------------------------------------------- kernel --

__global__ void __launch_bounds__(64) solve_tiles(SolveArgs a) {
    __shared__ double ring[kRing];
    const int lane = threadIdx.x;
    long long i = blockIdx.x;
    if (i >= a.nitems) return;
    int4 d = unpack_item(load_item(a, i, lane));
    Tile cur;
    if (!is_segment(d)) load_tile(a, d, lane, cur);
    int wnext = load_item(a, i + a.waves, lane);  // raw descriptor of the next item
    for (;;) {
        const long long in = i + a.waves, inn = in + a.waves;
        if (is_segment(d)) {
            run_segment(a, d, lane, ring);
            if (in >= a.nitems) break;
            d = unpack_item(wnext);
            if (!is_segment(d)) load_tile(a, d, lane, cur);
            wnext = load_item(a, inn, lane);
            i = in;
            continue;
        }
        const int4 dnext = unpack_item(wnext);
        // 1. every gather of the current tile in flight
        int32_t col[kRegChunks];
        unsigned long long g[kRegChunks];
#pragma unroll
        for (int c = 0; c < kRegChunks; ++c) {
            col[c] = tile_col(cur, c, lane);
            g[c] = load_cached(gather_addr(a, col[c]));
        }
        const bool lead = tile_lead(cur.d, lane);
        const double bi = a.b[lead ? cur.row : 0];
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        // 2. the next tile's terms and the descriptor after it
        Tile nxt;
        const bool nwide = in < a.nitems && !is_segment(dnext);
        load_tile(a, nwide ? dnext : d, lane, nxt);
        const int wnn = load_item(a, inn, lane);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        // 3. wait for the gathers, accumulate
        resolve_pending<kRegChunks, true>(a, col, g);
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kRegChunks; ++c) acc = fma(tile_val(cur, c, lane), term_value(col[c], g[c]), acc);
        // 4. rows longer than the register chunks: stream the rest
        if (cur.d.z > kRegChunks) {
            if (tile_active(cur.d, lane)) {
                const size_t base = (size_t)cur.d.x * 64 + lane;
                for (int c = kRegChunks; c < cur.d.z; ++c) {
                    const int32_t k = a.tcol[base + (size_t)c * 64];
                    const double v = a.tval[base + (size_t)c * 64];
                    unsigned long long gv = load_cached(gather_addr(a, k));
                    if (pending(a, k, gv)) gv = wait_slow(a.x, k, a.ws, a.wait_limit);
                    acc = fma(v, term_value(k, gv), acc);
                }
            }
        }
        // 5. row sums across the row's lanes, then x_i
        acc = group_sum(acc, cur.d.w & 0xff);
        if (lead) {
            const double xi = (bi + acc) / cur.diag;
            __hip_atomic_store(reinterpret_cast<unsigned long long *>(a.x) + cur.row,
                               (unsigned long long)__double_as_longlong(xi), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        if (in >= a.nitems) break;
        cur = nxt;
        d = dnext;
        wnext = wnn;
        i = in;
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
                                   int64_t nitems, int waves, uint64_t wait_limit, const double *b,
                                   double *x, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int fill_blocks = (int)std::min<int64_t>(2048, ((int64_t)n + 255) / 256);
    hipLaunchKernelGGL(fill_not_ready, dim3(fill_blocks), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long *>(x), n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    SolveArgs a;
    a.items = reinterpret_cast<const int4 *>(dev + lay->tiles);
    a.rows = reinterpret_cast<const int32_t *>(dev + lay->rows);
    a.diag = reinterpret_cast<const double *>(dev + lay->diag);
    a.tcol = reinterpret_cast<const int32_t *>(dev + lay->tcol);
    a.tval = reinterpret_cast<const double *>(dev + lay->tval);
    a.scol = reinterpret_cast<const int32_t *>(dev + lay->scol);
    a.sval = reinterpret_cast<const double *>(dev + lay->sval);
    a.srow = reinterpret_cast<const int2 *>(dev + lay->srow);
    a.sdiag = reinterpret_cast<const double *>(dev + lay->sdiag);
    a.ws = reinterpret_cast<sptrsv::Workspace *>(const_cast<unsigned char *>(dev) + lay->workspace);
    a.b = b;
    a.x = x;
    a.nitems = nitems;
    a.waves = waves;
    a.wait_limit = wait_limit;
    a.n = n;
    void *args[] = {&a};
    return (int)hipLaunchCooperativeKernel(reinterpret_cast<const void *>(solve_tiles), dim3(waves),
                                           dim3(64), args, 0, s);
}
