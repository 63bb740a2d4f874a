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
//   * Rows that no other row depends on (sinks) are off the dependency
//     chain: they are packed into a second queue, in level order, served by
//     waves of their own, so the chain's waves only carry rows something
//     waits for.  Chain rows depend only on chain rows (nothing depends on a
//     sink), so the argument above holds for each queue.
//   * Per-row readiness instead of a barrier per level: x itself is the flag.
//     Before the solve every x_i is set to a signalling-NaN bit pattern that
//     no arithmetic result can carry (results are quiet NaNs at worst).  A
//     lane that needs x_k polls it with device-scope loads until the pattern
//     is gone; the producer publishes x_i with one device-scope 8-byte store.
//     Device (agent) scope keeps the eight XCDs' L2 caches out of the way.
//   * Latency hiding in wide tiles: a wave issues every gather of its current
//     tile at once (x-terms and the row's constant), then the loads of its
//     next tile's terms, and only then waits for the gathers; the next
//     descriptor is fetched two items ahead.  The wait: one elected lane
//     polls until a term appears, then the whole wave re-reads its pending
//     terms each round (the rows a tile waits on finish together).
//   * Segments (runs of narrow levels, e.g. a long serial chain, or a whole
//     stage of the stage system) are one work item executed by one wave tile
//     after tile.  Rows the segment produced recently are read from the
//     wave's LDS ring instead of global memory, and the wave runs a software
//     pipeline: term loads kDepth tiles ahead, constant / external-x gathers
//     kDepth/2 tiles ahead, so the critical path waits only on LDS and on
//     loads issued several tiles before.  A plan whose segments read only the
//     ring runs an instance without the external-x machinery.
//   * Wide tiles keep 4 or 8 chunks of terms in registers (one instance
//     each, chosen per plan); x and b are addressed by 32-bit offsets from
//     their base.
//   * The rewritten right-hand side b' = b + M b depends on nothing the
//     solve computes, so the solve's tiles hold x-terms only and b' comes
//     from a step before it: either a fully parallel pass over M (prepare),
//     or -- since b'_S = D_S L_SS^-1 b_S on the rows S of a stage -- a solve
//     of the block-diagonal system L_B (the stages' diagonal blocks of L) by
//     the same kernel, whose chain is one stage deep and which reads nnz(L_B)
//     entries instead of nnz(M); the main solve then reads y and scales it
//     by the diagonal.
//   * The same kernels run in FP64 or, for plans stored in FP32, in FP32
//     (values, arithmetic and x; the readiness pattern is then an FP32
//     signalling NaN); iterative refinement adds an FP64 residual and an
//     FP64 update around the FP32 solve.
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

constexpr int32_t kPad = INT32_MIN;
// chunks of a wide tile held in registers (more are streamed): kernel
// instances for 4 and 8, chosen per plan by the packer (Layout::reg_chunks)
constexpr int kDepth = sptrsv::kSegDepth;  // segment pipeline depth (tiles)
constexpr int kSegChunks = sptrsv::kSegChunks;
constexpr int kRing = sptrsv::kRing;

// Per value type: the bit pattern of "not yet published" (a signalling NaN
// no arithmetic can produce) and of the NaN a failed wait yields.
template <typename T> struct Val;
template <> struct Val<double> {
    using Bits = unsigned long long;
    static constexpr Bits kNotReady = 0x7FF0DEADBEEF0001ull;
    static constexpr Bits kQuietNaN = 0x7FF8000000000000ull;
    __device__ static double of(Bits b) { return __longlong_as_double((long long)b); }
    __device__ static Bits bits(double v) { return (Bits)__double_as_longlong(v); }
};
template <> struct Val<float> {
    using Bits = unsigned int;
    static constexpr Bits kNotReady = 0x7FA0DEADu;
    static constexpr Bits kQuietNaN = 0x7FC00000u;
    __device__ static float of(Bits b) { return __uint_as_float(b); }
    __device__ static Bits bits(float v) { return __float_as_uint(v); }
};

template <typename T>
struct SolveArgs {
    const int4 *items;
    const int32_t *rows;
    const T *diag;
    const int32_t *tcol;
    const uint16_t *tcol16;  // the same section in the compact encoding (see tile_col)
    const T *tval;
    const int32_t *scol;
    const T *sval;
    const int4 *srow;
    const T *sdiag;
    sptrsv::Workspace *ws;
    const unsigned *skip;  // refinement: the grid returns at once if *skip (NULL: never)
    unsigned long long *stamps;  // timed solves: completion clock of every item and segment tile
    long long start_slot;        // stamps[start_slot]: the clock when the grid started
    const T *b;  // b' = b + M b (written by prepare), y (b' = diag * y), or b
    int bscale;  // the constants are y: b'_i = diag_i * y_i
    T *x;        // x in slot (schedule) order, its own readiness flag; terms index it
    T *xout;     // the caller's x, in its own order: every row stored once, plainly
    long long nitems;
    long long waves;
    // two work queues: items [0, nchain) hold the rows some row of a later
    // item depends on (the chain), in level order, taken round-robin by
    // waves [0, wchain); items [nchain, nitems) hold rows nothing depends
    // on (sinks), in level order, taken by the other waves.  One queue:
    // nchain = nitems, wchain = waves.
    long long nchain;
    long long wchain;
    unsigned long long wait_limit;
    int32_t n;
};

__device__ inline bool is_segment(const int4 d) { return d.w < 0; }



template <typename T>
__device__ inline typename Val<T>::Bits load_agent(const T *p) {
    using B = typename Val<T>::Bits;
    return __hip_atomic_load(reinterpret_cast<B *>(const_cast<T *>(p)), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// Bits of x[k] once it is published (a quiet NaN if the wait gave up).
// Only reached behind a wave-uniform branch (see resolve_pending), so the
// call and the waits it implies stay off the path where nothing is pending.
template <typename T>
__device__ __noinline__ typename Val<T>::Bits wait_slow(const T *x, int32_t k, sptrsv::Workspace *ws,
                                                        unsigned long long limit) {
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (unsigned it = 1;; ++it) {
        __builtin_amdgcn_s_sleep(1);
        const typename Val<T>::Bits v = load_agent(x + k);
        if (v != Val<T>::kNotReady) return v;
        if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
            __hip_atomic_fetch_or(&ws->status, (unsigned)SPTRSV_ERR_TIMEOUT, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            return Val<T>::kQuietNaN;
        }
        if ((it & 15u) == 0 &&
            __hip_atomic_load(&ws->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            return Val<T>::kQuietNaN;
    }
}

// Element k of a (uniform) array as a 32-bit byte offset from its base, so
// that the load takes the scalar-base form (no 64-bit address per lane; the
// packer keeps n * sizeof(T) below 2^32).
template <typename T>
__device__ inline typename Val<T>::Bits load_at(const T *base, int32_t k) {
    const uint32_t off = (uint32_t)k * (uint32_t)sizeof(T);
    return *reinterpret_cast<const typename Val<T>::Bits *>(reinterpret_cast<const char *>(base) + off);
}

// First attempt at a term's gather, an ordinary (cached) load: x_k for
// x-terms (0 <= k < n); x_0 for pads and LDS-ring terms (k outside [0, n)),
// whose value is not used.  Stream order makes the fill of x visible to this
// kernel and no cache holds x lines from before it, so within the solve a
// cached copy of x_k is either the not-ready pattern or the final value: a
// stale pattern only sends the lane to the device-scope poll, never yields a
// wrong value.  It lets repeated gathers of a published value hit in L2
// instead of going to memory each time.
template <typename T>
__device__ inline typename Val<T>::Bits gather_x(const SolveArgs<T> &a, int32_t k) {
    return load_at(a.x, k >= 0 && k < a.n ? k : 0);
}

template <typename T>
__device__ inline bool pending(const SolveArgs<T> &a, int32_t k, typename Val<T>::Bits v) {
    return k >= 0 && k < a.n && v == Val<T>::kNotReady;
}

// Waits for every gathered x-term that was not yet published.  The test is a
// wave-wide vote: with a lane-divergent branch the compiler would drain every
// load in flight (the prefetches too) before it on all paths.
//   kElect (wide tiles): one elected lane polls one of its pending terms
//     until it appears, which keeps the polling traffic to one lane per
//     waiting wave while nothing is ready (waves run ahead of the frontier).
//     The rows a wide tile waits on finish at about the same time, so that
//     first arrival opens a burst: from then on every lane re-reads its
//     pending terms each round until none is left, so the wave sees the last
//     of them within one round trip of its publication.
//   otherwise (segments, which rarely wait and then on a single row just
//     produced by another wave): every pending lane polls its own term.
template <int kN, bool kElect, typename T>
__device__ inline void resolve_pending(const SolveArgs<T> &a, const int32_t *col, typename Val<T>::Bits *g) {
    bool any = false;
#pragma unroll
    for (int c = 0; c < kN; ++c) any |= pending(a, col[c], g[c]);
    unsigned long long mask = __ballot(any);
    if (!mask) return;
    if (!kElect) {
#pragma unroll
        for (int c = 0; c < kN; ++c)
            if (pending(a, col[c], g[c])) g[c] = wait_slow(a.x, col[c], a.ws, a.wait_limit);
        return;
    }
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
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (unsigned it = 1;; ++it) {
        any = false;
#pragma unroll
        for (int c = 0; c < kN; ++c) {
            if (pending(a, col[c], g[c])) g[c] = load_agent(a.x + col[c]);
            any |= pending(a, col[c], g[c]);
        }
        if (!__ballot(any)) return;
        // give up like wait_slow: past the wait limit (marking the status
        // word), or once another wait has given up, take a quiet NaN
        const bool late = __builtin_amdgcn_s_memrealtime() - t0 > a.wait_limit;
        if (late || ((it & 15u) == 0 && __hip_atomic_load(&a.ws->status, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
#pragma unroll
            for (int c = 0; c < kN; ++c)
                if (pending(a, col[c], g[c])) g[c] = late ? wait_slow(a.x, col[c], a.ws, 0ull) : Val<T>::kQuietNaN;
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Value of a gathered term (after resolve_pending); 0 for pads.
template <typename T>
__device__ inline T term_value(int32_t k, typename Val<T>::Bits v) {
    return k == kPad ? T(0) : Val<T>::of(v);
}

// (the permutes used here read a lane of the same row for every lane, so no
// lane keeps an old value and none needs to be supplied)
template <int kCtrl>
__device__ inline double dpp_add(double v) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(bits & 0xffffffff), kCtrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), kCtrl, 0xf, 0xf, false);
    return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int kCtrl>
__device__ inline float dpp_add(float v) {
    return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), kCtrl, 0xf, 0xf, false));
}

// Sum over aligned groups of 2^lg lanes (every lane of a group gets the sum).
// Groups up to 16 lanes stay in the ALU (DPP quad permutes, then the
// half-row and row mirrors pair the two halves); 32 and 64 use permutes.
template <typename T>
__device__ inline T group_sum(T v, int lg) {
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
template <typename T>
__device__ inline int load_item(const SolveArgs<T> &a, long long i, int lane) {
    const long long idx = i < a.nitems ? i : 0;
    return reinterpret_cast<const int *>(a.items)[idx * 4 + (lane & 3)];
}
__device__ inline int4 unpack_item(int w) {
    return make_int4(__builtin_amdgcn_readlane(w, 0), __builtin_amdgcn_readlane(w, 1),
                     __builtin_amdgcn_readlane(w, 2), __builtin_amdgcn_readlane(w, 3));
}

// The slot-ordered x of the solve (and of the stage system's solve) := not ready.
template <typename T>
__global__ void fill_not_ready(typename Val<T>::Bits *__restrict__ x, typename Val<T>::Bits *__restrict__ y,
                               int32_t n, const unsigned *skip) {
    if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        x[i] = Val<T>::kNotReady;
        if (y) y[i] = Val<T>::kNotReady;
    }
}

// ---------------------------------------------------------------- prepare --

template <typename T>
struct PrepArgs {
    const int4 *tiles;       // M tiles
    const int32_t *rows;     // device row of each M-tile slot
    const int32_t *col;      // b-term columns (device index of b_j), kPad for pads
    const T *val;            // M_ij
    const T *b;
    T *bp;                   // out: b'
    typename Val<T>::Bits *x;  // out: the not-ready pattern, over the slot-ordered x
    int32_t n;
    long long ntiles;
    const unsigned *skip;    // refinement: return at once if *skip
};

// b'_i = b_i + sum_j M_ij b_j for every row (one wave per M tile,
// grid-stride, its chunks in groups of four with every load issued before
// the first use) and x := not ready.  Nothing here waits on another wave.
template <typename T>
__global__ void __launch_bounds__(256) prepare(PrepArgs<T> a) {
    if (a.skip && __hip_atomic_load(a.skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x)
        a.x[i] = Val<T>::kNotReady;
    const int lane = threadIdx.x & 63;
    const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
    for (long long t = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t < a.ntiles; t += nw) {
        const int4 dv = a.tiles[t];
        const int4 d = make_int4(__builtin_amdgcn_readfirstlane(dv.x), __builtin_amdgcn_readfirstlane(dv.y),
                                 __builtin_amdgcn_readfirstlane(dv.z), __builtin_amdgcn_readfirstlane(dv.w));
        const int lg = d.w & 0xff, nrows = d.w >> 8;
        const bool active = (lane >> lg) < nrows;
        const size_t base = (size_t)d.x * 64 + lane;
        T acc = T(0);
        for (int c0 = 0; c0 < d.z; c0 += 4) {
            int32_t k[4];
            T v[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const size_t idx = base + (size_t)(c0 + u < d.z ? c0 + u : c0) * 64;
                k[u] = a.col[idx];
                v[u] = a.val[idx];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (!active || c0 + u >= d.z) k[u] = kPad;
                bv[u] = a.b[k[u] == kPad ? 0 : k[u]];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = fma(v[u], k[u] == kPad ? T(0) : bv[u], acc);
        }
        acc = group_sum(acc, lg);
        if (active && (lane & ((1 << lg) - 1)) == 0) {
            const int32_t row = a.rows[d.y + (lane >> lg)];
            a.bp[row] = a.b[row] + acc;
        }
    }
}

// ----------------------------------------------------------- wide tiles --

// Registers of one wide tile as seen by one lane.  They hold loads in
// flight: nothing touches them until the tile is processed, so pads and
// inactive lanes read a dummy address and are masked at use.
template <typename T, int kReg>
struct Tile {
    int4 d;                     // {chunk offset, slot offset, chunks, nrows << 8 | log2 lanes per row}
    int32_t col[kReg];          // term columns of this lane, raw
    T val[kReg];                // term coefficients, raw
    int32_t row;                // row id of the lane's slot, raw
    T diag;
};

// Descriptor word of a wide tile: rows << 16 | first copy << 8 | log2 copies
// per row << 4 | log2 lanes per row.  Rows that are copies of one row (a
// batched plan's right-hand sides) share copy 0's terms: the lanes of copy c
// read them and gather c slots further.
__device__ inline int tile_lg(const int4 d) { return d.w & 0xf; }
__device__ inline int tile_lgk(const int4 d) { return (d.w >> 4) & 0xf; }
__device__ inline int tile_rows(const int4 d) { return d.w >> 16; }
__device__ inline bool tile_active(const int4 d, int lane) { return (lane >> tile_lg(d)) < tile_rows(d); }
__device__ inline bool tile_lead(const int4 d, int lane) {
    return tile_active(d, lane) && (lane & ((1 << tile_lg(d)) - 1)) == 0;
}
// where the lane's terms are stored within a chunk, and its copy index
__device__ inline int tile_term_lane(const int4 d, int lane) {
    const int lg = tile_lg(d);
    return (((lane >> lg) >> tile_lgk(d)) << lg) | (lane & ((1 << lg) - 1));
}
__device__ inline int32_t tile_copy(const int4 d, int lane) {
    return (((d.w >> 8) & 0xff) + (lane >> tile_lg(d))) & ((1 << tile_lgk(d)) - 1);
}
// A term's column: the slot of its x.  Compact plans (kCol16) store it as
// the distance back from the tile's first slot in 16 bits (every term reads
// an earlier level, so the distance is at least 1; 0 marks a pad).
template <bool kCol16>
__device__ inline int32_t decode_col(int32_t raw, const int4 d) {
    if (kCol16) return raw == 0 ? kPad : d.y - raw;
    return raw;
}
template <bool kCol16, typename V, int kReg>
__device__ inline int32_t tile_col(const Tile<V, kReg> &T, int c, int lane) {
    const int32_t k = decode_col<kCol16>(T.col[c], T.d);
    return tile_active(T.d, lane) && c < T.d.z && k != kPad ? k + tile_copy(T.d, lane) : kPad;
}
template <typename V, int kReg>
__device__ inline V tile_val(const Tile<V, kReg> &T, int c, int lane) {
    return tile_active(T.d, lane) && c < T.d.z ? T.val[c] : V(0);
}

template <bool kCol16, typename V, int kReg>
__device__ inline void load_tile(const SolveArgs<V> &a, const int4 d, int lane, Tile<V, kReg> &T) {
    T.d = d;
    const bool active = tile_active(d, lane);
    const size_t base = (size_t)d.x * 64 + tile_term_lane(d, lane);
#pragma unroll
    for (int c = 0; c < kReg; ++c) {
        const bool ok = active && c < d.z;
        // terms are read once per solve: streaming loads, so that they do
        // not evict the lines of x that the dependency chain reads back
        if (kCol16)
            T.col[c] = __builtin_nontemporal_load(ok ? a.tcol16 + base + (size_t)c * 64
                                                     : reinterpret_cast<const uint16_t *>(a.rows));
        else
            T.col[c] = __builtin_nontemporal_load(ok ? a.tcol + base + (size_t)c * 64 : a.rows);
        T.val[c] = __builtin_nontemporal_load(ok ? a.tval + base + (size_t)c * 64 : a.diag);
    }
    const int32_t slot = tile_lead(d, lane) ? d.y + (lane >> tile_lg(d)) : 0;
    T.row = a.rows[slot];
    T.diag = a.diag[slot];
}

// ------------------------------------------------------------- segments --

// One tile of a segment as seen by one lane, from load to finish.  As for
// Tile, the loaded registers are left untouched until they are used.
template <typename T> struct Four;
template <> struct Four<double> { double2 a, b; };  // 4 coefficients in two 16-byte loads
template <> struct Four<float> { float4 a; };       // ... or one

template <typename T>
struct SegSlot {
    int4 col;                                  // term columns
    Four<T> v;                                 // term coefficients
    int4 rm;                                   // {row (-1 if the lane finishes none), meta, slot, 0}
    T diag;
    typename Val<T>::Bits g[kSegChunks];       // gathered b / external x (bits)
    T bi;                                      // b of the lane's row (meaningful where rm.x >= 0)
};

template <typename T>
__device__ inline int32_t seg_col(const SegSlot<T> &S, int c) {
    return c == 0 ? S.col.x : c == 1 ? S.col.y : c == 2 ? S.col.z : S.col.w;
}
__device__ inline double seg_val(const SegSlot<double> &S, int c) {
    return c == 0 ? S.v.a.x : c == 1 ? S.v.a.y : c == 2 ? S.v.b.x : S.v.b.y;
}
__device__ inline float seg_val(const SegSlot<float> &S, int c) {
    return c == 0 ? S.v.a.x : c == 1 ? S.v.a.y : c == 2 ? S.v.a.z : S.v.a.w;
}

__device__ inline void load_four(const double *p, size_t ln, Four<double> &v) {
    v.a = reinterpret_cast<const double2 *>(p)[2 * ln];
    v.b = reinterpret_cast<const double2 *>(p)[2 * ln + 1];
}
__device__ inline void load_four(const float *p, size_t ln, Four<float> &v) {
    v.a = reinterpret_cast<const float4 *>(p)[ln];
}

template <typename T>
__device__ inline void seg_load(const SolveArgs<T> &a, long long st, int lane, SegSlot<T> &S) {
    static_assert(kSegChunks == 4, "segment tiles are fetched as one int4 of columns per lane");
    const size_t ln = (size_t)st * 64 + lane;
    S.col = reinterpret_cast<const int4 *>(a.scol)[ln];
    load_four(a.sval, ln, S.v);
    S.rm = a.srow[ln];  // one 16-byte load
    S.diag = a.sdiag[ln];
}

// kRingOnly: a segment whose terms are all LDS-ring terms (and pads, which
// read the ring's zero slot), so nothing is gathered but the constant.
template <typename T, bool kRingOnly>
__device__ inline void seg_gather(const SolveArgs<T> &a, SegSlot<T> &S) {
    if (!kRingOnly) {
#pragma unroll
        for (int c = 0; c < kSegChunks; ++c) S.g[c] = gather_x(a, seg_col(S, c));
    }
    S.bi = Val<T>::of(load_at(a.b, S.rm.x >= 0 ? S.rm.x : 0));
}

template <typename T, bool kRingOnly>
__device__ inline void seg_finish(const SolveArgs<T> &a, SegSlot<T> &S, T *ring) {
    int32_t col[kSegChunks];
#pragma unroll
    for (int c = 0; c < kSegChunks; ++c) col[c] = seg_col(S, c);
    // every chunk reads the ring (terms that are not ring terms read the
    // zero slot and discard it): the reads go out together, with one wait,
    // instead of one branch and one wait per chunk
    T rv[kSegChunks];
    T acc = T(0);
    if (kRingOnly) {
        // columns n + slot, pads n + kRing (the zero slot)
#pragma unroll
        for (int c = 0; c < kSegChunks; ++c) rv[c] = ring[(uint32_t)col[c] - (uint32_t)a.n];
#pragma unroll
        for (int c = 0; c < kSegChunks; ++c) acc = fma(seg_val(S, c), rv[c], acc);
    } else {
#pragma unroll
        for (int c = 0; c < kSegChunks; ++c)
            rv[c] = ring[min((uint32_t)col[c] - (uint32_t)a.n, (uint32_t)kRing)];
        resolve_pending<kSegChunks, false>(a, col, S.g);
#pragma unroll
        for (int c = 0; c < kSegChunks; ++c) {
            const int32_t k = col[c];
            const T v = k >= a.n ? rv[c] : term_value<T>(k, S.g[c]);
            acc = fma(seg_val(S, c), v, acc);
        }
    }
    acc = group_sum(acc, __builtin_amdgcn_readfirstlane(S.rm.y) & 0xff);
    if (S.rm.x >= 0) {
        // scaled here, not at the gather, so the pipeline never waits on it
        const T bi = a.bscale ? S.bi * S.diag : S.bi;
        const T xi = (bi + acc) / S.diag;
        ring[S.rm.y >> 8] = xi;
        __hip_atomic_store(reinterpret_cast<typename Val<T>::Bits *>(a.x) + S.rm.z, Val<T>::bits(xi),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.xout[S.rm.x] = xi;
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
template <typename T, bool kStamp, bool kRingOnly>
__device__ void run_segment(const SolveArgs<T> &a, const int4 d, int lane, T *ring) {
    const long long first = d.x, count = d.y, last = first + count - 1;
    SegSlot<T> S[kDepth];
    // Prologue in the steady state's order (the first half's loads, their
    // gathers, then the second half's loads), so that as many loads follow
    // each gather here as in the loop.  The wait counts the compiler places
    // at the loop head cover both ways in; with the gathers issued last, a
    // full memory round trip would be waited out once per kDepth tiles.
#pragma unroll
    for (int k = 0; k < kDepth / 2; ++k) seg_load(a, min(first + k, last), lane, S[k]);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kDepth / 2; ++k) seg_gather<T, kRingOnly>(a, S[k]);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = kDepth / 2; k < kDepth; ++k) seg_load(a, min(first + k, last), lane, S[k]);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    for (long long base = 0; base < count; base += kDepth) {
#pragma unroll
        for (int k = 0; k < kDepth; ++k) {
            const long long t = base + k;
            seg_finish<T, kRingOnly>(a, S[k], ring);
            if (kStamp && lane == 0) a.stamps[a.nitems + first + t] = __builtin_amdgcn_s_memrealtime();
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            seg_gather<T, kRingOnly>(a, S[(k + kDepth / 2) % kDepth]);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            seg_load(a, min(first + t + kDepth, last), lane, S[k]);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// ----------------------------------------------------------------- kernel --

// kRingSegs: every segment of the plan is flagged ring-only, and the
// instance carries only that (lighter) segment loop; otherwise the general
// loop runs every segment, ring-only ones included.
template <typename T, bool kStamp, int kReg, bool kRingSegs, bool kCol16>
__global__ void __launch_bounds__(64) solve_tiles(SolveArgs<T> a) {
    __shared__ T ring[kRing + 1];  // x of the segment's last kRing rows, then a zero slot
    const int lane = threadIdx.x;
    if (lane == 0) ring[kRing] = T(0);
    if (kStamp && blockIdx.x == 0 && lane == 0) a.stamps[a.start_slot] = __builtin_amdgcn_s_memrealtime();
    // this wave's queue: its first item, stride and end
    const bool on_chain = (long long)blockIdx.x < a.wchain;
    const long long stride = on_chain ? a.wchain : a.waves - a.wchain;
    const long long end = on_chain ? a.nchain : a.nitems;
    long long i = on_chain ? (long long)blockIdx.x : a.nchain + ((long long)blockIdx.x - a.wchain);
    if (i >= end) return;
    if (a.skip && __hip_atomic_load(a.skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    int4 d = unpack_item(load_item(a, i, lane));
    Tile<T, kReg> cur;
    if (!is_segment(d)) load_tile<kCol16>(a, d, lane, cur);
    int wnext = load_item(a, i + stride, lane);  // raw descriptor of the next item
    for (;;) {
        const long long in = i + stride, inn = in + stride;
        if (is_segment(d)) {
            run_segment<T, kStamp, kRingSegs>(a, d, lane, ring);
            if (kStamp && lane == 0) a.stamps[i] = __builtin_amdgcn_s_memrealtime();
            if (in >= end) break;
            d = unpack_item(wnext);
            if (!is_segment(d)) load_tile<kCol16>(a, d, lane, cur);
            wnext = load_item(a, inn, lane);
            i = in;
            continue;
        }
        const int4 dnext = unpack_item(wnext);
        // 1. every gather of the current tile in flight
        int32_t col[kReg];
        typename Val<T>::Bits g[kReg];
#pragma unroll
        for (int c = 0; c < kReg; ++c) {
            col[c] = tile_col<kCol16>(cur, c, lane);
            g[c] = gather_x(a, col[c]);
        }
        const bool lead = tile_lead(cur.d, lane);
        const T braw = Val<T>::of(load_at(a.b, lead ? cur.row : 0));
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        // 2. the next tile's terms and the descriptor after it
        Tile<T, kReg> nxt;
        const bool nwide = in < end && !is_segment(dnext);
        load_tile<kCol16>(a, nwide ? dnext : d, lane, nxt);
        const int wnn = load_item(a, inn, lane);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        // 3. wait for the gathers, accumulate
        resolve_pending<kReg, true>(a, col, g);
        T acc = T(0);
#pragma unroll
        for (int c = 0; c < kReg; ++c) acc = fma(tile_val(cur, c, lane), term_value<T>(col[c], g[c]), acc);
        // 4. rows longer than the register chunks: the rest, kReg
        //    chunks at a time, each group's loads and gathers issued together
        //    (the chunk count is uniform over the wave; pads and inactive
        //    lanes read their own pad slot and count as kPad)
        for (int c0 = kReg; c0 < cur.d.z; c0 += kReg) {
            const bool act = tile_active(cur.d, lane);
            const size_t base = (size_t)cur.d.x * 64 + tile_term_lane(cur.d, lane);
            const int32_t copy = tile_copy(cur.d, lane);
            int32_t kc[kReg];
            T vc[kReg];
            typename Val<T>::Bits gc[kReg];
#pragma unroll
            for (int u = 0; u < kReg; ++u) {
                const size_t idx = base + (size_t)(c0 + u < cur.d.z ? c0 + u : c0) * 64;
                if (kCol16)
                    kc[u] = __builtin_nontemporal_load(a.tcol16 + idx);
                else
                    kc[u] = __builtin_nontemporal_load(a.tcol + idx);
                vc[u] = __builtin_nontemporal_load(a.tval + idx);
            }
#pragma unroll
            for (int u = 0; u < kReg; ++u) {
                kc[u] = decode_col<kCol16>(kc[u], cur.d);
                kc[u] = !act || c0 + u >= cur.d.z || kc[u] == kPad ? kPad : kc[u] + copy;
                gc[u] = gather_x(a, kc[u]);
            }
            resolve_pending<kReg, true>(a, kc, gc);
#pragma unroll
            for (int u = 0; u < kReg; ++u) acc = fma(vc[u], term_value<T>(kc[u], gc[u]), acc);
        }
        // 5. row sums across the row's lanes, then x_i
        acc = group_sum(acc, tile_lg(cur.d));
        if (lead) {
            const T bi = a.bscale ? braw * cur.diag : braw;
            const T xi = (bi + acc) / cur.diag;
            __hip_atomic_store(reinterpret_cast<typename Val<T>::Bits *>(a.x) + cur.d.y + (lane >> tile_lg(cur.d)),
                               Val<T>::bits(xi), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            a.xout[cur.row] = xi;
        }
        if (kStamp && lane == 0) a.stamps[i] = __builtin_amdgcn_s_memrealtime();
        if (in >= end) break;
        cur = nxt;
        d = dnext;
        wnext = wnn;
        i = in;
    }
}

// ------------------------------------------------------------ refinement --
//
// Mixed-precision iterative refinement for plans stored in FP32: with x = 0
// and r = b, each step solves L d = r in FP32 with the schedule above,
// updates x += d in FP64 and recomputes r = b - L x in FP64 from the
// caller's FP64 matrix (one SpMV, a thread per entry of x).  The step's
// largest correction, relative to max(|x_i|, 1e-3 max|x|), is reduced on the
// device; once the error it implies is <= tol every later kernel of the call
// returns at once, so the host enqueues a fixed sequence and never waits.

constexpr int kRefBlock = 256;
constexpr int kRefGrid = 2048;

__device__ inline double block_max(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < kRefBlock / 64; ++k) v = fmax(v, red[k]);
    return v;  // meaningful in thread 0
}

__device__ inline void atomic_max_nonneg(unsigned long long *p, double v) {
    // non-negative doubles order like their bit patterns
    __hip_atomic_fetch_max(p, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline bool refine_done(const sptrsv::Workspace *ws) {
    return __hip_atomic_load(&ws->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

// x = 0, r32 = b rounded; clears the refinement words.
__global__ void __launch_bounds__(kRefBlock) refine_init(const double *__restrict__ b, double *__restrict__ x,
                                                         float *__restrict__ r32, sptrsv::Workspace *ws,
                                                         int32_t n) {
    const int32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid == 0) {
        ws->done = 0u;
        ws->iters = 0u;
    }
    if (tid < sptrsv::kMaxRefine) {
        ws->xmax[tid] = 0ull;
        ws->ratio[tid] = 0ull;
    }
    for (int32_t i = tid; i < n; i += gridDim.x * blockDim.x) {
        x[i] = 0.0;
        r32[i] = (float)b[i];
    }
}

// x += d; per-step max |x| and the step's relative correction (against the
// scale of the step before; the first step replaces x = 0 and is never final).
__global__ void __launch_bounds__(kRefBlock) refine_update(double *__restrict__ x, const float *__restrict__ d32,
                                                           sptrsv::Workspace *ws, int32_t n, int t) {
    __shared__ double red[kRefBlock / 64];
    if (refine_done(ws)) return;
    const double floor_ = t > 0 ? 1e-3 * __longlong_as_double((long long)ws->xmax[t - 1]) : 0.0;
    double xm = 0.0, rm = 0.0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double d = (double)d32[i];
        const double xi = x[i] + d;
        x[i] = xi;
        xm = fmax(xm, fabs(xi));
        // a NaN correction (a failed wait) counts as infinite: never converged
        rm = fmax(rm, t > 0 && d == d ? fabs(d) / fmax(fabs(xi), floor_) : __builtin_inf());
    }
    xm = block_max(xm, red);
    __syncthreads();
    rm = block_max(rm, red);
    if (threadIdx.x == 0) {
        atomic_max_nonneg(&ws->xmax[t], xm);
        atomic_max_nonneg(&ws->ratio[t], rm);
        if (blockIdx.x == 0) __hip_atomic_store(&ws->iters, (unsigned)(t + 1), __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    }
}

// After step t: converged if the error left in x is estimated <= tol (every
// block reads the same words and block 0 raises the flag), else r = b - L x
// in FP64, rounded to FP32 for the next correction.  The correction c_t of step t measures the error x had before it;
// with linear convergence the error after it is about c_t * rho, the rate
// rho estimated as c_t / c_{t-1} (capped at 1; from step 2 on, step 0's
// correction being the whole of x).
__global__ void __launch_bounds__(kRefBlock) refine_residual(const int4 *__restrict__ sys, int32_t nsys,
                                                             const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ col,
                                                             const double *__restrict__ val,
                                                             const double *__restrict__ b,
                                                             const double *__restrict__ x, float *__restrict__ r32,
                                                             sptrsv::Workspace *ws, int32_t n, int t, double tol) {
    if (refine_done(ws)) return;
    const double c = __longlong_as_double((long long)ws->ratio[t]);
    const double rho = t >= 2 ? fmin(1.0, c / __longlong_as_double((long long)ws->ratio[t - 1])) : 1.0;
    if (c * rho <= tol) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            __hip_atomic_store(&ws->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    for (int64_t first = (int64_t)blockIdx.x * kRefBlock; first < n; first += (int64_t)gridDim.x * kRefBlock) {
        // system holding the block's first index (the last with base <= it);
        // a thread steps forward from there to its own
        int lo = 0, hi = nsys - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sys[mid].x <= first) lo = mid; else hi = mid - 1;
        }
        const int32_t i = (int32_t)first + threadIdx.x;
        if (i >= n) continue;
        while (lo + 1 < nsys && sys[lo + 1].x <= i) ++lo;
        const int4 S = sys[lo];
        const int32_t rel = i - S.x, row = S.w + rel / S.z, c = rel % S.z;
        const int32_t e = rp[row + 1];
        double acc = b[i];
        // four entries per round, their loads issued together
        for (int32_t q = rp[row]; q < e; q += 4) {
            int32_t cc[4];
            double vv[4], xx[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t qq = q + u < e ? q + u : q;
                cc[u] = col[qq];
                vv[u] = val[qq];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) xx[u] = x[cc[u] + c];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (q + u < e) acc = fma(-vv[u], xx[u], acc);
        }
        r32[i] = (float)acc;
    }
}

template <typename T>
SolveArgs<T> solve_args(const unsigned char *dev, const sptrsv::Layout *lay, int32_t n,
                        const sptrsv::LaunchShape &sh, uint64_t wait_limit, const void *b, void *x,
                        const unsigned *skip, unsigned long long *stamps = nullptr, int64_t start_slot = 0) {
    SolveArgs<T> a;
    a.stamps = stamps;
    a.start_slot = start_slot;
    a.items = reinterpret_cast<const int4 *>(dev + lay->tiles);
    a.rows = reinterpret_cast<const int32_t *>(dev + lay->rows);
    a.diag = reinterpret_cast<const T *>(dev + lay->diag);
    a.tcol = reinterpret_cast<const int32_t *>(dev + lay->tcol);
    a.tcol16 = reinterpret_cast<const uint16_t *>(dev + lay->tcol);
    a.tval = reinterpret_cast<const T *>(dev + lay->tval);
    a.scol = reinterpret_cast<const int32_t *>(dev + lay->scol);
    a.sval = reinterpret_cast<const T *>(dev + lay->sval);
    a.srow = reinterpret_cast<const int4 *>(dev + lay->srow);
    a.sdiag = reinterpret_cast<const T *>(dev + lay->sdiag);
    a.ws = reinterpret_cast<sptrsv::Workspace *>(const_cast<unsigned char *>(dev) + lay->workspace);
    a.skip = skip;
    a.b = static_cast<const T *>(b);
    a.bscale = 0;
    a.x = reinterpret_cast<T *>(const_cast<unsigned char *>(dev) + lay->xs);
    a.xout = static_cast<T *>(x);
    a.nitems = sh.nitems;
    a.waves = sh.waves;
    a.nchain = sh.nchain;
    a.wchain = sh.chain_waves;
    a.wait_limit = wait_limit;
    a.n = n;
    return a;
}

template <typename T, bool kStamp, bool kCol16>
const void *tiles_kernel_of(const sptrsv::Layout *lay) {
    // the instrumented solve runs every plan with the general segment loop
    const bool ring = !kStamp && lay->ring_segs;
    if (lay->reg_chunks == 8)
        return ring ? reinterpret_cast<const void *>(solve_tiles<T, kStamp, 8, !kStamp, kCol16>)
                    : reinterpret_cast<const void *>(solve_tiles<T, kStamp, 8, false, kCol16>);
    return ring ? reinterpret_cast<const void *>(solve_tiles<T, kStamp, 4, !kStamp, kCol16>)
                : reinterpret_cast<const void *>(solve_tiles<T, kStamp, 4, false, kCol16>);
}
template <typename T, bool kStamp>
const void *tiles_kernel(const sptrsv::Layout *lay) {
    return lay->col16 ? tiles_kernel_of<T, kStamp, true>(lay) : tiles_kernel_of<T, kStamp, false>(lay);
}

template <typename T, bool kStamp = false>
hipError_t launch_tiles(SolveArgs<T> a, int waves, const sptrsv::Layout *lay, hipStream_t s) {
    void *args[] = {&a};
    return hipLaunchCooperativeKernel(tiles_kernel<T, kStamp>(lay), dim3(waves), dim3(64), args, 0, s);
}

template <typename T>
hipError_t launch_prepare(const unsigned char *dev, const sptrsv::Layout *lay, int32_t n, const void *b,
                          const unsigned *skip, hipStream_t s) {
    PrepArgs<T> p;
    p.tiles = reinterpret_cast<const int4 *>(dev + lay->mtiles);
    p.rows = reinterpret_cast<const int32_t *>(dev + lay->mrow);
    p.col = reinterpret_cast<const int32_t *>(dev + lay->mcol);
    p.val = reinterpret_cast<const T *>(dev + lay->mval);
    p.b = static_cast<const T *>(b);
    p.bp = reinterpret_cast<T *>(const_cast<unsigned char *>(dev) + lay->bp);
    p.x = reinterpret_cast<typename Val<T>::Bits *>(const_cast<unsigned char *>(dev) + lay->xs);
    p.n = n;
    p.ntiles = lay->nmtiles;
    p.skip = skip;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (lay->nmtiles + 3) / 4));
    hipLaunchKernelGGL(prepare<T>, dim3(blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

int fill_blocks(int32_t n) { return (int)std::min<int64_t>(2048, ((int64_t)n + 255) / 256); }

// One solve of L x = b in the plan's value type: the right-hand-side step of
// the plan's mode, then the dependent solve.  With kRhsStage the stage
// system runs first (its output y, in the caller's order, is the image's bp
// vector) and shares the main workspace, so a failed wait in either is
// reported by the same status word.  The readiness arrays (x in slot order,
// the main image's and the stage system's) are set to not-ready first.
template <typename T, bool kStamp>
hipError_t solve_once(const unsigned char *dev, const sptrsv::Layout *lay, int32_t n, const sptrsv::LaunchShape &sh,
                      const sptrsv::LaunchShape &sub, uint64_t wait_limit, const void *b, void *x,
                      const unsigned *skip, unsigned long long *stamps, int64_t start_slot, hipStream_t s) {
    using B = typename Val<T>::Bits;
    unsigned char *d = const_cast<unsigned char *>(dev);
    hipError_t e;
    const void *rhs = b;
    int bscale = 0;
    if (lay->rhs_mode == sptrsv::kRhsMPass) {
        if ((e = launch_prepare<T>(dev, lay, n, b, skip, s)) != hipSuccess) return e;
        rhs = d + lay->bp;
    } else {
        const bool stage = lay->rhs_mode == sptrsv::kRhsStage;
        B *xs = reinterpret_cast<B *>(d + lay->xs);
        B *sub_xs = stage ? reinterpret_cast<B *>(d + lay->sub + lay->sub_layout->xs) : nullptr;
        hipLaunchKernelGGL(fill_not_ready<T>, dim3(fill_blocks(n)), dim3(256), 0, s, xs, sub_xs, n, skip);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (stage) {
            T *y = reinterpret_cast<T *>(d + lay->bp);
            SolveArgs<T> sa = solve_args<T>(dev + lay->sub, lay->sub_layout, n, sub, wait_limit, b, y, skip);
            sa.ws = reinterpret_cast<sptrsv::Workspace *>(d + lay->workspace);
            if ((e = launch_tiles<T, false>(sa, sub.waves, lay->sub_layout, s)) != hipSuccess) return e;
            rhs = y;
            bscale = 1;
        }
    }
    SolveArgs<T> a = solve_args<T>(dev, lay, n, sh, wait_limit, rhs, x, skip, stamps, start_slot);
    a.bscale = bscale;
    return launch_tiles<T, kStamp>(a, sh.waves, lay, s);
}

// ------------------------------------------------------------ hop probe --
//
// Latency of one dependency hop as the solve sees it: one lane of workgroup
// 0 and one of workgroup `partner` take turns, each publishing a counter with
// a device-scope store and polling for the other's answer with device-scope
// loads (the solve's publish / wait pair).  Workgroup 0 times `hops` turns
// with the real-time clock.  Workgroups are dispatched to the eight XCDs in
// turn, so partner 1 sits on another XCD and partner 8 on the same one.  A
// wait longer than `limit` ticks ends the probe and flags it in out[1].
__global__ void __launch_bounds__(64) hop_probe(unsigned long long *flag, int hops, int partner,
                                                unsigned long long limit, unsigned long long *out) {
    const int b = blockIdx.x;
    if ((b != 0 && b != partner) || threadIdx.x != 0) return;
    const int mine = b == 0 ? 0 : 1;  // turns h with h % 2 == mine are this side's stores
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    unsigned long long failed = 0;
    for (int h = 0; h < hops && !failed; ++h) {
        const unsigned long long want = (unsigned long long)h + 1;
        if ((h & 1) == mine) {
            __hip_atomic_store(flag, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        const unsigned long long w0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
            if (__builtin_amdgcn_s_memrealtime() - w0 > limit) {
                failed = 1;
                break;
            }
        }
    }
    if (b == 0) {
        out[0] = __builtin_amdgcn_s_memrealtime() - t0;
        out[1] = failed;
    }
}

}  // namespace

extern "C" int sptrsv_launch_hop_probe(void *scratch, int hops, int partner, unsigned long long limit,
                                       void *stream) {
    unsigned long long *w = static_cast<unsigned long long *>(scratch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemsetAsync(w, 0, 4 * sizeof(unsigned long long), s);
    if (e != hipSuccess) return (int)e;
    unsigned long long *flag = w, *out = w + 2;
    void *args[] = {&flag, &hops, &partner, &limit, &out};
    return (int)hipLaunchCooperativeKernel(reinterpret_cast<const void *>(hop_probe), dim3(partner + 1), dim3(64),
                                           args, 0, s);
}

extern "C" int sptrsv_device_limits(int *cus, int *max_waves_per_cu) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    // every instance a plan may launch must be co-resident at this count
#define SPTRSV_INSTANCES(C)                                                     \
    reinterpret_cast<const void *>(solve_tiles<double, false, 4, false, C>),    \
        reinterpret_cast<const void *>(solve_tiles<double, false, 8, false, C>), \
        reinterpret_cast<const void *>(solve_tiles<double, false, 4, true, C>),  \
        reinterpret_cast<const void *>(solve_tiles<double, false, 8, true, C>),  \
        reinterpret_cast<const void *>(solve_tiles<float, false, 4, false, C>),  \
        reinterpret_cast<const void *>(solve_tiles<float, false, 8, false, C>),  \
        reinterpret_cast<const void *>(solve_tiles<float, false, 4, true, C>),   \
        reinterpret_cast<const void *>(solve_tiles<float, false, 8, true, C>),   \
        reinterpret_cast<const void *>(solve_tiles<double, true, 4, false, C>),  \
        reinterpret_cast<const void *>(solve_tiles<double, true, 8, false, C>)
    const void *inst[] = {SPTRSV_INSTANCES(false), SPTRSV_INSTANCES(true)};
#undef SPTRSV_INSTANCES
    int most = sptrsv::kMaxWavesPerCU;
    for (const void *k : inst) {
        int b = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, 64, 0);
        if (e != hipSuccess) return (int)e;
        // a kernel that spills to scratch may be held back by the scratch
        // backing even where the occupancy query says it fits: refuse it
        hipFuncAttributes fa;
        e = hipFuncGetAttributes(&fa, k);
        if (e != hipSuccess) return (int)e;
        if (fa.localSizeBytes != 0) return (int)hipErrorInvalidKernelFile;
        most = std::min(most, b);
    }
    *max_waves_per_cu = most;
    return 0;
}

extern "C" int sptrsv_launch_solve(const unsigned char *dev, const sptrsv::Layout *lay, int32_t n,
                                   const sptrsv::LaunchShape *sh, const sptrsv::LaunchShape *sub,
                                   uint64_t wait_limit, const void *b, void *x, unsigned long long *stamps,
                                   int64_t start_slot, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (lay->value_bytes == 4) {
        if (stamps) return (int)hipErrorNotSupported;
        return (int)solve_once<float, false>(dev, lay, n, *sh, *sub, wait_limit, b, x, nullptr, nullptr, 0, s);
    }
    if (stamps)
        return (int)solve_once<double, true>(dev, lay, n, *sh, *sub, wait_limit, b, x, nullptr, stamps, start_slot, s);
    return (int)solve_once<double, false>(dev, lay, n, *sh, *sub, wait_limit, b, x, nullptr, nullptr, 0, s);
}

extern "C" int sptrsv_launch_refined(const unsigned char *dev, const sptrsv::Layout *lay, int32_t n,
                                     const sptrsv::LaunchShape *sh, const sptrsv::LaunchShape *sub,
                                     uint64_t wait_limit, const double *b, double *x, int iterations, double tol,
                                     void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char *d = const_cast<unsigned char *>(dev);
    sptrsv::Workspace *ws = reinterpret_cast<sptrsv::Workspace *>(d + lay->workspace);
    float *r32 = reinterpret_cast<float *>(d + lay->r32);
    float *d32 = reinterpret_cast<float *>(d + lay->d32);
    const int grid = (int)std::min<int64_t>(kRefGrid, ((int64_t)n + kRefBlock - 1) / kRefBlock);
    hipLaunchKernelGGL(refine_init, dim3(std::max(grid, 1)), dim3(kRefBlock), 0, s, b, x, r32, ws, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    // each step: the FP32 solve of L d = r32 (right-hand-side step included)
    for (int t = 0; t < iterations; ++t) {
        if ((e = solve_once<float, false>(dev, lay, n, *sh, *sub, wait_limit, r32, d32, &ws->done, nullptr, 0,
                                          s)) != hipSuccess)
            return (int)e;
        hipLaunchKernelGGL(refine_update, dim3(grid), dim3(kRefBlock), 0, s, x, d32, ws, n, t);
        if ((e = hipGetLastError()) != hipSuccess) return (int)e;
        if (t + 1 == iterations) break;
        hipLaunchKernelGGL(refine_residual, dim3(grid), dim3(kRefBlock), 0, s,
                           reinterpret_cast<const int4 *>(dev + lay->sys), lay->nsys,
                           reinterpret_cast<const int32_t *>(dev + lay->res_rp),
                           reinterpret_cast<const int32_t *>(dev + lay->res_col),
                           reinterpret_cast<const double *>(dev + lay->res_val), b, x, r32, ws, n, t, tol);
        if ((e = hipGetLastError()) != hipSuccess) return (int)e;
    }
    return 0;
}
