// plan.hpp -- internal state of a plan and the host passes that build it.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "sptrsv.h"

namespace sptrsv {

// Host worker threads for the analysis passes: the cores, at most 16.
inline int hw_threads() {
    unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h, 16u));
}

// Run f(begin, end, worker) over [0, count) on up to `threads` workers.
template <class F>
void parallel_ranges(int64_t count, int threads, F &&f) {
    if (count <= 0) return;
    threads = (int)std::min<int64_t>(threads, std::max<int64_t>(1, count / 256));
    if (threads <= 1) {
        f((int64_t)0, count, 0);
        return;
    }
    std::vector<std::thread> pool;
    const int64_t step = (count + threads - 1) / threads;
    for (int w = 0; w < threads; ++w) {
        const int64_t b = w * step, e = std::min(count, b + step);
        if (b >= e) break;
        pool.emplace_back([&, b, e, w] { f(b, e, w); });
    }
    for (auto &t : pool) t.join();
}

// Allocator whose resize leaves new elements uninitialised, so that a large
// buffer can be cleared by several threads instead of one.
template <class T>
struct UninitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = UninitAlloc<U>;
    };
    UninitAlloc() = default;
    template <class U>
    UninitAlloc(const UninitAlloc<U> &) noexcept {}
    template <class U>
    void construct(U *p) noexcept {
        ::new ((void *)p) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};

// Zero `bytes` bytes at `p` with the host's worker threads, one contiguous
// range each (the page faults of a fresh allocation are taken in parallel).
inline void parallel_zero(unsigned char *p, size_t bytes) {
    constexpr size_t kBlock = size_t(1) << 20;
    const int64_t blocks = (int64_t)((bytes + kBlock - 1) / kBlock);
    const int threads = (int)std::min<int64_t>(hw_threads(), std::max<int64_t>(1, blocks / 4));
    if (threads <= 1) {
        std::memset(p, 0, bytes);
        return;
    }
    std::vector<std::thread> pool;
    const int64_t step = (blocks + threads - 1) / threads;
    for (int w = 0; w < threads; ++w) {
        const size_t b = (size_t)(w * step) * kBlock;
        if (b >= bytes) break;
        const size_t e = std::min(bytes, (size_t)((w + 1) * step) * kBlock);
        pool.emplace_back([p, b, e] { std::memset(p + b, 0, e - b); });
    }
    for (auto &t : pool) t.join();
}

// Error carried out of the host passes; the C ABI turns it into a status
// code and a thread-local message.
struct Error {
    sptrsv_status code;
    std::string msg;
};

// Shape constants of the device image shared by the packer and the kernels.
constexpr int kSegChunks = 4;     // chunks per segment tile
constexpr int kRing = 2048;       // x values a segment wave keeps in LDS (power of two)
constexpr int kNarrowTiles = 2;   // a level of at most this many segment tiles is narrow
constexpr int kMinSegLevels = 16; // shortest run of narrow levels executed as a segment
constexpr int kSegDepth = 8;      // segment software-pipeline depth; segments hold a multiple of it
constexpr int kStageSegTiles = 4; // a stage of a stage system is one segment if it needs at most this
                                  // many segment tiles per level

constexpr int kMaxRefine = 16;    // refinement iterations per call (slots in the workspace)

// Most single-wave workgroups per CU the cooperative solve grid may use.
// Every wave must be resident for the grid to drain (a wave that never
// starts holds items others wait on), and 8 per CU is what the kernels'
// resources prove: at most 256 VGPRs (2 waves per SIMD, 4 SIMDs) and a
// 16,392-byte LDS ring, 8 of which fit in 160 KB of LDS even at a 2 KB
// allocation granularity (9 would need a granularity below ~1.8 KB).  The
// occupancy query can report more; it is capped here.
constexpr int kMaxWavesPerCU = 8;

// How the solve applies the rewritten right-hand side b' = b + M b.
enum RhsMode : int32_t {
    kRhsNone = 0,   // no b-terms: the solve reads b
    kRhsMPass = 1,  // a parallel SpMV over M tiles writes b' before the solve
    kRhsStage = 2,  // b' = D y with L_B y = b, L_B the block-diagonal part of L
                    // inside the stages (stage_of_level equal): one more solve
                    // whose chain is the depth of a stage, reading nnz(L_B)
                    // entries instead of nnz(M)
};

struct Layout;

// Launch of one cooperative solve: work items, how many of them form the
// chain queue (the rest are sinks), waves, and how many waves serve the
// chain queue.  One queue: nchain = nitems and chain_waves = waves.
struct LaunchShape {
    int64_t nitems = 0;
    int64_t nchain = 0;
    int waves = 0;
    int chain_waves = 0;
};

// Device image layout: byte offsets of each section inside the caller's
// buffer.  Sections are 256-byte aligned.  Values (diag, tval, sval, sdiag)
// are FP64, or FP32 in a plan stored in FP32 (value_bytes 4).
struct Layout {
    int value_bytes = 8;
    int reg_chunks = 4;  // wide-tile chunks the solve kernel holds in registers (4 or 8)
    int ring_segs = 0;   // every segment reads only its LDS ring (the lighter kernel instance)
    int col16 = 0;       // wide-tile columns as 16-bit distances back from the tile's first slot
    int32_t rhs_mode = kRhsNone;
    size_t sub = 0;               // kRhsStage: offset of the stage system's image
    const Layout *sub_layout = nullptr;
    size_t workspace = 0;  // Workspace block
    size_t tiles = 0;      // int4[nitems]: wide tile {chunk_off, row_off, nchunks,
                           //   nrows<<16 | first copy<<8 | log2 copies<<4 | log2 lanes}
                           //   or segment {first segment tile, count, 0, 1<<31}
    size_t rows = 0;       // int32[n]      row id of each packed slot
    size_t diag = 0;       // double[n]     diagonal of each packed slot
    size_t tcol = 0;       // int32[64*nchunks] term column: slot of the x-term's row, INT32_MIN pad;
                           //   col16: uint16[64*nchunks] first slot of the tile minus that slot, 0 pad
    size_t tval = 0;       // double[64*nchunks] term coefficient (x-terms negated)
    size_t scol = 0;       // int32[nseg_tiles][64][kSegChunks] as tcol, plus n + ring index for LDS x-terms
                           // (n + kRing, a zero slot, for the pads of a segment without gathers)
    size_t sval = 0;       // double[nseg_tiles][64][kSegChunks]
    size_t srow = 0;       // int32[nseg_tiles][64][4]: row finished by the lane (-1 if none),
                           //   log2 lanes per row | ring index << 8, its slot, 0
    size_t sdiag = 0;      // double[nseg_tiles][64] its diagonal
    // right-hand side b' = b + M b, computed by a parallel pass before the solve
    size_t mtiles = 0;     // int4[nmtiles]: {chunk_off, row_off, nchunks, nrows<<8 | log2 lanes}
    size_t mrow = 0;       // int32[n]  device row of each M-tile slot
    size_t mcol = 0;       // int32[64*mchunks] device index of b_j (INT32_MIN pad)
    size_t mval = 0;       // double[64*mchunks] M_ij
    size_t bp = 0;         // double[n] b' (kRhsMPass) or y (kRhsStage), device indices
    size_t xs = 0;         // double[n] x in slot order: the solve's readiness flags and gathered values
    int64_t nmtiles = 0;
    int64_t nnz_rhs = 0;   // entries the right-hand-side step reads (M, or L_B)
    // FP32 plans only: what iterative refinement needs next to the FP32
    // schedule -- the caller's matrices in FP64 for the residual, and two
    // FP32 vectors (residual, correction) indexed like b and x
    size_t sys = 0;        // int4[nsys] {device base, rows, right-hand sides, first residual row}
    size_t res_rp = 0;     // int32[res_rows + 1]
    size_t res_col = 0;    // int32[res_nnz] device index of column l for right-hand side 0: base + l*k
    size_t res_val = 0;    // double[res_nnz]
    size_t r32 = 0;        // float[n]
    size_t d32 = 0;        // float[n]
    int32_t nsys = 0;
    int64_t res_rows = 0, res_nnz = 0;
    size_t total = 0;
};

// Per-solve bookkeeping shared by the kernels (lives at layout.workspace).
struct Workspace {
    unsigned int status;  // 0 ok, else SPTRSV_ERR_TIMEOUT; cleared by sptrsv_check
    unsigned int done;    // refinement: converged, later steps skip their work
    unsigned int iters;   // refinement: corrections applied by the last call
    unsigned int pad0;
    // refinement, per iteration t: max |x| after the update (FP64 bits), and
    // the largest correction relative to max(|x_i|, 1e-3 max|x|)
    unsigned long long xmax[kMaxRefine];
    unsigned long long ratio[kMaxRefine];
    unsigned long long pad[30];
};
static_assert(sizeof(Workspace) == 512, "workspace block is 512 bytes");

struct Plan {
    // ---- analysed matrix (Sec. II / IV); for an upper-triangular input the
    // matrix is held with its index order reversed (row i <-> n-1-i), which
    // makes it lower triangular, and only the device image uses the caller's
    // indices
    int32_t n = 0;
    bool upper = false;
    int32_t batch_count = 0;
    // the caller's systems as the plan holds them: rows, right-hand sides
    // and device base of each (one entry for an unbatched plan)
    std::vector<int32_t> sys_n, sys_k;
    std::vector<int64_t> sys_base;
    // value type of the device image: 64 (FP64) or 32 (FP32 storage and
    // arithmetic, refined to FP64 by sptrsv_solve_refined)
    int precision = 64;
    // right-hand-side step: requested (-1 = chosen from the sizes of M and
    // L_B) and, for kRhsStage, the plan of the stage system L_B
    int32_t rhs_request = -1;
    // row-to-wavefront tiling: a row of len terms gets the smallest power of
    // two g of lanes with len <= terms_per_lane * g (capped at 64)
    int terms_per_lane = 4;
    // work queues of the device schedule: 2 = chain and sinks apart, 1 = one
    // queue of every row in level order
    int queues = 2;
    std::unique_ptr<struct Plan> sub;
    bool is_sub = false;  // a stage system (no residual data, no sub-plan)
    // a stage system's stage of each row: its diagonal blocks are
    // independent systems, and a narrow one is packed as one segment
    std::vector<int32_t> comp;
    std::vector<int32_t> rp, ci;
    std::vector<double> val;
    std::vector<int32_t> level;  // level of each row of L
    int32_t nlev = 0;
    std::vector<int32_t> level_ptr, level_rows;

    // ---- rewrite (Sec. III)
    sptrsv_policy policy{};
    std::vector<int32_t> stage_of_level;
    std::vector<int64_t> delta_of_level;
    int32_t nstages = 0;
    std::vector<int64_t> lp_ptr, m_ptr;  // L' and M in CSR
    std::vector<int32_t> lp_col, m_col;
    std::vector<double> lp_val, m_val;
    // M's entries are held (m_col, m_val) unless the stage solve replaces
    // the M pass; m_ptr always holds its row counts
    bool m_kept = true;
    int64_t nnz_m() const { return m_ptr.empty() ? 0 : m_ptr.back(); }
    std::vector<int32_t> level_rw;  // levels of L'
    int32_t nlev_rw = 0;
    std::vector<int32_t> sched_ptr, sched_rows;

    // ---- packed device image (host copy) and its layout
    Layout layout;
    std::vector<unsigned char, UninitAlloc<unsigned char>> image;
    int64_t ntiles = 0;      // work items (wide tiles and segments)
    int64_t nchain = 0;      // of which the chain queue (the rest hold only rows nothing depends on)
    int64_t chain_work = 0, sink_work = 0;  // 64-lane chunks plus rows packed in each queue
    int64_t nnz_streamed = 0;  // entries of L' the image holds (copies sharing terms count once)
    int64_t nnz_col16 = 0;     // of them, wide-tile terms whose column is stored in 16 bits
    int64_t nchunks = 0;
    int32_t nseg = 0;        // segments
    int64_t nseg_tiles = 0;  // tiles inside segments
    int32_t comp_segs = 0;   // segments that are whole independent stages
    int32_t ring_segs = 0;   // segments whose terms all come from the LDS ring
    // executed level (of L') whose rows each item and each segment tile
    // finish, -1 for segment items and padding tiles: the map of the
    // completion stamps of an instrumented solve
    std::vector<int32_t> stamp_level;

    // ---- device state
    void *dev = nullptr;
    bool uploaded = false;
    int cus = 0;                         // compute units of the device uploaded to
    int max_waves_per_cu = 0;            // co-resident solve workgroups per CU
    int waves_per_cu = 0;                // requested; 0 = chosen from the plan's shape
    int chain_share = 0;                 // chain queue's share of the waves requested (per mille); 0 = chosen
    uint64_t wait_limit = 200000000ull;  // 2 s at 100 MHz

    // ---- captured solve graph (sptrsv_solve_graph)
    void *graph_exec = nullptr;          // hipGraphExec_t
    void *capture_stream = nullptr;      // hipStream_t owned by the plan
    const void *graph_b = nullptr, *graph_x = nullptr;
    int graph_waves = 0, graph_chain_waves = 0;
    ~Plan();
};

// analyse.cpp
void validate_csr(int32_t n, const int32_t *rp, const int32_t *ci, const double *val);
void analyse(Plan &p, int32_t n, const int32_t *rp, const int32_t *ci, const double *val);
void analyse_upper(Plan &p, int32_t n, const int32_t *rp, const int32_t *ci, const double *val);
void analyse_batch(Plan &p, int32_t count, const int32_t *n, const int32_t *const *rp,
                   const int32_t *const *ci, const double *const *val, const int32_t *k);
void level_sets(int32_t n, const int32_t *level, int32_t nlev, std::vector<int32_t> &ptr,
                std::vector<int32_t> &rows);

// rewrite.cpp
void validate_policy(const sptrsv_policy &pol);
void rewrite(Plan &p, const sptrsv_policy &pol);
// M's entries of a plan whose rewrite did not store them (same values)
void materialise_m(Plan &p);

// pack.cpp
void pack(Plan &p);
// entries of L_B (entries of L whose two rows' levels share a stage)
int64_t stage_system_nnz(const Plan &p);
// right-hand-side step for nnz_m entries of M and nnz_b of L_B
int32_t choose_rhs(const Plan &p, int64_t nnz_m, int64_t nnz_b);

}  // namespace sptrsv

// solve.hip -- kernel launchers (return a hipError_t as int).  b and x are
// double or float as lay->value_bytes says.
// With stamps (FP64 plans only), the instrumented kernel also writes the
// real-time clock (100 MHz) as every item and every segment tile completes
// (slots [0, nitems) and nitems + segment tile), and its start at start_slot.
// sub_nitems / sub_waves: the stage system's solve (kRhsStage).
extern "C" int sptrsv_launch_solve(const unsigned char *dev, const sptrsv::Layout *lay, int32_t n,
                                   const sptrsv::LaunchShape *sh, const sptrsv::LaunchShape *sub,
                                   uint64_t wait_limit, const void *b, void *x, unsigned long long *stamps,
                                   int64_t start_slot, void *stream);
// mlp.hip -- cost model kernels (FP32 parameter vector of 4673 floats)
extern "C" size_t sptrsv_launch_mlp_workspace(int32_t m);
extern "C" int sptrsv_launch_mlp_forward(const float *params, const float *X, float *Y, int32_t m, void *stream);
extern "C" int sptrsv_launch_mlp_grad(const float *params, const float *X, const float *T, int32_t m, float *grad,
                                      float *loss, void *workspace, void *stream);
// device address (for the current device) and size of the gradient's static workspace
extern "C" int sptrsv_mlp_static_workspace(void **ptr, size_t *bytes);
extern "C" int sptrsv_launch_mlp_adam(float *params, const float *grad, float *m1, float *m2, int32_t step,
                                      float lr, float beta1, float beta2, float eps, void *stream);
// FP32 plans: `iterations` refinement steps on x (FP64), all on stream; the
// steps after convergence (correction <= tol) skip their work on the device.
extern "C" int sptrsv_launch_refined(const unsigned char *dev, const sptrsv::Layout *lay, int32_t n,
                                     const sptrsv::LaunchShape *sh, const sptrsv::LaunchShape *sub,
                                     uint64_t wait_limit, const double *b, double *x, int iterations,
                                     double tol, void *stream);
extern "C" int sptrsv_device_limits(int *cus, int *max_waves_per_cu);
// hop latency probe: scratch = 4 device uint64 (flag, unused, ticks, failed)
extern "C" int sptrsv_launch_hop_probe(void *scratch, int hops, int partner, unsigned long long limit,
                                       void *stream);
