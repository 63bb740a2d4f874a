/*
 * sptrsv.h -- C ABI of a level-scheduled sparse lower-triangular solver for
 * AMD Instinct MI355X (gfx950) with host-side equation rewriting.
 *
 * Method: Yilmaz, "Graph Transformation and Specialized Code Generation for
 * Sparse Triangular Solve (SpTRSV)", arXiv:2103.11445.
 *   - the solve of L x = b by forward substitution over CSR and the
 *     dependency DAG of L, grouped into levels: Sec. II (Algorithm 1, Fig. 1);
 *   - equation rewriting of rows in thin levels, which moves them to earlier
 *     levels and removes synchronisation points: Sec. III (Fig. 2, Fig. 3);
 *   - matrix analysis (rows, nonzeros, DAG, level sets, per-level
 *     statistics) feeding the rewrite: Sec. IV.
 *
 * Conventions shared by every entry point:
 *   - Nothing throws across this boundary; each call returns a status code
 *     and, on failure, leaves a message readable with sptrsv_last_error().
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device allocations on the GPU that is current when the call is made.
 *   - Streams are hipStream_t passed as void* (NULL = the null stream).
 *   - L is n x n lower triangular in CSR with int32 indices and FP64 values:
 *     row_ptr[0] = 0, row_ptr non-decreasing, within each row the columns
 *     strictly increase and the last entry is the diagonal (non-zero).
 *   - A plan is not thread-safe: calls on one plan must not overlap, and two
 *     solves of one plan must not run concurrently on different streams
 *     (they share the plan's device workspace).  Distinct plans are
 *     independent.
 */
#ifndef SPTRSV_H
#define SPTRSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque plan.  Owned by the library; release with sptrsv_plan_destroy. */
typedef struct sptrsv_plan_s *sptrsv_plan;

typedef enum {
    SPTRSV_OK = 0,
    SPTRSV_ERR_ARG = 1,      /* null pointer, negative size, invalid policy field,
                                b aliasing x, buffer too small */
    SPTRSV_ERR_CSR = 2,      /* row_ptr[0] != 0 or decreasing, empty row, column
                                out of range, columns not strictly increasing,
                                entry above the diagonal */
    SPTRSV_ERR_DIAG = 3,     /* a row whose last entry is not its diagonal, or a
                                zero diagonal */
    SPTRSV_ERR_OVERFLOW = 4, /* the rewritten system does not fit int32 device
                                indexing, or n x value bytes reaches 2^32 (x
                                and b are addressed by 32-bit offsets) */
    SPTRSV_ERR_OOM = 5,      /* host allocation failed */
    SPTRSV_ERR_HIP = 6,      /* a HIP runtime call failed (message has details) */
    SPTRSV_ERR_STATE = 7,    /* solve before upload, or after a rewrite made the
                                uploaded image stale */
    SPTRSV_ERR_TIMEOUT = 8   /* reported by sptrsv_check: a dependency wait in
                                the kernel gave up (the solution is invalid) */
} sptrsv_status;

/* Which levels to rewrite (Sec. III: rows of thin levels are moved into an
 * earlier level by substituting the equations of their dependencies; the
 * paper chooses them by hand, Sec. IV and V).
 *
 * Levels are cut into consecutive stages.  A stage keeps its first level a;
 * every row of a later level l of the stage has its dependencies of level
 * >= a substituted away (original equations, latest dependency first, equal
 * x terms merged: Fig. 2 and Fig. 3), so after rewriting it depends only on
 * rows of earlier stages.  Level 0 always opens stage 0.  Level l >= 1 joins
 * the current stage when:
 *   SPTRSV_POLICY_NONE       never (plain level-set schedule);
 *   SPTRSV_POLICY_THRESHOLD  width(l) <= max_width, the stage holds fewer than
 *                            max_depth levels, the entries added by all
 *                            absorbed levels stay <= floor(max_fill * nnz(L)),
 *                            and nnz(L') + nnz(M) stays <= max_entries;
 *   SPTRSV_POLICY_EXPLICIT   absorb[l] != 0 (l < absorb_len) and
 *                            nnz(L') + nnz(M) stays <= max_entries;
 *   SPTRSV_POLICY_LEARNED    the stage holds fewer than max_depth levels, the
 *                            budgets of THRESHOLD hold (max_fill,
 *                            max_entries; max_width is ignored), and the
 *                            cost model `model` (see sptrsv_mlp_forward)
 *                            predicts that merging l into the stage adds less
 *                            time than l costs as a stage of its own.  The
 *                            model maps the shape of a group of rows
 *                            (sptrsv_plan_level_features) to the log of its
 *                            time in microseconds; it runs on the current
 *                            device, once or twice per level, during the call.
 * Entries added by absorbing l: over its rows, (x-terms + b-terms after
 * rewriting) - (off-diagonals before), counted symbolically. */
enum {
    SPTRSV_POLICY_NONE = 0,
    SPTRSV_POLICY_THRESHOLD = 1,
    SPTRSV_POLICY_EXPLICIT = 2,
    SPTRSV_POLICY_LEARNED = 3
};

typedef struct {
    int32_t kind;           /* SPTRSV_POLICY_* */
    int32_t max_width;      /* >= 0; a level is thin if it has <= max_width rows */
    int32_t max_depth;      /* >= 1; levels per stage, including its first */
    double max_fill;        /* >= 0; added entries budget as a multiple of nnz(L) */
    int64_t max_entries;    /* >= 0; cap on nnz(L') + nnz(M) */
    const uint8_t *absorb;  /* host, absorb_len bytes; EXPLICIT only (may be NULL
                               when absorb_len == 0); read during the call only */
    int32_t absorb_len;     /* >= 0 */
    const float *model;     /* LEARNED only: device, SPTRSV_MLP_PARAMS floats; read
                               during the call only */
} sptrsv_policy;

/* Fills *p with THRESHOLD, max_width 4, max_depth 64, max_fill 0.25,
 * max_entries INT32_MAX, no mask, no model. */
void sptrsv_policy_default(sptrsv_policy *p);

/* Matrix analysis (Sec. IV; DAG and level sets of Sec. II).  Validates and
 * copies L (host arrays, read during the call only; the caller keeps
 * ownership), builds the level of every row (0 for rows without
 * off-diagonals, else 1 + the deepest dependency) and the level sets.  The
 * new plan carries the plain schedule (as after SPTRSV_POLICY_NONE).
 * n == 0 gives an empty plan whose solve does nothing.  On error *out is
 * set to NULL.  Errors: ARG (n < 0, null pointer with n > 0 or out NULL),
 * CSR, DIAG, OOM. */
sptrsv_status sptrsv_analyse(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             const double *val, sptrsv_plan *out);

/* Analysis of an UPPER-triangular U (CSR, columns strictly increasing, the
 * diagonal FIRST in each row, non-zero), for the backward substitution
 * U x = b that follows the forward solve in LU / incomplete-LU
 * preconditioners.  The plan holds U with its index order reversed (row i of
 * the plan is row n-1-i of U), which is lower triangular, so rewriting
 * (Sec. III works on the dependency graph, whatever its orientation) and
 * solving are unchanged; sptrsv_solve takes b and x in U's own order.  The
 * introspection calls (levels, stages, schedule, export) report the reversed
 * matrix.  Errors as sptrsv_analyse (CSR also for an entry below the
 * diagonal). */
sptrsv_status sptrsv_analyse_upper(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                   const double *val, sptrsv_plan *out);

/* Analysis of a batch: `count` lower-triangular systems (n[j], row_ptr[j],
 * col_idx[j], val[j] as for sptrsv_analyse, host, read during the call), the
 * j-th with k[j] >= 1 right-hand sides.  The plan is the block-diagonal union
 * of k[j] copies of each matrix, so one solve (one launch, the levels of all
 * systems interleaved) handles every system and every right-hand side.
 * sptrsv_solve then takes b and x as the concatenation, in order j = 0..,
 * of row-major n[j] x k[j] blocks (entry (i, c) of system j at
 * base_j + i*k[j] + c, base_j = sum_{j' < j} n[j'] k[j']).  The union
 * is numbered the same way: copy c of row i of system j is union row
 * base_j + i*k[j] + c, so the copies of a row share its level and sit side by
 * side in the schedule, and the gathers of a term for all right-hand sides
 * read one contiguous run of x.  Introspection reports the union.  Errors: as
 * sptrsv_analyse (message names the system), ARG (k < 1, null arrays),
 * OVERFLOW (union beyond int32). */
sptrsv_status sptrsv_analyse_batch(int32_t count, const int32_t *n, const int32_t *const *row_ptr,
                                   const int32_t *const *col_idx, const double *const *val,
                                   const int32_t *k, sptrsv_plan *out);

/* Equation rewriting (Sec. III) under *policy, always starting again from
 * the analysed L (so repeated calls do not compound).  Builds the rewritten
 * rows L' (x-terms plus the unchanged diagonal), the right-hand-side
 * combination M (b'_i = b_i + sum_j M_ij b_j), re-levels L' (emptied levels
 * vanish) and packs the device image.  Host only; invalidates a previous
 * upload.  Errors: ARG (bad policy), OVERFLOW (the device image would need
 * more than INT32_MAX 64-lane chunks or entries, or n times the value size
 * reaches 2^32 bytes: the kernels address x and b by 32-bit offsets), OOM. */
sptrsv_status sptrsv_rewrite(sptrsv_plan plan, const sptrsv_policy *policy);

/* Size in bytes of the device buffer the current plan needs (image plus
 * workspace). */
sptrsv_status sptrsv_device_bytes(sptrsv_plan plan, size_t *bytes);

/* Copies the packed plan into dev_buf (device, >= sptrsv_device_bytes, owned
 * by the caller, 256-byte aligned, must stay allocated while the plan is
 * solved with) on stream, and waits for the copy to finish.  The plan
 * remembers dev_buf.  Errors: ARG (null, too small, misaligned), HIP (also
 * when a solve kernel was built with scratch memory, whose co-residency the
 * cooperative launch cannot rely on). */
sptrsv_status sptrsv_upload(sptrsv_plan plan, void *dev_buf, size_t bytes, void *stream);

/* Solves L x = b (device arrays of n doubles, b != x, neither overlapping
 * the plan buffer) with the uploaded schedule: enqueues on stream the
 * right-hand-side step (see sptrsv_set_rhs_mode: one pass over M, or a fill
 * and one cooperative solve of the stage system; a fill of x without
 * b-terms) and one cooperative solve kernel, and returns without waiting.
 * Every row waits only for the rows it still depends on (per-row readiness,
 * in level order), so the level structure bounds the critical path.
 * Numerical problems are not reported (zero diagonals were rejected by
 * analyse); a dependency wait that exceeds the wait limit is reported by
 * sptrsv_check.  Errors: ARG, STATE (not uploaded, stale, or stored in
 * FP32), HIP. */
sptrsv_status sptrsv_solve(sptrsv_plan plan, const double *b, double *x, void *stream);

/* As sptrsv_solve (FP64 plans), through a HIP graph: its launches are
 * captured once (on a stream the plan owns) for these b and x and replayed
 * on `stream` by later calls with the same pointers (a different b, x, launch
 * shape, rewrite or upload captures again).  For callers that replay one
 * solve many times.  Errors: as sptrsv_solve, HIP (capture refused). */
sptrsv_status sptrsv_solve_graph(sptrsv_plan plan, const double *b, double *x, void *stream);

/* How a solve applies the rewritten right-hand side b' = b + M b (Sec. III,
 * Fig. 3's updated b entries).  The b-terms depend on nothing the solve
 * computes, so they are taken off the dependent chain in one of two ways:
 *   SPTRSV_RHS_MPASS  a fully parallel pass over the entries of M before the
 *                     solve (reads nnz(M) entries);
 *   SPTRSV_RHS_STAGE  on the rows S of a stage, b'_S = D_S L_SS^-1 b_S (the
 *                     rewriting eliminates exactly the in-stage couplings), so
 *                     b' = D y with L_B y = b, L_B the block-diagonal part of
 *                     L inside the stages: one more solve, by the same kernel,
 *                     whose chain is one stage deep (the stages are
 *                     independent) and which reads nnz(L_B) <= nnz(L) entries;
 *                     a stage of at most a few segment tiles per level is
 *                     solved start to finish by one wave (its values kept in
 *                     LDS), the others level by level across the grid.
 *   SPTRSV_RHS_AUTO   (default) the stage solve when nnz(M) > 2 nnz(L_B).
 * The results agree up to rounding.  Repacks the host image (the upload
 * becomes stale); the rewrite and its introspection are unchanged.
 * Errors: ARG (unknown mode), OVERFLOW, OOM. */
enum { SPTRSV_RHS_AUTO = 0, SPTRSV_RHS_MPASS = 1, SPTRSV_RHS_STAGE = 2 };
sptrsv_status sptrsv_set_rhs_mode(sptrsv_plan plan, int32_t mode);

/* Row-to-wavefront tiling of the device schedule: within a level, a row of
 * len terms gets g lanes of a 64-lane tile, g the smallest power of two with
 * len <= terms_per_lane * g (capped at 64), and a tile holds 64 / g rows of
 * equal g.  terms_per_lane in {1, 2, 4, 8, 16}; default 4.  Fewer terms per
 * lane spread a row over more lanes (shorter per-lane chains, fewer rows per
 * tile); more pack more rows per tile.  Repacks the host image (the upload
 * becomes stale); the schedule and the rewrite are unchanged.  For tuning the
 * launch to a matrix (the batched benchmark's autotuner searches it).
 * Errors: ARG, OVERFLOW, OOM. */
sptrsv_status sptrsv_set_tiling(sptrsv_plan plan, int32_t terms_per_lane);

/* Value type of the device image: 64 (FP64, the default) or 32.  A plan
 * stored in FP32 keeps every value of L' and M and every diagonal rounded to
 * nearest FP32 and solves in FP32 arithmetic (sptrsv_solve_fp32), with x in
 * FP32; it also carries the caller's matrices in FP64 for the residual of
 * sptrsv_solve_refined.  Repacks the host image (the upload becomes stale);
 * the schedule, the rewrite and the introspection calls are unchanged.  The
 * precision survives later rewrites.  Errors: ARG (bits not 32 or 64),
 * OVERFLOW, OOM. */
sptrsv_status sptrsv_set_precision(sptrsv_plan plan, int32_t bits);

/* As sptrsv_solve for a plan stored in FP32: b and x are device arrays of n
 * floats.  Errors: as sptrsv_solve; STATE for a plan stored in FP64. */
sptrsv_status sptrsv_solve_fp32(sptrsv_plan plan, const float *b, float *x, void *stream);

/* Mixed-precision iterative refinement for a plan stored in FP32 (an
 * extension; the paper's solve is a single pass): b and x are device arrays
 * of n doubles.  With x = 0 and r = b, each step solves L d = r (r rounded to
 * FP32) with the FP32 schedule, updates x += d in FP64 and recomputes
 * r = b - L x in FP64 with the caller's FP64 matrix.  Step t's correction
 * c_t = max_i |d_i| / max(|x_i|, 1e-3 max_j |x_j|) (step 0's counts as
 * infinite) measures the error before the step; the error after it is
 * estimated as c_t * min(1, c_t / c_{t-1}) from step 2 on (linear
 * convergence at the observed rate), as c_1 at step 1.  Once the estimate
 * is <= tol, checked on the device, the remaining steps do nothing.
 * At most `iterations` (1..16) steps; everything is enqueued on stream
 * without waiting.  sptrsv_refine_stats reports the steps taken.  Errors: as
 * sptrsv_solve_fp32; ARG (iterations out of range, tol < 0 or NaN). */
sptrsv_status sptrsv_solve_refined(sptrsv_plan plan, const double *b, double *x, int32_t iterations,
                                   double tol, void *stream);

/* Waits for stream, then reports the last refinement: *iterations = steps
 * applied, *correction = c_t of the last step applied (+inf after a single
 * step).  Errors: ARG, STATE (not uploaded, or FP64
 * plan), HIP. */
sptrsv_status sptrsv_refine_stats(sptrsv_plan plan, void *stream, int32_t *iterations,
                                  double *correction);

/* Waits for stream, then reads and clears the plan's device status word:
 * *device_status = 0 if every solve since the last check completed normally,
 * else SPTRSV_ERR_TIMEOUT.  Errors: ARG, STATE, HIP. */
sptrsv_status sptrsv_check(sptrsv_plan plan, void *stream, int32_t *device_status);

/* Launch shape of the solve: waves (one per workgroup, all co-resident) per
 * compute unit, at most 8 (the co-residency the kernels' registers and LDS
 * prove; every wave must be resident for the grid to drain) and capped by
 * what the device reports it can keep resident; 0 (the default) picks 1..8
 * from the plan's tiles per level.  Takes effect at the next solve.
 * Errors: ARG (negative, or above 8). */
sptrsv_status sptrsv_set_launch(sptrsv_plan plan, int32_t waves_per_cu);

/* Work queues of the device schedule.  2 (the default): rows that some
 * other row depends on (the chain) and rows nothing depends on (sinks) are
 * packed into separate tiles, the chain's tiles and segments forming one
 * queue and the sinks' tiles another, each in level order, served by
 * separate waves (see sptrsv_set_chain_share), so sinks never hold up the
 * dependency chain.  1: every row in one queue, in level order.  Repacks
 * the host image (the upload becomes stale); the schedule and the rewrite
 * are unchanged.  Errors: ARG (not 1 or 2), OVERFLOW, OOM. */
sptrsv_status sptrsv_set_queues(sptrsv_plan plan, int32_t queues);

/* Share of the solve grid's waves, in per mille, that serves the chain
 * queue (rows that some other row depends on, in level order); the others
 * serve the sink queue (rows nothing depends on: their time is bandwidth,
 * not the dependency chain).  0 (the default) gives each queue the share of
 * the waves its share of the work asks for (64-lane chunks of terms plus
 * rows packed), kept within [1/8, 7/8]; an explicit share is applied as
 * given, leaving each queue at least one wave.  A plan with one queue
 * ignores it.  Takes effect at the next solve.  Errors: ARG (outside
 * [0, 1000]). */
sptrsv_status sptrsv_set_chain_share(sptrsv_plan plan, int32_t per_mille);

/* The launch shape the next solve of an uploaded plan uses: waves of the
 * cooperative grid and, of them, waves serving the chain queue (equal to
 * waves for a plan with one queue).  Errors: ARG, STATE (not uploaded). */
sptrsv_status sptrsv_launch_shape(sptrsv_plan plan, int32_t *waves, int32_t *chain_waves);

/* Upper bound, in ticks of the 100 MHz GPU real-time clock, on a single
 * dependency wait (default 200,000,000 = 2 s).  A wait that reaches it
 * gives up, marks the plan's status word and lets the kernel drain.
 * For tests of the failure path.  Takes effect at the next solve.
 * Errors: ARG (plan NULL). */
sptrsv_status sptrsv_set_wait_limit(sptrsv_plan plan, uint64_t ticks);

/* Plan statistics (Sec. V reports levels and FLOPs before and after).
 * flops: 2 per stored off-diagonal x-term or b-term plus 1 per row.
 * bytes: compulsory traffic of one solve in the plan's value type (v = 8
 * bytes for FP64, 4 for FP32): 4 + v per stored entry (int32 column + value,
 * diagonals included) + 8 + 2v per row (row offset, row id, b_i, x_i);
 * gathers of x and b are counted as cache hits.  bytes_rw counts the entries
 * of L' the solve reads (nnz_streamed) and those the right-hand-side step
 * reads (nnz_rhs), plus 2v per row for the M pass (b' written and read) or
 * 8 + 2v per row for the stage solve, less 2 per term whose column a
 * compact plan stores in 16 bits (compact_terms). */
typedef struct {
    int32_t n;
    int32_t levels;      /* levels of L */
    int32_t stages;      /* stages chosen by the rewrite */
    int32_t levels_rw;   /* levels of L' (the executed schedule) */
    int64_t nnz;         /* nnz(L), diagonals included */
    int64_t nnz_rw;      /* nnz(L'), diagonals included */
    int64_t nnz_m;       /* nnz(M) */
    int64_t flops;       /* of the plain solve */
    int64_t flops_rw;    /* of the rewritten solve */
    int64_t bytes;       /* of the plain solve */
    int64_t bytes_rw;    /* of the rewritten solve */
    int64_t device_bytes;/* size of the device image + workspace */
    int64_t tiles;       /* work items of the device schedule: 64-lane wide
                            tiles, and segments (counted once each) */
    int32_t precision;   /* 64 or 32: value type of the device image */
    int64_t seg_tiles;   /* tiles inside segments (runs of narrow levels one
                            wave executes in order) */
    int32_t rhs_mode;    /* right-hand-side step in use: 0 none (no b-terms),
                            SPTRSV_RHS_MPASS or SPTRSV_RHS_STAGE */
    int64_t nnz_rhs;     /* entries it reads: nnz(M), or the entries of L_B
                            its solve reads */
    int32_t rhs_segments;/* stage solve: stages solved whole by one wave each
                            (no wait on another wave); the others run level
                            by level across the grid */
    int32_t reg_chunks;  /* 64-lane chunks of a wide tile the solve holds in
                            registers, its terms gathered before the wait
                            (4, or 8 when most tiles have more than 4) */
    int32_t segments;    /* segments of the schedule (seg_tiles is their
                            tiles) */
    int32_t ring_segments;/* of which every term comes from the wave's LDS
                            ring; when all do, the solve runs a lighter
                            segment loop that gathers only the constants */
    int64_t chain_items; /* work items holding rows that some other row
                            depends on (the chain queue); the other
                            tiles - chain_items hold only rows nothing
                            depends on (the sink queue) */
    int64_t nnz_streamed;/* entries of L' a solve reads: nnz_rw, less the
                            terms of the copies of a batched plan's rows
                            that read copy 0's (power-of-two k <= 64
                            right-hand sides share one copy of the terms) */
    int32_t m_stored;    /* 1 if the plan holds M's entries.  The rewrite
                            stores them only when the right-hand-side step
                            reads them (the M pass); a plan that solves the
                            stage system instead keeps only M's row counts,
                            and sptrsv_plan_export or a switch to the M pass
                            builds the entries then (as long as the rewrite
                            itself, same values) */
    int32_t compact_cols;/* 1 if the wide tiles store each term's column as
                            a 16-bit distance back from the tile's first
                            slot (2 bytes instead of 4 per term): chosen by
                            the packer when every distance fits and no
                            copies share terms.  The environment variable
                            SPTRSV_COMPACT_COLS=0, read at packing, keeps
                            32-bit columns.  Results are the same bit for
                            bit either way. */
    int64_t compact_terms;/* terms stored with 16-bit columns (0 unless
                            compact_cols) */
} sptrsv_info;
sptrsv_status sptrsv_plan_info(sptrsv_plan plan, sptrsv_info *out);

/* Level of every row (host int32[n]): which = 0 for L, 1 for L'. */
sptrsv_status sptrsv_plan_levels(sptrsv_plan plan, int32_t which, int32_t *level);

/* Stage of every level of L (host int32[levels]) and the entries each
 * absorbed level added (host int64[levels], 0 for levels that open a stage);
 * either pointer may be NULL. */
sptrsv_status sptrsv_plan_stages(sptrsv_plan plan, int32_t *stage_of_level,
                                 int64_t *delta_of_level);

/* The executed schedule: level sets of L' (host int32[levels_rw + 1] and
 * int32[n]; rows ascending within a level). */
sptrsv_status sptrsv_plan_schedule(sptrsv_plan plan, int32_t *level_ptr, int32_t *rows);

/* The rewritten system as CSR (host arrays sized by sptrsv_plan_info):
 * L' = (lp_ptr int64[n+1], lp_col int32[nnz_rw], lp_val double[nnz_rw]) with
 * ascending columns and the diagonal last, and M = (m_ptr int64[n+1],
 * m_col int32[nnz_m], m_val double[nnz_m]) with ascending columns.  With
 * m_ptr NULL only L' is written (M can be far larger).  A plan that does not
 * hold M's entries (sptrsv_info.m_stored 0) builds them first: host time and
 * memory of the order of the rewrite; the device image is unchanged.
 * Errors: ARG, OOM. */
sptrsv_status sptrsv_plan_export(sptrsv_plan plan, int64_t *lp_ptr, int32_t *lp_col,
                                 double *lp_val, int64_t *m_ptr, int32_t *m_col,
                                 double *m_val);

/* ---- Timing and the learned cost model ----------------------------------
 *
 * The paper picks the levels to rewrite by hand (Sec. IV, V).  The LEARNED
 * policy picks them with a small cost model trained on solve times that the
 * library itself measures: an instrumented solve stamps the GPU real-time
 * clock (100 MHz) as each unit of work completes, sptrsv_plan_stamp_levels
 * maps the stamps to executed levels, sptrsv_plan_level_features gives each
 * executed level's shape, and the model (a 6-64-64-1 perceptron in FP32,
 * tanh hidden layers) is trained with the kernels below.  Parameter vector,
 * SPTRSV_MLP_PARAMS floats: W1[64][6], b1[64], W2[64][64], b2[64], w3[64], b3;
 * the output is w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3. */
#define SPTRSV_MLP_INPUTS 6
#define SPTRSV_MLP_PARAMS 4673

/* As sptrsv_solve (FP64 plans) with an instrumented kernel that also writes
 * stamps (device, tiles + seg_tiles + 1 uint64, owned by the caller):
 * stamps[u] = clock when unit u completed (units: the tiles of the schedule,
 * then the segment tiles), stamps[tiles + seg_tiles] = clock when the grid
 * started.  Slower than sptrsv_solve by a store per unit.  Errors: as
 * sptrsv_solve; ARG (stamps NULL); STATE (FP32 plan). */
sptrsv_status sptrsv_solve_stamped(sptrsv_plan plan, const double *b, double *x, uint64_t *stamps,
                                   void *stream);

/* Executed level (of L') of the rows each stamp unit finishes (host int32,
 * tiles + seg_tiles entries); -1 for units that finish no level by
 * themselves (whole segments, padding tiles).  A level's completion time is
 * the latest stamp among its units. */
sptrsv_status sptrsv_plan_stamp_levels(sptrsv_plan plan, int32_t *level);

/* Shape of every executed level as the model's inputs (host float
 * [levels_rw][SPTRSV_MLP_INPUTS]): log2(1 + rows) / 16, log2(1 + entries) / 24,
 * entries added by rewriting per entry of L (capped at 16) / 4,
 * log2(1 + longest row) / 8, entries per row (capped at 256) / 16,
 * log2(original levels merged) / 8; entries of a row = x-terms + b-terms +
 * diagonal. */
sptrsv_status sptrsv_plan_level_features(sptrsv_plan plan, float *features);

/* y[s] = model(x[s]) for s < m (device arrays: params SPTRSV_MLP_PARAMS
 * floats, x [m][SPTRSV_MLP_INPUTS], y [m]); enqueued on stream.  Errors: ARG. */
sptrsv_status sptrsv_mlp_forward(const float *params, const float *x, float *y, int32_t m, void *stream);

/* Bytes of the device workspace sptrsv_mlp_grad needs for m samples. */
sptrsv_status sptrsv_mlp_grad_workspace(int32_t m, size_t *bytes);

/* Gradient of the mean squared error (1/m) sum_s (model(x[s]) - t[s])^2 with
 * respect to the parameters, by back-propagation (device: grad
 * SPTRSV_MLP_PARAMS floats, loss one float or NULL, workspace as sized by
 * sptrsv_mlp_grad_workspace); sums run in a fixed order, so the result is
 * deterministic.  Enqueued on stream.  Errors: ARG (m < 1, null, workspace
 * too small), HIP. */
sptrsv_status sptrsv_mlp_grad(const float *params, const float *x, const float *t, int32_t m,
                              float *grad, float *loss, void *workspace, size_t workspace_bytes,
                              void *stream);

/* As sptrsv_mlp_grad, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the workspace is a file-scope device array of the library,
 * sized for m <= SPTRSV_MLP_NOALLOC_MAX_SAMPLES (about 8.6 MB, held on every
 * GPU the library runs on until the process ends), so the call makes no
 * allocation.  Results equal sptrsv_mlp_grad's bit for bit (same kernels,
 * same summation order).  All calls on one GPU share the array: calls that
 * overlap on one GPU (on different streams or threads) race and must not be
 * issued.  The array's device address is looked up on the first call on
 * each device.  Errors: ARG (m < 1, m above the maximum, null), HIP. */
#define SPTRSV_MLP_NOALLOC_MAX_SAMPLES 8192
sptrsv_status sptrsv_mlp_grad_noalloc(const float *params, const float *x, const float *t, int32_t m,
                                      float *grad, float *loss, void *stream);

/* One Adam step (Kingma and Ba, 2015) on params with moment buffers m1, m2
 * (device, SPTRSV_MLP_PARAMS floats each, zero before step 1); step >= 1 is
 * the step number for the bias corrections.  Errors: ARG, HIP. */
sptrsv_status sptrsv_mlp_adam(float *params, const float *grad, float *m1, float *m2, int32_t step,
                              float lr, float beta1, float beta2, float eps, void *stream);

/* ---- Diagnostics ----------------------------------------------------------
 *
 * Latency of one dependency hop as the solve sees it (the other bound of a
 * level-scheduled solve, next to memory bandwidth: a solve of a schedule
 * with L levels takes at least L hops).  Two waves on two compute units take
 * `hops` turns (2 .. 2^24), each publishing a counter with a device-scope
 * store and polling for the other's with device-scope loads, like a row
 * published by one wave and gathered by another.  same_xcd != 0 puts the
 * partner on the same XCD (workgroups 0 and 8), else on the next one (0 and
 * 1), given the in-turn dispatch of workgroups to XCDs.  dev_scratch: device,
 * >= 32 bytes, 8-byte aligned, owned by the caller.  Waits for stream, then
 * writes the mean nanoseconds per hop.  Errors: ARG, HIP, TIMEOUT (a wait
 * passed 100 ms). */
sptrsv_status sptrsv_probe_hop(int32_t hops, int32_t same_xcd, void *dev_scratch, size_t bytes,
                               double *ns_per_hop, void *stream);

/* Releases the plan (host memory only; the caller frees its device buffer
 * after the last solve that uses it has finished).  NULL is ignored. */
void sptrsv_plan_destroy(sptrsv_plan plan);

/* Message of the last failed call on this thread ("" if none); valid until
 * the next call on this thread. */
const char *sptrsv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPTRSV_H */
