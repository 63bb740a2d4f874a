/*
 * oracle.c -- plain, slow, obviously correct CPU reference ("the oracle") for
 * level-scheduled sparse lower-triangular solve with equation rewriting
 * (Yilmaz, "Graph Transformation and Specialized Code Generation for Sparse
 * Triangular Solve (SpTRSV)", arXiv:2103.11445).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source
 * with the GPU library and must never be on the product path.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -fPIC -shared oracle.c -o liboracle.so
 * (-ffp-contract=off: every a*b+c below is a rounded product followed by a
 *  rounded sum, exactly as written; OpenMP only for the level-set solve).
 *
 * Input format (all functions): L is n x n lower triangular in CSR,
 *   row_ptr int32[n+1], col_idx int32[nnz], val double[nnz];
 * columns strictly increasing within a row, every row holds its diagonal.
 *
 * Readings of the paper that this file fixes (the paper is silent on them):
 *   R1  levels are numbered from 0 (a row with no off-diagonal is level 0);
 *   R2  a rewritten row substitutes the ORIGINAL equations of its
 *       dependencies, latest (highest-numbered) dependency first, and the
 *       repeated x[k] terms are merged into one coefficient (the grouping of
 *       equal x accesses and the rearrangement into Lx=b form of Sec. III,
 *       Fig. 3);
 *   R3  the substituted right-hand-side entries are kept as a sparse
 *       combination M (b'_i = b_i + sum_j M_ij b_j) applied at solve time,
 *       because b is an input of every solve;
 *   R4  the thin levels to rewrite are chosen by the threshold rule of
 *       oracle_select_stages (the paper picks them by hand);
 *   R5  structure is symbolic: an entry created by substitution is kept even
 *       if its value cancels to zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- solve -- */

/* Serial forward substitution (Sec. II, Algorithm 1 / Fig. 1 right): for
 * each row, accumulate the partial sum over its off-diagonal nonzeros (its
 * dependencies) in ascending column order, then divide by the diagonal. */
void oracle_solve(int n, const int *row_ptr, const int *col_idx,
                  const double *val, const double *b, double *x)
{
    for (int i = 0; i < n; ++i) {
        double s = 0.0, d = 0.0;
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int j = col_idx[p];
            if (j < i)
                s = s + val[p] * x[j];
            else
                d = val[p];
        }
        x[i] = (b[i] - s) / d;
    }
}

/* The type the extended-precision twin computes in: x87 extended precision
 * (64-bit significand) on x86-64. */
typedef long double ext_t;

/* The same substitution carried in ext_t; xl holds the extended values, x
 * the values rounded once to double at the end. */
void oracle_solve_ld(int n, const int *row_ptr, const int *col_idx,
                     const double *val, const double *b, double *x)
{
    ext_t *xl = (ext_t *)malloc(sizeof(ext_t) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        ext_t s = 0, d = 0;
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int j = col_idx[p];
            if (j < i)
                s = s + (ext_t)val[p] * xl[j];
            else
                d = (ext_t)val[p];
        }
        xl[i] = ((ext_t)b[i] - s) / d;
        x[i] = (double)xl[i];
    }
    free(xl);
}

/* Backward substitution for an upper-triangular U (diagonal first in each
 * row): for i = n-1 down to 0, x_i = (b_i - sum_{j>i} U_ij x_j) / U_ii, the
 * partial sum taken in ascending column order.  This is the triangular solve
 * that follows the forward one in LU / ILU preconditioners; the rewriting of
 * Sec. III applies to its dependency DAG unchanged (Sec. III notes the method
 * works on the dependency graph itself). */
void oracle_solve_upper(int n, const int *row_ptr, const int *col_idx,
                        const double *val, const double *b, double *x)
{
    for (int i = n - 1; i >= 0; --i) {
        double s = 0.0, d = 0.0;
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int j = col_idx[p];
            if (j > i)
                s = s + val[p] * x[j];
            else
                d = val[p];
        }
        x[i] = (b[i] - s) / d;
    }
}

/* --------------------------------------------------------------- levels -- */

/* Level of every row in DAG_L (Sec. II; level sets as in the level-set
 * methods the paper builds on): a row with no dependency is level 0,
 * otherwise its level is one more than the deepest level among the rows it
 * depends on.  Returns the number of levels. */
int oracle_levels(int n, const int *row_ptr, const int *col_idx, int *level)
{
    int nlev = 0;
    for (int i = 0; i < n; ++i) {
        int lv = 0;
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int j = col_idx[p];
            if (j < i && level[j] + 1 > lv)
                lv = level[j] + 1;
        }
        level[i] = lv;
        if (lv + 1 > nlev)
            nlev = lv + 1;
    }
    return nlev;
}

/* Level sets: the rows of each level, in ascending row order.
 * level_ptr int32[nlev+1], rows int32[n]. */
void oracle_level_sets(int n, const int *level, int nlev, int *level_ptr, int *rows)
{
    for (int l = 0; l <= nlev; ++l)
        level_ptr[l] = 0;
    for (int i = 0; i < n; ++i)
        level_ptr[level[i] + 1] += 1;
    for (int l = 0; l < nlev; ++l)
        level_ptr[l + 1] += level_ptr[l];
    int *fill = (int *)malloc(sizeof(int) * (size_t)(nlev > 0 ? nlev : 1));
    for (int l = 0; l < nlev; ++l)
        fill[l] = level_ptr[l];
    for (int i = 0; i < n; ++i)
        rows[fill[level[i]]++] = i;
    free(fill);
}

/* ------------------------------------------------- symbolic rewriting -- */

/* Structure of row i after rewriting it into a stage that starts at level a
 * (Sec. III, Fig. 2): every dependency with level >= a is replaced by its
 * own equation, repeatedly, until only dependencies below level a remain.
 * Equivalently (this is how it is computed here): walk from row i through
 * dependency edges, entering only rows of level >= a.  Every such row
 * reached (other than i) contributes one b-term (|M_i|); every row of level
 * < a adjacent to i or to a reached row is one remaining x-term (|L'_i|).
 * stamp/mark/stack are caller scratch of length n; *stampc is bumped. */
static void reach_count(int i, int a, const int *row_ptr, const int *col_idx,
                        const int *level, int *mark, int *stack, int *stampc,
                        int64_t *nx, int64_t *nb)
{
    int stamp = ++(*stampc);
    int top = 0;
    int64_t cx = 0, cb = 0;
    stack[top++] = i;
    mark[i] = stamp;
    while (top > 0) {
        int u = stack[--top];
        for (int p = row_ptr[u]; p < row_ptr[u + 1]; ++p) {
            int k = col_idx[p];
            if (k >= u || mark[k] == stamp)
                continue;
            mark[k] = stamp;
            if (level[k] >= a) {
                cb += 1;
                stack[top++] = k;
            } else {
                cx += 1;
            }
        }
    }
    *nx = cx;
    *nb = cb;
}

/* Stage selection (the thin-level choice of Sec. III / Sec. V; threshold
 * reading R4).  Levels are cut into consecutive stages; level l joins the
 * current stage (which keeps its first level a) when
 *   kind 1 (threshold): width(l) <= max_width, the stage holds fewer than
 *       max_depth levels, the entries added so far plus those added by
 *       absorbing l stay within floor(max_fill * nnz(L)), and the total
 *       stored entries stay within max_entries;
 *   kind 2 (explicit): absorb[l] != 0 (l < absorb_len) and the total stays
 *       within max_entries;
 *   kind 0: never.
 * Otherwise l opens a new stage.  Level 0 always opens stage 0.
 * Entries added by absorbing l = sum over its rows of
 *   |L'_i| + |M_i| - (off-diagonals of row i)  (rewritten against start a).
 * Outputs stage_of_level int32[nlev] and delta_of_level int64[nlev]
 * (entries added for absorbed levels, 0 for levels that open a stage).
 * Returns the number of stages. */
int oracle_select_stages(int n, const int *row_ptr, const int *col_idx,
                         const int *level, int nlev, int kind, int max_width,
                         int max_depth, double max_fill, int64_t max_entries,
                         const unsigned char *absorb, int absorb_len,
                         int *stage_of_level, int64_t *delta_of_level)
{
    if (nlev <= 0)
        return 0;
    int *level_ptr = (int *)malloc(sizeof(int) * (size_t)(nlev + 1));
    int *rows = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *mark = (int *)calloc((size_t)(n > 0 ? n : 1), sizeof(int));
    int *stack = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    oracle_level_sets(n, level, nlev, level_ptr, rows);

    int64_t nnz = row_ptr[n];
    int64_t budget;
    double lim = max_fill * (double)nnz;
    if (lim >= 9.0e18)
        budget = INT64_MAX;
    else
        budget = (int64_t)floor(lim);

    int stamp = 0, stage = 0, a = 0, depth = 1;
    int64_t added = 0, total = nnz;
    stage_of_level[0] = 0;
    delta_of_level[0] = 0;
    for (int l = 1; l < nlev; ++l) {
        int width = level_ptr[l + 1] - level_ptr[l];
        int candidate = 0;
        if (kind == 1)
            candidate = width <= max_width && depth < max_depth;
        else if (kind == 2)
            candidate = l < absorb_len && absorb[l] != 0;
        int take = 0;
        int64_t delta = 0;
        if (candidate) {
            for (int q = level_ptr[l]; q < level_ptr[l + 1]; ++q) {
                int i = rows[q];
                int64_t nx, nb;
                reach_count(i, a, row_ptr, col_idx, level, mark, stack, &stamp, &nx, &nb);
                delta += nx + nb - (row_ptr[i + 1] - row_ptr[i] - 1);
            }
            if (kind == 1)
                take = added + delta <= budget && total + delta <= max_entries;
            else
                take = total + delta <= max_entries;
        }
        if (take) {
            stage_of_level[l] = stage;
            delta_of_level[l] = delta;
            depth += 1;
            added += delta;
            total += delta;
        } else {
            stage += 1;
            stage_of_level[l] = stage;
            delta_of_level[l] = 0;
            a = l;
            depth = 1;
        }
    }
    free(level_ptr);
    free(rows);
    free(mark);
    free(stack);
    return stage + 1;
}

/* First level of the stage holding each level. */
static int *stage_start_levels(int nlev, const int *stage_of_level)
{
    int *start = (int *)malloc(sizeof(int) * (size_t)(nlev > 0 ? nlev : 1));
    for (int l = 0; l < nlev; ++l)
        start[l] = (l > 0 && stage_of_level[l] == stage_of_level[l - 1]) ? start[l - 1] : l;
    return start;
}

/* Sizes of the rewritten system: nnz of L' (with diagonals) and of M. */
void oracle_rewrite_count(int n, const int *row_ptr, const int *col_idx,
                          const int *level, int nlev, const int *stage_of_level,
                          int64_t *nnz_lp, int64_t *nnz_m)
{
    int *start = stage_start_levels(nlev, stage_of_level);
    int *mark = (int *)calloc((size_t)(n > 0 ? n : 1), sizeof(int));
    int *stack = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int stamp = 0;
    int64_t cl = 0, cm = 0;
    for (int i = 0; i < n; ++i) {
        int a = start[level[i]];
        if (level[i] == a) {
            cl += row_ptr[i + 1] - row_ptr[i];
        } else {
            int64_t nx, nb;
            reach_count(i, a, row_ptr, col_idx, level, mark, stack, &stamp, &nx, &nb);
            cl += nx + 1;
            cm += nb;
        }
    }
    *nnz_lp = cl;
    *nnz_m = cm;
    free(start);
    free(mark);
    free(stack);
}

/* -------------------------------------------------- numeric rewriting -- */

/* Rewrite every row of an absorbed level (Sec. III, Fig. 2 and Fig. 3,
 * readings R2, R3, R5).  For row i in a stage starting at level a the
 * equation is held as a sorted list of (column, coefficient) pairs.  Going
 * down from the highest column, each coefficient c_j on a row j of level
 * >= a is removed by substituting row j's original equation
 *     x_j = (b_j - sum_k L_jk x_k) / L_jj,
 * which adds -(c_j / L_jj) * L_jk to the coefficient of every x_k of row j
 * (a new coefficient starts from 0.0) and leaves the term (c_j / L_jj) b_j
 * on the right-hand side, i.e. M_ij = -(c_j / L_jj).  Rows of the first
 * level of their stage are copied unchanged.  The diagonal is never touched
 * (no substituted row contains x_i).
 * Outputs are CSR with ascending columns: L' (diagonal last) and M (no
 * diagonal; the implicit M_ii = 1).  Arrays are sized by
 * oracle_rewrite_count.  Returns 0, or -1 if scratch allocation failed. */
int oracle_rewrite(int n, const int *row_ptr, const int *col_idx, const double *val,
                   const int *level, int nlev, const int *stage_of_level,
                   int64_t *lp_ptr, int *lp_col, double *lp_val,
                   int64_t *m_ptr, int *m_col, double *m_val)
{
    int *start = stage_start_levels(nlev, stage_of_level);
    double *diag = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    size_t cap = 64;
    int *acol = (int *)malloc(sizeof(int) * cap);
    double *aval = (double *)malloc(sizeof(double) * cap);
    size_t mcap = 64;
    int *mc = (int *)malloc(sizeof(int) * mcap);
    double *mv = (double *)malloc(sizeof(double) * mcap);
    if (!start || !diag || !acol || !aval || !mc || !mv)
        return -1;
    for (int i = 0; i < n; ++i)
        diag[i] = val[row_ptr[i + 1] - 1];

    int64_t lq = 0, mq = 0;
    lp_ptr[0] = 0;
    m_ptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        int a = start[level[i]];
        size_t len = 0, mlen = 0;
        /* the row's own off-diagonals */
        for (int p = row_ptr[i]; p < row_ptr[i + 1] - 1; ++p) {
            if (len == cap) {
                cap *= 2;
                acol = (int *)realloc(acol, sizeof(int) * cap);
                aval = (double *)realloc(aval, sizeof(double) * cap);
            }
            acol[len] = col_idx[p];
            aval[len] = val[p];
            ++len;
        }
        if (level[i] != a) {
            /* below = number of list entries with a column smaller than the
             * column just examined; start above the top entry */
            size_t below = len;
            while (below > 0) {
                size_t p = below - 1;
                int j = acol[p];
                if (level[j] < a) {
                    below = p;
                    continue;
                }
                double c = aval[p] / diag[j];
                if (mlen == mcap) {
                    mcap *= 2;
                    mc = (int *)realloc(mc, sizeof(int) * mcap);
                    mv = (double *)realloc(mv, sizeof(double) * mcap);
                }
                mc[mlen] = j;
                mv[mlen] = -c;
                ++mlen;
                /* drop x_j */
                memmove(acol + p, acol + p + 1, sizeof(int) * (len - p - 1));
                memmove(aval + p, aval + p + 1, sizeof(double) * (len - p - 1));
                --len;
                below = p;
                /* add -c * (row j's off-diagonals); all their columns are < j */
                for (int r = row_ptr[j]; r < row_ptr[j + 1] - 1; ++r) {
                    int k = col_idx[r];
                    double t = c * val[r];
                    /* binary search for k among the first `below` entries */
                    size_t lo = 0, hi = below;
                    while (lo < hi) {
                        size_t mid = (lo + hi) / 2;
                        if (acol[mid] < k)
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    if (lo < below && acol[lo] == k) {
                        aval[lo] = aval[lo] - t;
                    } else {
                        if (len == cap) {
                            cap *= 2;
                            acol = (int *)realloc(acol, sizeof(int) * cap);
                            aval = (double *)realloc(aval, sizeof(double) * cap);
                        }
                        memmove(acol + lo + 1, acol + lo, sizeof(int) * (len - lo));
                        memmove(aval + lo + 1, aval + lo, sizeof(double) * (len - lo));
                        acol[lo] = k;
                        aval[lo] = 0.0 - t;
                        ++len;
                        ++below;
                    }
                }
            }
        }
        for (size_t p = 0; p < len; ++p) {
            lp_col[lq] = acol[p];
            lp_val[lq] = aval[p];
            ++lq;
        }
        lp_col[lq] = i;
        lp_val[lq] = diag[i];
        ++lq;
        lp_ptr[i + 1] = lq;
        /* M entries were recorded in descending column order */
        for (size_t p = mlen; p > 0; --p) {
            m_col[mq] = mc[p - 1];
            m_val[mq] = mv[p - 1];
            ++mq;
        }
        m_ptr[i + 1] = mq;
    }
    free(start);
    free(diag);
    free(acol);
    free(aval);
    free(mc);
    free(mv);
    return 0;
}

/* Solve the rewritten system L' x = b + M b (Sec. III, Fig. 3: the
 * rearranged equations are again in Lx=b form with updated b entries),
 * serially in row order, in the same operation order as oracle_solve. */
void oracle_solve_rewritten(int n, const int64_t *lp_ptr, const int *lp_col,
                            const double *lp_val, const int64_t *m_ptr,
                            const int *m_col, const double *m_val,
                            const double *b, double *x)
{
    for (int i = 0; i < n; ++i) {
        double bi = b[i];
        for (int64_t p = m_ptr[i]; p < m_ptr[i + 1]; ++p)
            bi = bi + m_val[p] * b[m_col[p]];
        double s = 0.0, d = 0.0;
        for (int64_t p = lp_ptr[i]; p < lp_ptr[i + 1]; ++p) {
            int k = lp_col[p];
            if (k < i)
                s = s + lp_val[p] * x[k];
            else
                d = lp_val[p];
        }
        x[i] = (bi - s) / d;
    }
}

/* Level-set execution on the host (Sec. II: the rows of one level do not
 * depend on each other, so they run in parallel, and a barrier separates
 * consecutive levels), with OpenMP on `threads` cores: the CPU comparator
 * of the GPU solve.  It runs a rewritten system L' x = b + M b (Sec. III,
 * Fig. 3) over the level sets of L' (level_ptr int32[nlev+1], rows
 * int32[n]); a plain system is L' = L with an empty M.  Every row is
 * computed exactly as in oracle_solve_rewritten, so the result is
 * bit-identical to it whatever the thread count. */
void oracle_solve_levelset(int n, const int *level_ptr, const int *rows, int nlev,
                           const int64_t *lp_ptr, const int *lp_col, const double *lp_val,
                           const int64_t *m_ptr, const int *m_col, const double *m_val,
                           const double *b, double *x, int threads)
{
    (void)n;
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
    for (int l = 0; l < nlev; ++l) {
        /* the implicit barrier at the end of the loop is the level barrier */
#pragma omp for schedule(static)
        for (int q = level_ptr[l]; q < level_ptr[l + 1]; ++q) {
            int i = rows[q];
            double bi = b[i];
            for (int64_t p = m_ptr[i]; p < m_ptr[i + 1]; ++p)
                bi = bi + m_val[p] * b[m_col[p]];
            double s = 0.0, d = 0.0;
            for (int64_t p = lp_ptr[i]; p < lp_ptr[i + 1]; ++p) {
                int k = lp_col[p];
                if (k < i)
                    s = s + lp_val[p] * x[k];
                else
                    d = lp_val[p];
            }
            x[i] = (bi - s) / d;
        }
    }
}
