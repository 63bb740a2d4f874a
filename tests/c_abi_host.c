/* The C ABI from C (no GPU): analyse and rewrite a unit lower-bidiagonal
 * chain, read the plan back and check it against its closed form.  Compiled
 * as C11 with warnings as errors by tests/test_c_abi_host.py, which also runs
 * it.  Exit status 0 on success.
 *
 * Chain of n rows, x_i = b_i + x_{i-1} (L = I - subdiagonal).  Stages of 3
 * levels: in a stage starting at row a, row i > a keeps the x-term of row
 * a - 1 (if a > 0) with coefficient -1 and gets b-terms from rows a..i-1,
 * each with coefficient 1 (substituting x_j = b_j + x_{j-1}). */
#include <stdio.h>
#include <stdlib.h>
#include "sptrsv.h"

#define N 7

static int fail(const char *what) {
    printf("FAIL: %s (%s)\n", what, sptrsv_last_error());
    return 1;
}

int main(void) {
    int32_t rp[N + 1], ci[2 * N];
    double val[2 * N];
    int32_t q = 0;
    for (int32_t i = 0; i < N; ++i) {
        rp[i] = q;
        if (i > 0) { ci[q] = i - 1; val[q] = -1.0; ++q; }
        ci[q] = i; val[q] = 1.0; ++q;
    }
    rp[N] = q;

    sptrsv_plan plan = NULL, bad = (sptrsv_plan)1;
    if (sptrsv_analyse(-1, rp, ci, val, &bad) != SPTRSV_ERR_ARG || bad != NULL) return fail("n < 0 rejected");
    if (sptrsv_analyse(N, rp, ci, val, &plan) != SPTRSV_OK) return fail("analyse");

    sptrsv_policy pol;
    sptrsv_policy_default(&pol);
    pol.max_width = 1000;
    pol.max_depth = 3;
    pol.max_fill = 10.0;
    if (sptrsv_rewrite(plan, &pol) != SPTRSV_OK) return fail("rewrite");

    sptrsv_info info;
    if (sptrsv_plan_info(plan, &info) != SPTRSV_OK) return fail("info");
    /* 7 levels -> stages {0,1,2} {3,4,5} {6}: 3 executed levels; b-terms
     * 1 + 2 per full stage */
    if (info.n != N || info.levels != N || info.stages != 3 || info.levels_rw != 3 || info.nnz_m != 6)
        return fail("plan shape");

    int32_t lev[N];
    if (sptrsv_plan_levels(plan, 1, lev) != SPTRSV_OK) return fail("levels of L'");
    for (int32_t i = 0; i < N; ++i)
        if (lev[i] != i / 3) return fail("level of a rewritten row");

    int64_t lp_ptr[N + 1], m_ptr[N + 1];
    int32_t lp_col[2 * N], m_col[N];
    double lp_val[2 * N], m_val[N];
    if (sptrsv_plan_export(plan, lp_ptr, lp_col, lp_val, m_ptr, m_col, m_val) != SPTRSV_OK) return fail("export");
    for (int32_t i = 0; i < N; ++i) {
        const int32_t a = i - i % 3;                 /* first row of the stage */
        const int64_t nx = lp_ptr[i + 1] - lp_ptr[i] - 1;
        if (lp_col[lp_ptr[i + 1] - 1] != i || lp_val[lp_ptr[i + 1] - 1] != 1.0) return fail("diagonal kept last");
        /* every row of a stage (its first one unchanged) keeps one x-term,
         * on the last row of the previous stage */
        if (nx != (a > 0 ? 1 : 0)) return fail("x-terms of a row");
        if (nx == 1 && (lp_col[lp_ptr[i]] != a - 1 || lp_val[lp_ptr[i]] != -1.0)) return fail("x-term of a row");
        if (m_ptr[i + 1] - m_ptr[i] != i - a) return fail("b-terms of a row");
        for (int64_t p = m_ptr[i]; p < m_ptr[i + 1]; ++p)
            if (m_col[p] != a + (int32_t)(p - m_ptr[i]) || m_val[p] != 1.0) return fail("b-term");
    }
    sptrsv_plan_destroy(plan);
    sptrsv_plan_destroy(NULL);
    printf("ok\n");
    return 0;
}
