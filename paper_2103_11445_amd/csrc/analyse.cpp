// analyse.cpp -- matrix analysis (arXiv:2103.11445, Sec. IV): validate and
// copy L, build DAG_L's level of every row and the level sets (Sec. II).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>

#include "plan.hpp"

namespace sptrsv {

static void fail(sptrsv_status code, const std::string &msg) { throw Error{code, msg}; }

void validate_csr(int32_t n, const int32_t *rp, const int32_t *ci, const double *val) {
    if (n < 0) fail(SPTRSV_ERR_ARG, "n < 0");
    if (n == 0) return;
    if (!rp || !ci || !val) fail(SPTRSV_ERR_ARG, "null CSR array");
    if (rp[0] != 0) fail(SPTRSV_ERR_CSR, "row_ptr[0] != 0");
    for (int32_t i = 0; i < n; ++i) {
        const int32_t b = rp[i], e = rp[i + 1];
        if (e < b) fail(SPTRSV_ERR_CSR, "row_ptr decreases at row " + std::to_string(i));
        if (e == b) fail(SPTRSV_ERR_DIAG, "row " + std::to_string(i) + " is empty (no diagonal)");
        int32_t prev = -1;
        for (int32_t p = b; p < e; ++p) {
            const int32_t c = ci[p];
            if (c < 0 || c >= n) fail(SPTRSV_ERR_CSR, "column out of range in row " + std::to_string(i));
            if (c <= prev) fail(SPTRSV_ERR_CSR, "columns not strictly increasing in row " + std::to_string(i));
            if (c > i) fail(SPTRSV_ERR_CSR, "entry above the diagonal in row " + std::to_string(i));
            prev = c;
        }
        if (ci[e - 1] != i) fail(SPTRSV_ERR_DIAG, "row " + std::to_string(i) + " has no diagonal");
        if (val[e - 1] == 0.0) fail(SPTRSV_ERR_DIAG, "zero diagonal in row " + std::to_string(i));
    }
}

void level_sets(int32_t n, const int32_t *level, int32_t nlev, std::vector<int32_t> &ptr,
                std::vector<int32_t> &rows) {
    ptr.assign((size_t)nlev + 1, 0);
    rows.resize((size_t)n);
    for (int32_t i = 0; i < n; ++i) ++ptr[(size_t)level[i] + 1];
    for (int32_t l = 0; l < nlev; ++l) ptr[(size_t)l + 1] += ptr[(size_t)l];
    std::vector<int32_t> cur(ptr.begin(), ptr.end() - 1);
    for (int32_t i = 0; i < n; ++i) rows[(size_t)cur[(size_t)level[i]]++] = i;
}

void analyse(Plan &p, int32_t n, const int32_t *rp, const int32_t *ci, const double *val) {
    validate_csr(n, rp, ci, val);
    p.n = n;
    const size_t nnz = n ? (size_t)rp[n] : 0;
    p.rp.assign(rp, rp + (size_t)n + 1 - (n == 0));
    if (n == 0) p.rp.assign(1, 0);
    p.ci.assign(ci, ci + nnz);
    p.val.assign(val, val + nnz);
    // Level of a row: one more than the deepest row it depends on; rows
    // depend only on earlier rows, so one pass in row order suffices.
    p.level.resize((size_t)n);
    int32_t maxlev = -1;
    for (int32_t i = 0; i < n; ++i) {
        int32_t lv = 0;
        for (int32_t q = rp[i]; q < rp[i + 1] - 1; ++q) lv = std::max(lv, p.level[(size_t)ci[q]] + 1);
        p.level[(size_t)i] = lv;
        maxlev = std::max(maxlev, lv);
    }
    p.nlev = maxlev + 1;
    level_sets(n, p.level.data(), p.nlev, p.level_ptr, p.level_rows);
    p.sys_n.assign(1, n);
    p.sys_k.assign(1, 1);
    p.sys_base.assign(1, 0);
}

// Upper-triangular U (diagonal first in each row): validate, then hold it with
// the index order reversed, U'[n-1-i][n-1-j] = U[i][j], which is lower
// triangular with the diagonal last.  Backward substitution on U is forward
// substitution on U' with b and x reversed; the device image maps indices back.
void analyse_upper(Plan &p, int32_t n, const int32_t *rp, const int32_t *ci, const double *val) {
    if (n < 0) fail(SPTRSV_ERR_ARG, "n < 0");
    if (n > 0) {
        if (!rp || !ci || !val) fail(SPTRSV_ERR_ARG, "null CSR array");
        if (rp[0] != 0) fail(SPTRSV_ERR_CSR, "row_ptr[0] != 0");
        for (int32_t i = 0; i < n; ++i) {
            const int32_t b = rp[i], e = rp[i + 1];
            if (e < b) fail(SPTRSV_ERR_CSR, "row_ptr decreases at row " + std::to_string(i));
            if (e == b) fail(SPTRSV_ERR_DIAG, "row " + std::to_string(i) + " is empty (no diagonal)");
            int32_t prev = -1;
            for (int32_t q = b; q < e; ++q) {
                const int32_t c = ci[q];
                if (c < 0 || c >= n) fail(SPTRSV_ERR_CSR, "column out of range in row " + std::to_string(i));
                if (c <= prev) fail(SPTRSV_ERR_CSR, "columns not strictly increasing in row " + std::to_string(i));
                if (c < i) fail(SPTRSV_ERR_CSR, "entry below the diagonal in row " + std::to_string(i));
                prev = c;
            }
            if (ci[b] != i) fail(SPTRSV_ERR_DIAG, "row " + std::to_string(i) + " has no diagonal");
            if (val[b] == 0.0) fail(SPTRSV_ERR_DIAG, "zero diagonal in row " + std::to_string(i));
        }
    }
    const size_t nnz = n ? (size_t)rp[n] : 0;
    std::vector<int32_t> rrp((size_t)n + 1, 0), rci(nnz);
    std::vector<double> rval(nnz);
    size_t q = 0;
    for (int32_t r = 0; r < n; ++r) {
        const int32_t i = n - 1 - r;
        for (int32_t t = rp[i + 1] - 1; t >= rp[i]; --t) {
            rci[q] = n - 1 - ci[t];
            rval[q] = val[t];
            ++q;
        }
        rrp[(size_t)r + 1] = (int32_t)q;
    }
    analyse(p, n, rrp.data(), rci.data(), rval.data());
    p.upper = true;
}

// Many systems at once: matrix j (n_j rows) with k_j right-hand sides becomes
// k_j copies of its block on the diagonal of one lower-triangular union, so a
// single plan (and a single launch) solves all of them.  The copies are
// interleaved: copy c of row i of system j is union row base_j + i*k_j + c,
// which is also where its b and x entries sit in the concatenation of the
// callers' row-major n_j x k_j blocks.  The k_j copies of a row then share a
// level and sit side by side in the device schedule, so the gathers of one
// term for all right-hand sides touch one contiguous run of x.
void analyse_batch(Plan &p, int32_t count, const int32_t *n, const int32_t *const *rp,
                   const int32_t *const *ci, const double *const *val, const int32_t *k) {
    if (count < 0) fail(SPTRSV_ERR_ARG, "count < 0");
    if (count > 0 && (!n || !rp || !ci || !val || !k)) fail(SPTRSV_ERR_ARG, "null batch array");
    int64_t rows = 0, nnz = 0;
    for (int32_t j = 0; j < count; ++j) {
        if (k[j] < 1) fail(SPTRSV_ERR_ARG, "k < 1 for system " + std::to_string(j));
        try {
            validate_csr(n[j], rp[j], ci[j], val[j]);
        } catch (Error &e) {
            e.msg = "system " + std::to_string(j) + ": " + e.msg;
            throw;
        }
        rows += (int64_t)n[j] * k[j];
        nnz += (int64_t)(n[j] ? rp[j][n[j]] : 0) * k[j];
    }
    if (rows > (int64_t)INT32_MAX - kRing || nnz > (int64_t)INT32_MAX)
        fail(SPTRSV_ERR_OVERFLOW, "batch too large for int32 indexing");
    std::vector<int32_t> urp((size_t)rows + 1, 0), uci((size_t)nnz);
    std::vector<double> uval((size_t)nnz);
    int64_t r = 0, q = 0, base = 0;
    for (int32_t j = 0; j < count; ++j) {
        const int64_t kj = k[j];
        for (int32_t i = 0; i < n[j]; ++i) {
            for (int64_t c = 0; c < kj; ++c) {
                for (int32_t t = rp[j][i]; t < rp[j][i + 1]; ++t) {
                    uci[(size_t)q] = (int32_t)(base + (int64_t)ci[j][t] * kj + c);
                    uval[(size_t)q] = val[j][t];
                    ++q;
                }
                urp[(size_t)++r] = (int32_t)q;
            }
        }
        base += (int64_t)n[j] * kj;
    }
    analyse(p, (int32_t)rows, urp.data(), uci.data(), uval.data());
    p.batch_count = count;
    p.sys_n.assign(n, n + count);
    p.sys_k.assign(k, k + count);
    p.sys_base.resize((size_t)count);
    for (int32_t j = 0, b = 0; j < count; ++j) {
        p.sys_base[(size_t)j] = b;
        b += n[j] * k[j];
    }
}

}  // namespace sptrsv
