// rewrite.cpp -- equation rewriting of thin levels (arXiv:2103.11445,
// Sec. III): stage selection, symbolic and numeric rewriting of the rows of
// absorbed levels, re-levelling of the rewritten system.
//
// A stage is a run of consecutive levels [a, e).  Rows of level a keep their
// equation.  A row i of a later level of the stage has every dependency of
// level >= a replaced by that row's original equation, latest dependency
// first, with equal x terms merged into one coefficient (Fig. 2 and the
// rearrangement of Fig. 3).  Symbolically, with S_j / X_j the b-terms and
// x-terms of an already rewritten in-stage row j:
//     S_i = U_{j in dep(i), lev j >= a} ({j} u S_j)
//     X_i = {k in dep(i) : lev k < a} u U_{j in dep(i), lev j >= a} X_j
// (X_j = dep(j) for rows of level a).  Numerically, with a sparse
// accumulator over X_i u S_i, for j in S_i in descending order:
//     c = acc[j] / L_jj,  M_ij = -c,  acc[k] -= c * L_jk  for k in dep(j),
// so that L'_i x = b_i + sum_j M_ij b_j.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <memory>
#include <thread>

#include <hip/hip_runtime_api.h>

#include "features.hpp"
#include "plan.hpp"

namespace sptrsv {

static void fail(sptrsv_status code, const std::string &msg) { throw Error{code, msg}; }

void validate_policy(const sptrsv_policy &pol) {
    switch (pol.kind) {
    case SPTRSV_POLICY_NONE:
        return;
    case SPTRSV_POLICY_THRESHOLD:
        if (pol.max_width < 0) fail(SPTRSV_ERR_ARG, "policy.max_width < 0");
        if (pol.max_depth < 1) fail(SPTRSV_ERR_ARG, "policy.max_depth < 1");
        if (!(pol.max_fill >= 0.0)) fail(SPTRSV_ERR_ARG, "policy.max_fill must be >= 0");
        if (pol.max_entries < 0) fail(SPTRSV_ERR_ARG, "policy.max_entries < 0");
        return;
    case SPTRSV_POLICY_EXPLICIT:
        if (pol.absorb_len < 0) fail(SPTRSV_ERR_ARG, "policy.absorb_len < 0");
        if (pol.absorb_len > 0 && !pol.absorb) fail(SPTRSV_ERR_ARG, "policy.absorb is NULL");
        if (pol.max_entries < 0) fail(SPTRSV_ERR_ARG, "policy.max_entries < 0");
        return;
    case SPTRSV_POLICY_LEARNED:
        if (!pol.model) fail(SPTRSV_ERR_ARG, "policy.model is NULL");
        if (pol.max_depth < 1) fail(SPTRSV_ERR_ARG, "policy.max_depth < 1");
        if (!(pol.max_fill >= 0.0)) fail(SPTRSV_ERR_ARG, "policy.max_fill must be >= 0");
        if (pol.max_entries < 0) fail(SPTRSV_ERR_ARG, "policy.max_entries < 0");
        return;
    default:
        fail(SPTRSV_ERR_ARG, "unknown policy kind " + std::to_string(pol.kind));
    }
}

namespace {

// Symbolic structure of the rewritten rows.  A row of a stage whose local
// index space is small holds its x-terms and b-terms as one bit set over
// that space (dense); any other rewritten row holds them as sorted lists in
// one arena (sparse).
struct Symbolic {
    std::vector<int64_t> off;    // per row: arena offset, -1 if not sparse
    std::vector<int32_t> nx, nb; // per row: counts (every rewritten row)
    std::vector<int32_t> arena;  // x-terms then b-terms of each sparse row
    // dense rows: a bit set over the ranks (ascending row id) of the stage's
    // local index space; the stage's table maps a rank to its row and marks
    // the ranks that are rows of the stage (b-terms)
    std::vector<int64_t> doff;     // per row: word offset into bits, -1 if not dense
    std::vector<int32_t> dstage;   // per row: its stage table
    std::vector<uint64_t> bits;
    std::vector<int32_t> st_words;               // per table: words of a row's set
    std::vector<int64_t> st_roff, st_woff;       // per table: offsets into st_rows, st_isb
    std::vector<int32_t> st_rows;                // rank -> row
    std::vector<uint64_t> st_isb;                // rank is a row of the stage
};

// Scratch of one worker: a stamp array over columns for de-duplication.
struct Marker {
    std::vector<uint32_t> stamp;
    uint32_t cur = 0;
    explicit Marker(int32_t n) : stamp((size_t)n, 0u) {}
    void next() {
        if (++cur == 0) {
            std::fill(stamp.begin(), stamp.end(), 0u);
            cur = 1;
        }
    }
    bool add(int32_t k) {
        if (stamp[(size_t)k] == cur) return false;
        stamp[(size_t)k] = cur;
        return true;
    }
};

// Structure of row i rewritten against a stage starting at level a, from
// the structures of its in-stage dependencies.
void row_structure(const Plan &p, const Symbolic &sym, int32_t i, int32_t a, Marker &mk,
                   std::vector<int32_t> &xs, std::vector<int32_t> &bs) {
    xs.clear();
    bs.clear();
    mk.next();
    for (int32_t q = p.rp[(size_t)i]; q < p.rp[(size_t)i + 1] - 1; ++q) {
        const int32_t j = p.ci[(size_t)q];
        const int32_t lj = p.level[(size_t)j];
        if (lj < a) {
            if (mk.add(j)) xs.push_back(j);
            continue;
        }
        if (mk.add(j)) bs.push_back(j);
        if (lj == a) {
            for (int32_t r = p.rp[(size_t)j]; r < p.rp[(size_t)j + 1] - 1; ++r) {
                const int32_t k = p.ci[(size_t)r];
                if (mk.add(k)) xs.push_back(k);
            }
        } else {
            const int32_t *s = sym.arena.data() + sym.off[(size_t)j];
            for (int32_t t = 0; t < sym.nx[(size_t)j]; ++t)
                if (mk.add(s[t])) xs.push_back(s[t]);
            s += sym.nx[(size_t)j];
            for (int32_t t = 0; t < sym.nb[(size_t)j]; ++t)
                if (mk.add(s[t])) bs.push_back(s[t]);
        }
    }
    std::sort(xs.begin(), xs.end());
    std::sort(bs.begin(), bs.end());
}

// Predicted cost (the model's output is the log of a time) of groups of
// rows, evaluated by the model's forward kernel on the current device.
class CostModel {
  public:
    explicit CostModel(const float *params) : params_(params) {
        hipError_t e = hipMalloc(&dx_, sizeof(float) * 2 * kFeatures);
        if (e == hipSuccess) e = hipMalloc(&dy_, sizeof(float) * 2);
        if (e != hipSuccess) {
            release();
            fail(SPTRSV_ERR_HIP, std::string("cost model buffers: ") + hipGetErrorString(e));
        }
    }
    ~CostModel() { release(); }
    CostModel(const CostModel &) = delete;
    CostModel &operator=(const CostModel &) = delete;

    // costs of one or two groups
    void eval(const GroupShape *g, int count, double *cost) {
        float x[2 * kFeatures], y[2];
        for (int r = 0; r < count; ++r) group_features(g[r], x + r * kFeatures);
        hipError_t e = hipMemcpy(dx_, x, sizeof(float) * kFeatures * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = (hipError_t)sptrsv_launch_mlp_forward(params_, dx_, dy_, count, nullptr);
        if (e == hipSuccess) e = hipMemcpy(y, dy_, sizeof(float) * count, hipMemcpyDeviceToHost);
        if (e != hipSuccess) fail(SPTRSV_ERR_HIP, std::string("cost model: ") + hipGetErrorString(e));
        for (int r = 0; r < count; ++r) cost[r] = std::exp((double)y[r]);
    }

  private:
    void release() {
        if (dx_) hipFree(dx_);
        if (dy_) hipFree(dy_);
        dx_ = dy_ = nullptr;
    }
    const float *params_;
    float *dx_ = nullptr, *dy_ = nullptr;
};

// Shape of level l left as it is (a stage of its own).
GroupShape plain_level(const Plan &p, int32_t l) {
    GroupShape g;
    for (int32_t q = p.level_ptr[(size_t)l]; q < p.level_ptr[(size_t)l + 1]; ++q) {
        const int32_t i = p.level_rows[(size_t)q];
        const int64_t len = p.rp[(size_t)i + 1] - p.rp[(size_t)i];
        ++g.rows;
        g.terms += len;
        g.orig += len;
        g.maxlen = std::max(g.maxlen, len);
    }
    return g;
}

// Largest local index space (bits of a row's set) of a stage rewritten
// with bit sets; a stage whose space grows beyond it continues with sorted
// lists.  A chain of narrow levels (the banded matrices) stays far below it,
// and there every row's sets cover most of the space, so a union of bit sets
// replaces a merge of long lists.  SPTRSV_DENSE_STAGE_BITS overrides the
// limit (0: every stage with lists); both representations give the same plan.
int64_t dense_stage_bits() {
    const char *s = std::getenv("SPTRSV_DENSE_STAGE_BITS");
    if (s && *s) {
        char *end = nullptr;
        const long long v = std::strtoll(s, &end, 10);
        if (end && *end == '\0' && v >= 0) return (int64_t)v;
    }
    return int64_t(1) << 14;
}

inline int popcount64(uint64_t v) { return __builtin_popcountll(v); }

// The open stage while it is rewritten with bit sets: its local index space
// (the stage's rows and the earlier rows they depend on, numbered in order of
// first appearance) and the sets of the rows rewritten so far, over the
// space as it was when each row was added.
struct StageSpace {
    enum { kUnset = 0, kDense = 1, kSparse = 2 };
    std::vector<int32_t> loc;     // per row of L: local index, -1 outside the space
    std::vector<int32_t> glob;    // local index -> row
    std::vector<uint64_t> isb;    // local index is a row of the stage
    std::vector<int64_t> uoff;    // per local index of a rewritten row: word offset into bits
    std::vector<int32_t> uwords;  // and its word count
    std::vector<int32_t> rows;    // rewritten rows, in the order taken
    std::vector<uint64_t> bits;
    int mode = kUnset;
    explicit StageSpace(int32_t n) : loc((size_t)n, -1) {}
    int32_t size() const { return (int32_t)glob.size(); }
    int32_t add(int32_t r, bool stage_row) {
        int32_t u = loc[(size_t)r];
        if (u >= 0) return u;
        u = (int32_t)glob.size();
        loc[(size_t)r] = u;
        glob.push_back(r);
        if ((size_t)(u >> 6) >= isb.size()) isb.push_back(0);
        if (stage_row) isb[(size_t)(u >> 6)] |= uint64_t(1) << (u & 63);
        return u;
    }
    void reset(int new_mode) {
        for (int32_t g : glob) loc[(size_t)g] = -1;
        glob.clear();
        isb.clear();
        uoff.clear();
        uwords.clear();
        rows.clear();
        bits.clear();
        mode = new_mode;
    }
};

// Opens the space of a stage whose first level is a: its rows and their
// dependencies.  Bit sets only while the space fits the limit.
void open_stage(StageSpace &sp, const Plan &p, int32_t a, int64_t cap) {
    sp.reset(StageSpace::kDense);
    const int32_t b0 = p.level_ptr[(size_t)a], b1 = p.level_ptr[(size_t)a + 1];
    if ((int64_t)(b1 - b0) > cap) {
        sp.mode = StageSpace::kSparse;
        return;
    }
    for (int32_t q = b0; q < b1; ++q) sp.add(p.level_rows[(size_t)q], true);
    for (int32_t q = b0; q < b1 && (int64_t)sp.size() <= cap; ++q) {
        const int32_t j = p.level_rows[(size_t)q];
        for (int32_t r = p.rp[(size_t)j]; r < p.rp[(size_t)j + 1] - 1; ++r) sp.add(p.ci[(size_t)r], false);
    }
    if ((int64_t)sp.size() > cap) sp.reset(StageSpace::kSparse);
}

// Sets of the stage's rewritten rows as sorted lists (the space outgrew the
// limit); the stage continues with lists.
void stage_to_lists(StageSpace &sp, Symbolic &sym) {
    std::vector<int32_t> xs, bs;
    for (int32_t i : sp.rows) {
        const int32_t u = sp.loc[(size_t)i];
        const uint64_t *B = sp.bits.data() + sp.uoff[(size_t)u];
        xs.clear();
        bs.clear();
        for (int32_t w = 0; w < sp.uwords[(size_t)u]; ++w)
            for (uint64_t m = B[w]; m; m &= m - 1) {
                const int32_t v = w * 64 + __builtin_ctzll(m);
                const bool stage_row = (sp.isb[(size_t)(v >> 6)] >> (v & 63)) & 1;
                (stage_row ? bs : xs).push_back(sp.glob[(size_t)v]);
            }
        std::sort(xs.begin(), xs.end());
        std::sort(bs.begin(), bs.end());
        sym.off[(size_t)i] = (int64_t)sym.arena.size();
        sym.arena.insert(sym.arena.end(), xs.begin(), xs.end());
        sym.arena.insert(sym.arena.end(), bs.begin(), bs.end());
    }
    sp.reset(StageSpace::kSparse);
}

// Closes a stage rewritten with bit sets: its space is renumbered by
// ascending row id (ranks) into a table, and every set is rewritten over the
// ranks, so that the numeric pass reads the terms in column order.
void close_stage(StageSpace &sp, Symbolic &sym, int threads) {
    if (sp.mode == StageSpace::kDense && !sp.rows.empty()) {
        const int32_t U = sp.size(), W = (U + 63) / 64;
        std::vector<int32_t> order((size_t)U), rank((size_t)U);
        for (int32_t u = 0; u < U; ++u) order[(size_t)u] = u;
        std::sort(order.begin(), order.end(),
                  [&](int32_t x, int32_t y) { return sp.glob[(size_t)x] < sp.glob[(size_t)y]; });
        const int32_t table = (int32_t)sym.st_words.size();
        sym.st_words.push_back(W);
        sym.st_roff.push_back((int64_t)sym.st_rows.size());
        sym.st_woff.push_back((int64_t)sym.st_isb.size());
        const size_t isb0 = sym.st_isb.size();
        sym.st_isb.resize(isb0 + (size_t)W, 0);
        for (int32_t r = 0; r < U; ++r) {
            const int32_t u = order[(size_t)r];
            rank[(size_t)u] = r;
            sym.st_rows.push_back(sp.glob[(size_t)u]);
            if ((sp.isb[(size_t)(u >> 6)] >> (u & 63)) & 1) sym.st_isb[isb0 + (size_t)(r >> 6)] |= uint64_t(1) << (r & 63);
        }
        const size_t base = sym.bits.size();
        sym.bits.resize(base + sp.rows.size() * (size_t)W, 0);
        parallel_ranges((int64_t)sp.rows.size(), threads, [&](int64_t lo, int64_t hi, int) {
            for (int64_t k = lo; k < hi; ++k) {
                const int32_t i = sp.rows[(size_t)k];
                const int32_t u = sp.loc[(size_t)i];
                const uint64_t *src = sp.bits.data() + sp.uoff[(size_t)u];
                uint64_t *dst = sym.bits.data() + base + (size_t)k * W;
                for (int32_t w = 0; w < sp.uwords[(size_t)u]; ++w)
                    for (uint64_t m = src[w]; m; m &= m - 1) {
                        const int32_t r = rank[(size_t)(w * 64 + __builtin_ctzll(m))];
                        dst[r >> 6] |= uint64_t(1) << (r & 63);
                    }
                sym.doff[(size_t)i] = (int64_t)(base + (size_t)k * W);
                sym.dstage[(size_t)i] = table;
            }
        });
    }
    sp.reset(StageSpace::kUnset);
}

}  // namespace

// Stage selection, level by level (Sec. III, and the rule of the policy):
// fills stage_of_level, delta_of_level and nstages, and the structure of
// every rewritten row.
static void select_stages(Plan &p, const sptrsv_policy &pol, Symbolic &sym) {
    const int32_t n = p.n, nlev = p.nlev;
    const int64_t nnz = n ? (int64_t)p.rp[(size_t)n] : 0;
    p.stage_of_level.assign((size_t)nlev, 0);
    p.delta_of_level.assign((size_t)nlev, 0);
    sym.off.assign((size_t)n, -1);
    sym.nx.assign((size_t)n, 0);
    sym.nb.assign((size_t)n, 0);
    sym.doff.assign((size_t)n, -1);
    sym.dstage.assign((size_t)n, -1);

    const int threads = hw_threads();
    std::vector<Marker> markers;
    markers.reserve((size_t)threads);
    for (int w = 0; w < threads; ++w) markers.emplace_back(n);
    StageSpace sp(n);
    const int64_t cap = dense_stage_bits();

    int64_t budget = std::numeric_limits<int64_t>::max();
    if (pol.kind == SPTRSV_POLICY_THRESHOLD || pol.kind == SPTRSV_POLICY_LEARNED) {
        const double lim = pol.max_fill * (double)nnz;
        if (lim < 9.0e18) budget = (int64_t)std::floor(lim);
    }
    int32_t stage = 0, a = 0, depth = 1;
    int64_t added = 0, total = nnz;
    std::vector<std::vector<int32_t>> lvl_x, lvl_b;  // per row of the candidate level (lists)
    std::vector<uint64_t> lvl_bits;                  // per row of the candidate level (bit sets)
    std::vector<int32_t> lvl_nx, lvl_nb;
    // LEARNED: shape and predicted cost of the current stage; a level joins
    // it when the predicted cost of the merged stage grows by less than the
    // cost of the level on its own
    const bool learned = pol.kind == SPTRSV_POLICY_LEARNED;
    std::unique_ptr<CostModel> model;
    GroupShape cur;
    double cur_cost = 0.0;
    if (learned && nlev > 0) {
        model.reset(new CostModel(pol.model));
        cur = plain_level(p, 0);
        model->eval(&cur, 1, &cur_cost);
    }
    for (int32_t l = 1; l < nlev; ++l) {
        const int32_t b0 = p.level_ptr[(size_t)l], b1 = p.level_ptr[(size_t)l + 1];
        const int32_t width = b1 - b0;
        bool candidate = false;
        if (pol.kind == SPTRSV_POLICY_THRESHOLD)
            candidate = width <= pol.max_width && depth < pol.max_depth;
        else if (pol.kind == SPTRSV_POLICY_EXPLICIT)
            candidate = l < pol.absorb_len && pol.absorb[l] != 0;
        else if (learned)
            candidate = depth < pol.max_depth;
        bool take = false;
        int64_t delta = 0, longest = 0;
        int32_t words = 0;
        if (candidate) {
            if (sp.mode == StageSpace::kUnset) open_stage(sp, p, a, cap);
            if (sp.mode == StageSpace::kDense) {
                // the level's dependencies before the stage join the space
                for (int32_t q = b0; q < b1 && (int64_t)sp.size() <= cap; ++q) {
                    const int32_t i = p.level_rows[(size_t)q];
                    for (int32_t r = p.rp[(size_t)i]; r < p.rp[(size_t)i + 1] - 1; ++r)
                        if (p.level[(size_t)p.ci[(size_t)r]] < a) sp.add(p.ci[(size_t)r], false);
                }
                if ((int64_t)sp.size() > cap) stage_to_lists(sp, sym);
            }
            std::vector<int64_t> part((size_t)threads, 0), part_max((size_t)threads, 0);
            if (sp.mode == StageSpace::kDense) {
                words = (sp.size() + 63) / 64;
                lvl_bits.assign((size_t)width * (size_t)words, 0);
                lvl_nx.resize((size_t)width);
                lvl_nb.resize((size_t)width);
                parallel_ranges(width, threads, [&](int64_t lo, int64_t hi, int w) {
                    int64_t d = 0, mx = 0;
                    for (int64_t q = lo; q < hi; ++q) {
                        const int32_t i = p.level_rows[(size_t)(b0 + q)];
                        uint64_t *B = lvl_bits.data() + (size_t)q * words;
                        for (int32_t r = p.rp[(size_t)i]; r < p.rp[(size_t)i + 1] - 1; ++r) {
                            const int32_t j = p.ci[(size_t)r];
                            const int32_t u = sp.loc[(size_t)j];
                            B[u >> 6] |= uint64_t(1) << (u & 63);
                            const int32_t lj = p.level[(size_t)j];
                            if (lj == a) {
                                for (int32_t s = p.rp[(size_t)j]; s < p.rp[(size_t)j + 1] - 1; ++s) {
                                    const int32_t v = sp.loc[(size_t)p.ci[(size_t)s]];
                                    B[v >> 6] |= uint64_t(1) << (v & 63);
                                }
                            } else if (lj > a) {
                                const uint64_t *S = sp.bits.data() + sp.uoff[(size_t)u];
                                for (int32_t t = 0; t < sp.uwords[(size_t)u]; ++t) B[t] |= S[t];
                            }
                        }
                        int32_t cnt = 0, nbq = 0;
                        for (int32_t t = 0; t < words; ++t) {
                            cnt += popcount64(B[t]);
                            nbq += popcount64(B[t] & sp.isb[(size_t)t]);
                        }
                        lvl_nx[(size_t)q] = cnt - nbq;
                        lvl_nb[(size_t)q] = nbq;
                        d += cnt - (p.rp[(size_t)i + 1] - p.rp[(size_t)i] - 1);
                        mx = std::max(mx, (int64_t)cnt + 1);
                    }
                    part[(size_t)w] = d;
                    part_max[(size_t)w] = mx;
                });
            } else {
                lvl_x.resize((size_t)width);
                lvl_b.resize((size_t)width);
                parallel_ranges(width, threads, [&](int64_t lo, int64_t hi, int w) {
                    int64_t d = 0, mx = 0;
                    for (int64_t q = lo; q < hi; ++q) {
                        const int32_t i = p.level_rows[(size_t)(b0 + q)];
                        row_structure(p, sym, i, a, markers[(size_t)w], lvl_x[(size_t)q], lvl_b[(size_t)q]);
                        const int64_t len = (int64_t)lvl_x[(size_t)q].size() + (int64_t)lvl_b[(size_t)q].size();
                        d += len - (p.rp[(size_t)i + 1] - p.rp[(size_t)i] - 1);
                        mx = std::max(mx, len + 1);
                    }
                    part[(size_t)w] = d;
                    part_max[(size_t)w] = mx;
                });
            }
            for (int64_t d : part) delta += d;
            for (int64_t m : part_max) longest = std::max(longest, m);
            if (pol.kind == SPTRSV_POLICY_THRESHOLD || learned)
                take = added + delta <= budget && total + delta <= pol.max_entries;
            else
                take = total + delta <= pol.max_entries;
        }
        GroupShape alone;
        double alone_cost = 0.0;
        if (learned) {
            alone = plain_level(p, l);
            if (take) {
                GroupShape both[2] = {cur, alone};
                both[0].rows += alone.rows;
                both[0].terms += alone.orig + delta;
                both[0].orig += alone.orig;
                both[0].maxlen = std::max(cur.maxlen, longest);
                both[0].span = depth + 1;
                double c[2];
                model->eval(both, 2, c);
                alone_cost = c[1];
                take = c[0] - cur_cost < alone_cost;
                if (take) {
                    cur = both[0];
                    cur_cost = c[0];
                }
            } else {
                model->eval(&alone, 1, &alone_cost);
            }
            if (!take) {
                cur = alone;
                cur_cost = alone_cost;
            }
        }
        if (take) {
            p.stage_of_level[(size_t)l] = stage;
            p.delta_of_level[(size_t)l] = delta;
            ++depth;
            added += delta;
            total += delta;
            if (sp.mode == StageSpace::kDense) {
                for (int32_t q = 0; q < width; ++q) {
                    const int32_t i = p.level_rows[(size_t)(b0 + q)];
                    const int32_t u = sp.add(i, true);
                    if (sp.uoff.size() <= (size_t)u) {
                        sp.uoff.resize((size_t)u + 1, -1);
                        sp.uwords.resize((size_t)u + 1, 0);
                    }
                    sp.uoff[(size_t)u] = (int64_t)sp.bits.size();
                    sp.uwords[(size_t)u] = words;
                    sp.bits.insert(sp.bits.end(), lvl_bits.begin() + (size_t)q * words,
                                   lvl_bits.begin() + (size_t)(q + 1) * words);
                    sp.rows.push_back(i);
                    sym.nx[(size_t)i] = lvl_nx[(size_t)q];
                    sym.nb[(size_t)i] = lvl_nb[(size_t)q];
                }
            } else {
                for (int32_t q = 0; q < width; ++q) {
                    const int32_t i = p.level_rows[(size_t)(b0 + q)];
                    sym.off[(size_t)i] = (int64_t)sym.arena.size();
                    sym.nx[(size_t)i] = (int32_t)lvl_x[(size_t)q].size();
                    sym.nb[(size_t)i] = (int32_t)lvl_b[(size_t)q].size();
                    sym.arena.insert(sym.arena.end(), lvl_x[(size_t)q].begin(), lvl_x[(size_t)q].end());
                    sym.arena.insert(sym.arena.end(), lvl_b[(size_t)q].begin(), lvl_b[(size_t)q].end());
                }
            }
        } else {
            close_stage(sp, sym, threads);
            ++stage;
            p.stage_of_level[(size_t)l] = stage;
            a = l;
            depth = 1;
        }
    }
    close_stage(sp, sym, threads);
    p.nstages = nlev > 0 ? stage + 1 : 0;
}

// The rewritten system L' and the counts of M; M's entries too when keep_m.
// Every rewritten row is rebuilt with a dense accumulator: its equation,
// then its in-stage b-terms eliminated from the highest column down.
static void build_rewritten(Plan &p, const Symbolic &sym, bool keep_m) {
    const int32_t n = p.n;
    auto rewritten = [&](int32_t i) { return sym.off[(size_t)i] >= 0 || sym.doff[(size_t)i] >= 0; };
    p.lp_ptr.assign((size_t)n + 1, 0);
    p.m_ptr.assign((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        const bool rw = rewritten(i);
        p.lp_ptr[(size_t)i + 1] = p.lp_ptr[(size_t)i] +
                                  (rw ? sym.nx[(size_t)i] + 1 : p.rp[(size_t)i + 1] - p.rp[(size_t)i]);
        p.m_ptr[(size_t)i + 1] = p.m_ptr[(size_t)i] + (rw ? sym.nb[(size_t)i] : 0);
    }
    const int64_t nlp = p.lp_ptr[(size_t)n], nm = p.m_ptr[(size_t)n];
    p.lp_col.resize((size_t)nlp);
    p.lp_val.resize((size_t)nlp);
    p.m_col.clear();
    p.m_val.clear();
    p.m_col.shrink_to_fit();
    p.m_val.shrink_to_fit();
    if (keep_m) {
        p.m_col.resize((size_t)nm);
        p.m_val.resize((size_t)nm);
    }
    p.m_kept = keep_m;

    parallel_ranges(n, hw_threads(), [&](int64_t lo, int64_t hi, int) {
        std::vector<double> acc;  // dense accumulator, zero outside the current row
        for (int64_t ii = lo; ii < hi; ++ii) {
            const int32_t i = (int32_t)ii;
            const int64_t out = p.lp_ptr[(size_t)i];
            if (!rewritten(i)) {
                const int32_t b = p.rp[(size_t)i], e = p.rp[(size_t)i + 1];
                std::copy(p.ci.begin() + b, p.ci.begin() + e, p.lp_col.begin() + out);
                std::copy(p.val.begin() + b, p.val.begin() + e, p.lp_val.begin() + out);
                continue;
            }
            if (acc.empty()) acc.assign((size_t)n, 0.0);
            for (int32_t q = p.rp[(size_t)i]; q < p.rp[(size_t)i + 1] - 1; ++q)
                acc[(size_t)p.ci[(size_t)q]] = p.val[(size_t)q];
            const int64_t mo = p.m_ptr[(size_t)i];
            // b-term j (the t-th in column order): eliminate x_j with j's equation
            auto eliminate = [&](int32_t j, int64_t t) {
                const int32_t je = p.rp[(size_t)j + 1] - 1;
                const double c = acc[(size_t)j] / p.val[(size_t)je];
                acc[(size_t)j] = 0.0;
                if (keep_m) {
                    p.m_col[(size_t)(mo + t)] = j;
                    p.m_val[(size_t)(mo + t)] = -c;
                }
                for (int32_t r = p.rp[(size_t)j]; r < je; ++r) {
                    const int32_t k = p.ci[(size_t)r];
                    const double prod = c * p.val[(size_t)r];
                    acc[(size_t)k] = acc[(size_t)k] - prod;
                }
            };
            auto emit = [&](int32_t k, int64_t t) {
                p.lp_col[(size_t)(out + t)] = k;
                p.lp_val[(size_t)(out + t)] = acc[(size_t)k];
                acc[(size_t)k] = 0.0;
            };
            const int32_t nx = sym.nx[(size_t)i], nb = sym.nb[(size_t)i];
            if (sym.off[(size_t)i] >= 0) {
                const int32_t *xs = sym.arena.data() + sym.off[(size_t)i];
                const int32_t *bs = xs + nx;
                for (int32_t t = nb - 1; t >= 0; --t) eliminate(bs[t], t);
                for (int32_t t = 0; t < nx; ++t) emit(xs[t], t);
            } else {
                const int32_t st = sym.dstage[(size_t)i], W = sym.st_words[(size_t)st];
                const uint64_t *B = sym.bits.data() + sym.doff[(size_t)i];
                const int32_t *rows = sym.st_rows.data() + sym.st_roff[(size_t)st];
                const uint64_t *isb = sym.st_isb.data() + sym.st_woff[(size_t)st];
                int64_t t = nb - 1;
                for (int32_t w = W - 1; w >= 0; --w)
                    for (uint64_t m = B[w] & isb[w]; m;) {
                        const int bit = 63 - __builtin_clzll(m);
                        m &= ~(uint64_t(1) << bit);
                        eliminate(rows[w * 64 + bit], t--);
                    }
                t = 0;
                for (int32_t w = 0; w < W; ++w)
                    for (uint64_t m = B[w] & ~isb[w]; m; m &= m - 1) emit(rows[w * 64 + __builtin_ctzll(m)], t++);
            }
            p.lp_col[(size_t)(out + nx)] = i;
            p.lp_val[(size_t)(out + nx)] = p.val[(size_t)p.rp[(size_t)i + 1] - 1];
        }
    });
}

void rewrite(Plan &p, const sptrsv_policy &pol) {
    validate_policy(pol);
    const int32_t n = p.n;
    p.policy = pol;
    p.policy.absorb = nullptr;  // the mask and the model are read during this call only
    p.policy.model = nullptr;

    Symbolic sym;
    select_stages(p, pol, sym);

    // M's entries are stored only when the right-hand-side step will read
    // them; the stage solve reads L_B instead (materialise_m builds M later)
    int64_t nm = 0;
    for (int32_t i = 0; i < n; ++i) nm += sym.nb[(size_t)i];
    const bool keep_m = p.is_sub || nm == 0 || choose_rhs(p, nm, stage_system_nnz(p)) != kRhsStage;
    build_rewritten(p, sym, keep_m);
    sym = Symbolic();

    // ---- re-level L' (emptied levels vanish) and build the schedule
    p.level_rw.resize((size_t)n);
    int32_t maxlev = -1;
    for (int32_t i = 0; i < n; ++i) {
        int32_t lv = 0;
        for (int64_t q = p.lp_ptr[(size_t)i]; q < p.lp_ptr[(size_t)i + 1] - 1; ++q)
            lv = std::max(lv, p.level_rw[(size_t)p.lp_col[(size_t)q]] + 1);
        p.level_rw[(size_t)i] = lv;
        maxlev = std::max(maxlev, lv);
    }
    p.nlev_rw = maxlev + 1;
    level_sets(n, p.level_rw.data(), p.nlev_rw, p.sched_ptr, p.sched_rows);
    pack(p);
}

void materialise_m(Plan &p) {
    if (p.m_kept) return;
    // the stages are fixed: select them again as an explicit mask (the same
    // structures, deltas and stages) and rebuild with M's entries
    const int32_t nlev = p.nlev;
    std::vector<uint8_t> mask((size_t)std::max(nlev, 1), 0);
    for (int32_t l = 1; l < nlev; ++l)
        mask[(size_t)l] = p.stage_of_level[(size_t)l] == p.stage_of_level[(size_t)l - 1];
    sptrsv_policy fixed{};
    fixed.kind = SPTRSV_POLICY_EXPLICIT;
    fixed.absorb = mask.data();
    fixed.absorb_len = nlev;
    fixed.max_entries = std::numeric_limits<int64_t>::max();
    Symbolic sym;
    select_stages(p, fixed, sym);
    build_rewritten(p, sym, true);
}

}  // namespace sptrsv
