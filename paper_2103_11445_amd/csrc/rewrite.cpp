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

// Symbolic structure of the rewritten rows: for every rewritten row, its
// sorted x-terms and b-terms in one arena.
struct Symbolic {
    std::vector<int64_t> off;    // per row: arena offset, -1 if not rewritten
    std::vector<int32_t> nx, nb; // per row: counts
    std::vector<int32_t> arena;  // x-terms then b-terms of each rewritten row
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

int hw_threads() {
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

}  // namespace

void rewrite(Plan &p, const sptrsv_policy &pol) {
    validate_policy(pol);
    const int32_t n = p.n, nlev = p.nlev;
    const int64_t nnz = n ? (int64_t)p.rp[(size_t)n] : 0;
    p.policy = pol;
    p.policy.absorb = nullptr;  // the mask and the model are read during this call only
    p.policy.model = nullptr;
    p.stage_of_level.assign((size_t)nlev, 0);
    p.delta_of_level.assign((size_t)nlev, 0);

    Symbolic sym;
    sym.off.assign((size_t)n, -1);
    sym.nx.assign((size_t)n, 0);
    sym.nb.assign((size_t)n, 0);

    const int threads = hw_threads();
    std::vector<Marker> markers;
    markers.reserve((size_t)threads);
    for (int w = 0; w < threads; ++w) markers.emplace_back(n);

    // ---- stage selection, level by level
    int64_t budget = std::numeric_limits<int64_t>::max();
    if (pol.kind == SPTRSV_POLICY_THRESHOLD || pol.kind == SPTRSV_POLICY_LEARNED) {
        const double lim = pol.max_fill * (double)nnz;
        if (lim < 9.0e18) budget = (int64_t)std::floor(lim);
    }
    int32_t stage = 0, a = 0, depth = 1;
    int64_t added = 0, total = nnz;
    std::vector<std::vector<int32_t>> lvl_x, lvl_b;  // per row of the candidate level
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
        if (candidate) {
            lvl_x.resize((size_t)width);
            lvl_b.resize((size_t)width);
            std::vector<int64_t> part((size_t)threads, 0), part_max((size_t)threads, 0);
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
            for (int32_t q = 0; q < width; ++q) {
                const int32_t i = p.level_rows[(size_t)(b0 + q)];
                sym.off[(size_t)i] = (int64_t)sym.arena.size();
                sym.nx[(size_t)i] = (int32_t)lvl_x[(size_t)q].size();
                sym.nb[(size_t)i] = (int32_t)lvl_b[(size_t)q].size();
                sym.arena.insert(sym.arena.end(), lvl_x[(size_t)q].begin(), lvl_x[(size_t)q].end());
                sym.arena.insert(sym.arena.end(), lvl_b[(size_t)q].begin(), lvl_b[(size_t)q].end());
            }
        } else {
            ++stage;
            p.stage_of_level[(size_t)l] = stage;
            a = l;
            depth = 1;
        }
    }
    p.nstages = nlev > 0 ? stage + 1 : 0;
    lvl_x.clear();
    lvl_b.clear();

    // ---- rewritten system L' and M
    p.lp_ptr.assign((size_t)n + 1, 0);
    p.m_ptr.assign((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        const bool rw = sym.off[(size_t)i] >= 0;
        p.lp_ptr[(size_t)i + 1] = p.lp_ptr[(size_t)i] +
                                  (rw ? sym.nx[(size_t)i] + 1 : p.rp[(size_t)i + 1] - p.rp[(size_t)i]);
        p.m_ptr[(size_t)i + 1] = p.m_ptr[(size_t)i] + (rw ? sym.nb[(size_t)i] : 0);
    }
    const int64_t nlp = p.lp_ptr[(size_t)n], nm = p.m_ptr[(size_t)n];
    p.lp_col.resize((size_t)nlp);
    p.lp_val.resize((size_t)nlp);
    p.m_col.resize((size_t)nm);
    p.m_val.resize((size_t)nm);

    parallel_ranges(n, threads, [&](int64_t lo, int64_t hi, int) {
        std::vector<double> acc;  // dense accumulator, zero outside the current row
        for (int64_t ii = lo; ii < hi; ++ii) {
            const int32_t i = (int32_t)ii;
            const int64_t out = p.lp_ptr[(size_t)i];
            if (sym.off[(size_t)i] < 0) {
                const int32_t b = p.rp[(size_t)i], e = p.rp[(size_t)i + 1];
                std::copy(p.ci.begin() + b, p.ci.begin() + e, p.lp_col.begin() + out);
                std::copy(p.val.begin() + b, p.val.begin() + e, p.lp_val.begin() + out);
                continue;
            }
            if (acc.empty()) acc.assign((size_t)n, 0.0);
            const int32_t *xs = sym.arena.data() + sym.off[(size_t)i];
            const int32_t nx = sym.nx[(size_t)i], nb = sym.nb[(size_t)i];
            const int32_t *bs = xs + nx;
            for (int32_t q = p.rp[(size_t)i]; q < p.rp[(size_t)i + 1] - 1; ++q)
                acc[(size_t)p.ci[(size_t)q]] = p.val[(size_t)q];
            const int64_t mo = p.m_ptr[(size_t)i];
            for (int32_t t = nb - 1; t >= 0; --t) {
                const int32_t j = bs[t];
                const int32_t je = p.rp[(size_t)j + 1] - 1;
                const double c = acc[(size_t)j] / p.val[(size_t)je];
                acc[(size_t)j] = 0.0;
                p.m_col[(size_t)(mo + t)] = j;
                p.m_val[(size_t)(mo + t)] = -c;
                for (int32_t r = p.rp[(size_t)j]; r < je; ++r) {
                    const int32_t k = p.ci[(size_t)r];
                    const double prod = c * p.val[(size_t)r];
                    acc[(size_t)k] = acc[(size_t)k] - prod;
                }
            }
            for (int32_t t = 0; t < nx; ++t) {
                p.lp_col[(size_t)(out + t)] = xs[t];
                p.lp_val[(size_t)(out + t)] = acc[(size_t)xs[t]];
                acc[(size_t)xs[t]] = 0.0;
            }
            p.lp_col[(size_t)(out + nx)] = i;
            p.lp_val[(size_t)(out + nx)] = p.val[(size_t)p.rp[(size_t)i + 1] - 1];
        }
    });
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

}  // namespace sptrsv
