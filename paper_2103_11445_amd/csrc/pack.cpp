// pack.cpp -- device image of a plan: the executed schedule (level sets of
// L') as a list of work items in level order, and what the right-hand-side
// step b' = b + M b needs.
//
// Right-hand side.  The b-terms of the rewritten rows depend on nothing the
// solve computes, so they are not part of the schedule.  Either a fully
// parallel pass over "M tiles" (rows binned by their count of b-terms, the
// same tile shape as below) computes b'_i = b_i + sum_j M_ij b_j for every
// row (and resets x), or, when M is large, the image carries a second plan:
// the stages' diagonal blocks of L (L_B), whose solve y gives b' = D y.  The
// solve tiles hold x-terms only and read b' (or y, scaled by the diagonal).
//
// Wide items.  Within a level, rows are binned by x-term count: a row of
// `len` terms gets g lanes, the smallest power of two with
// len <= t * g (capped at 64), t the plan's terms per lane (4 by default,
// sptrsv_set_tiling).  A tile holds 64/g rows of one bin
// of one level; its terms occupy `nchunks` chunks of 64 slots, the t-th term
// of the tile's r-th row at chunk t / g, lane r * g + t % g.  A term is an
// x-term (column k, coefficient -L'_ik); unused slots hold INT32_MIN.
// Columns are slots, not rows: the solve keeps x in slot (schedule) order
// in the image, where a level's rows sit side by side, so a tile's results
// go to a few consecutive lines and the values a level gathers from the one
// before it are near each other; every value is also stored once, in the
// caller's order, into the caller's x.
//
// Segments.  A level is narrow when its rows fit in at most kNarrowTiles
// tiles of kSegChunks chunks (g = 64 / rows-per-tile, as many lanes per row
// as the tile allows).  A run of at least kMinSegLevels narrow levels is a
// segment, executed by one wave from first tile to last: dependencies on
// rows of the same segment produced at most kRing rows earlier are read
// from the wave's LDS ring (column n + ring index) instead of global memory.
// A segment whose terms all come from the ring is flagged in its descriptor
// and gathers nothing but the constants; its pads point at the ring's zero
// slot (column n + kRing).
// Segment tiles are stored with a fixed stride, lane-major (each lane's
// kSegChunks columns, then its coefficients, contiguous; one {row id, meta,
// slot} record and one diagonal per lane) so the wave prefetches a tile with a few
// wide loads, several tiles ahead, without reading a descriptor first.
//
// Items are ordered by level, so an item only depends on items before it.
// Within a wide level, rows that some other row depends on (the chain) and
// rows nothing depends on (sinks) go to separate tiles: chain tiles and
// segments form the first queue of items, sink tiles the second (each in
// level order), served by separate waves.  A sink never delays a chain row.
#include <algorithm>
#include <cstdlib>
#include <climits>
#include <cstring>
#include <memory>
#include <string>

#include "plan.hpp"

namespace sptrsv {

namespace {

constexpr int kBins = 7;  // g = 1, 2, 4, ..., 64
constexpr int kKinds = 7;  // copies per row: 1, 2, 4, ..., 64
constexpr int32_t kPad = INT32_MIN;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int bin_of(int64_t len, int terms_per_lane) {
    int lg = 0;
    while (lg < kBins - 1 && len > (int64_t)terms_per_lane << lg) ++lg;
    return lg;
}

// log2 of the lanes per row of a segment tile whose longest row has
// `maxlen` terms (kSegChunks chunks), or -1 if no width fits.
int seg_lanes_log2(int64_t maxlen) {
    for (int lg = 0; lg <= 6; ++lg)
        if (maxlen <= (int64_t)kSegChunks << lg) return lg;
    return -1;
}
}  // namespace

// The block-diagonal part of L inside the stages: entries (i, j) whose
// levels belong to the same stage (diagonal included), in CSR.
static void stage_system(const Plan &p, std::vector<int32_t> &rp, std::vector<int32_t> &ci,
                         std::vector<double> &val) {
    const int32_t n = p.n;
    rp.assign((size_t)n + 1, 0);
    ci.clear();
    val.clear();
    for (int32_t i = 0; i < n; ++i) {
        const int32_t si = p.stage_of_level[(size_t)p.level[(size_t)i]];
        for (int32_t q = p.rp[(size_t)i]; q < p.rp[(size_t)i + 1]; ++q) {
            const int32_t j = p.ci[(size_t)q];
            if (p.stage_of_level[(size_t)p.level[(size_t)j]] != si) continue;
            ci.push_back(j);
            val.push_back(p.val[(size_t)q]);
        }
        rp[(size_t)i + 1] = (int32_t)ci.size();
    }
}

int64_t stage_system_nnz(const Plan &p) {
    int64_t c = 0;
    for (int32_t i = 0; i < p.n; ++i) {
        const int32_t si = p.stage_of_level[(size_t)p.level[(size_t)i]];
        for (int32_t q = p.rp[(size_t)i]; q < p.rp[(size_t)i + 1]; ++q)
            c += p.stage_of_level[(size_t)p.level[(size_t)p.ci[(size_t)q]]] == si;
    }
    return c;
}

// Choice of the right-hand-side step: none without b-terms; else as
// requested, or the stage solves when M holds more than twice the entries
// of L_B (its bytes then dominate the M pass).
int32_t choose_rhs(const Plan &p, int64_t nnz_m, int64_t nnz_b) {
    if (nnz_m == 0 || p.is_sub) return kRhsNone;
    if (p.rhs_request == kRhsMPass || p.rhs_request == kRhsStage) return p.rhs_request;
    return nnz_m > 2 * nnz_b ? kRhsStage : kRhsMPass;
}

void pack(Plan &p) {
    const int32_t n = p.n;
    if ((int64_t)n + kRing > INT32_MAX)
        throw Error{SPTRSV_ERR_OVERFLOW, "n too large for the device encoding"};
    // the kernels address x and b by 32-bit byte offsets
    if ((uint64_t)n * (uint64_t)(p.precision / 8) > 0xFFFFFFFFull)
        throw Error{SPTRSV_ERR_OVERFLOW, "n * value bytes beyond 2^32 (32-bit gather offsets)"};
    // ---- right-hand-side step
    int32_t rhs_mode = kRhsNone;
    int64_t nnz_rhs = 0;
    p.sub.reset();
    if (p.nnz_m() > 0 && !p.is_sub) {
        std::vector<int32_t> brp, bci;
        std::vector<double> bval;
        stage_system(p, brp, bci, bval);
        rhs_mode = choose_rhs(p, p.nnz_m(), (int64_t)bci.size());
        if (rhs_mode == kRhsMPass) materialise_m(p);
        if (rhs_mode == kRhsStage) {
            std::unique_ptr<Plan> sub(new Plan());
            sub->is_sub = true;
            sub->precision = p.precision;
            sub->terms_per_lane = p.terms_per_lane;
            analyse(*sub, n, brp.data(), bci.data(), bval.data());
            sub->upper = p.upper;
            // the stage system of a batched plan holds the same copies
            sub->batch_count = p.batch_count;
            sub->sys_n = p.sys_n;
            sub->sys_k = p.sys_k;
            sub->sys_base = p.sys_base;
            sub->comp.resize((size_t)n);
            for (int32_t i = 0; i < n; ++i) sub->comp[(size_t)i] = p.stage_of_level[(size_t)p.level[(size_t)i]];
            sptrsv_policy none{};
            none.kind = SPTRSV_POLICY_NONE;
            rewrite(*sub, none);  // packs the stage system's image
            nnz_rhs = sub->nnz_streamed;
            p.sub = std::move(sub);
        } else {
            nnz_rhs = p.nnz_m();
        }
    }
    std::vector<int64_t> len((size_t)n);
    for (int32_t i = 0; i < n; ++i) len[(size_t)i] = p.lp_ptr[(size_t)i + 1] - p.lp_ptr[(size_t)i] - 1;

    // ---- classify levels: narrow levels and their segment tile shape
    const int32_t L = p.nlev_rw;
    std::vector<int8_t> seg_lg((size_t)L, -1);  // lanes-per-row log2 if narrow
    for (int32_t l = 0; l < L; ++l) {
        const int32_t b0 = p.sched_ptr[(size_t)l], b1 = p.sched_ptr[(size_t)l + 1];
        int64_t mx = 0;
        for (int32_t q = b0; q < b1; ++q) mx = std::max(mx, len[(size_t)p.sched_rows[(size_t)q]]);
        const int lg = seg_lanes_log2(mx);
        if (lg < 0) continue;
        const int32_t per = 64 >> lg;
        if ((b1 - b0 + per - 1) / per <= kNarrowTiles) seg_lg[(size_t)l] = (int8_t)lg;
    }
    std::vector<char> in_seg((size_t)L, 0);
    for (int32_t l = 0; l < L;) {
        int32_t e = l;
        while (e < L && seg_lg[(size_t)e] >= 0) ++e;
        if (e - l >= kMinSegLevels)
            for (int32_t q = l; q < e; ++q) in_seg[(size_t)q] = 1;
        l = std::max(e, l + 1);
    }

    // ---- order rows and cut items
    std::vector<int32_t> slot_row((size_t)n);
    // a wide tile: its chunks, slots, rows, lanes per row (2^lg) and, for rows
    // that are copies of one row for several right-hand sides (a batched
    // plan), 2^lgk copies per row with the first row's copy index c0
    struct Tile { int64_t chunk_off; int32_t row_off, nch, nrows, lg, lgk = 0, c0 = 0; };
    struct SegTile { int32_t row_off, nrows, lg, level; };
    struct Item { int kind; int64_t a, b; int32_t level; };  // wide: a = wide tile; seg: a = first seg tile, b = count
    std::vector<Tile> tiles;
    std::vector<SegTile> stiles;
    std::vector<Item> items, sink_items;  // the chain queue, the sink queue
    // rows of L' that another row of L' depends on
    // (with one queue every row counts as needed: all go to the first queue)
    std::vector<char> needed((size_t)n, p.queues == 1 ? 1 : 0);
    if (p.queues != 1)
        for (int32_t i = 0; i < n; ++i)
            for (int64_t q = p.lp_ptr[(size_t)i]; q < p.lp_ptr[(size_t)i + 1] - 1; ++q)
                needed[(size_t)p.lp_col[(size_t)q]] = 1;
    std::vector<int32_t> seg_of_slot((size_t)n, -1);   // segment id of each slot
    // copies per row (log2) where a batched plan holds a power-of-two k <= 64
    // copies of each row of a system (0 otherwise: each row its own terms),
    // and the copy index of each row
    std::vector<int8_t> copies_lg((size_t)n, 0);
    std::vector<int32_t> copy_of((size_t)n, 0);
    for (size_t j = 0; j < p.sys_k.size(); ++j) {
        const int32_t kj = p.sys_k[j];
        if (kj <= 1 || kj > 64 || (kj & (kj - 1)) || p.upper) continue;
        int lgk = 0;
        while ((1 << lgk) < kj) ++lgk;
        const int64_t b0 = p.sys_base[j], b1 = b0 + (int64_t)p.sys_n[j] * kj;
        for (int64_t u = b0; u < b1; ++u) {
            copies_lg[(size_t)u] = (int8_t)lgk;
            copy_of[(size_t)u] = (int32_t)((u - b0) & (kj - 1));
        }
    }
    int64_t nchunks = 0;
    int32_t slot = 0, nseg = 0;

    // rows[0, count) of level l (ascending) as wide tiles, binned by length
    // and by copies per row, appended to the chain queue or, for sinks, to
    // the sink queue.  The copies of a row (same level, length and
    // dependents) are consecutive in a bin, so copy c of a row sits c slots
    // after copy 0 and its terms are copy 0's shifted by c slots: a tile
    // stores the terms of copy 0 only, and the lanes of copy c add c.
    auto bin2 = [&](int32_t r) { return bin_of(len[(size_t)r], p.terms_per_lane) * kKinds + copies_lg[(size_t)r]; };
    auto wide_tiles = [&](const int32_t *rows, int32_t count, int32_t l, bool sink) {
        int32_t cnt[kBins * kKinds] = {0};
        for (int32_t q = 0; q < count; ++q) ++cnt[bin2(rows[q])];
        int32_t start[kBins * kKinds];
        int32_t acc = slot;
        for (int b = 0; b < kBins * kKinds; ++b) {
            start[b] = acc;
            acc += cnt[b];
        }
        int32_t cur[kBins * kKinds];
        std::copy(start, start + kBins * kKinds, cur);
        for (int32_t q = 0; q < count; ++q) {
            const int32_t r = rows[q];
            slot_row[(size_t)cur[bin2(r)]++] = r;
        }
        for (int b = 0; b < kBins * kKinds; ++b) {
            const int g = b / kKinds, lgk = b % kKinds;
            const int32_t per = 64 >> g;
            int64_t group_chunks = 0;  // chunks of the tile holding copy 0 of the current row
            for (int32_t s = start[b]; s < start[b] + cnt[b]; s += per) {
                const int32_t nr = std::min(per, start[b] + cnt[b] - s);
                int64_t mx = 0;
                for (int32_t r = 0; r < nr; ++r) mx = std::max(mx, len[(size_t)slot_row[(size_t)(s + r)]]);
                const int64_t nch = (mx + (1 << g) - 1) >> g;
                const int32_t c0 = copy_of[(size_t)slot_row[(size_t)s]];
                (sink ? sink_items : items).push_back({0, (int64_t)tiles.size(), 0, l});
                if (lgk > 0 && c0 > 0) {
                    // later copies of one row (more copies than rows per
                    // tile): read the terms of the tile with copy 0
                    tiles.push_back({group_chunks, s, (int32_t)nch, nr, g, lgk, c0});
                    continue;
                }
                group_chunks = nchunks;
                tiles.push_back({nchunks, s, (int32_t)nch, nr, g, lgk, c0});
                nchunks += nch;
            }
        }
        slot = acc;
    };
    std::vector<int32_t> chain_rows, sink_rows;
    auto wide_level = [&](const int32_t *rows, int32_t count, int32_t l) {
        chain_rows.clear();
        sink_rows.clear();
        for (int32_t q = 0; q < count; ++q) (needed[(size_t)rows[q]] ? chain_rows : sink_rows).push_back(rows[q]);
        if (!chain_rows.empty()) wide_tiles(chain_rows.data(), (int32_t)chain_rows.size(), l, false);
        if (!sink_rows.empty()) wide_tiles(sink_rows.data(), (int32_t)sink_rows.size(), l, true);
    };
    // a new segment
    auto open_segment = [&]() {
        items.push_back({1, (int64_t)stiles.size(), 0, -1});
        ++nseg;
    };
    // rows[0, count) of level l appended to the open segment as tiles of
    // 2^lg lanes per row; `level` is what their stamps report
    auto seg_level = [&](const int32_t *rows, int32_t count, int lg, int32_t level) {
        const int32_t per = 64 >> lg;
        for (int32_t q = 0; q < count; ++q) {
            slot_row[(size_t)(slot + q)] = rows[q];
            seg_of_slot[(size_t)(slot + q)] = nseg - 1;
        }
        for (int32_t s = slot; s < slot + count; s += per) {
            stiles.push_back({s, std::min(per, slot + count - s), lg, level});
            items.back().b += 1;
        }
        slot += count;
    };
    // pad the open segment to a whole number of pipeline steps with empty
    // tiles (no rows, no terms)
    auto close_segment = [&]() {
        while (items.back().b % kSegDepth) {
            stiles.push_back({slot, 0, 0, -1});
            items.back().b += 1;
        }
    };

    // ---- independent stages of a stage system: a stage whose levels need
    // at most kStageSegTiles segment tiles each (on average) runs as one
    // segment, start to finish on one wave, with no wait on another wave;
    // the remaining rows follow as wide tiles, level by level
    std::vector<int32_t> comp_rows, comp_ptr;  // rows of each stage in schedule order
    std::vector<char> comp_seg;
    int32_t ncomp = 0, comp_segs = 0;
    if (!p.comp.empty()) {
        for (int32_t i = 0; i < n; ++i) ncomp = std::max(ncomp, p.comp[(size_t)i] + 1);
        comp_ptr.assign((size_t)ncomp + 1, 0);
        for (int32_t i = 0; i < n; ++i) ++comp_ptr[(size_t)p.comp[(size_t)i] + 1];
        for (int32_t c = 0; c < ncomp; ++c) comp_ptr[(size_t)c + 1] += comp_ptr[(size_t)c];
        comp_rows.resize((size_t)n);
        std::vector<int32_t> fill(comp_ptr.begin(), comp_ptr.end() - 1);
        for (int32_t q = 0; q < n; ++q) {
            const int32_t r = p.sched_rows[(size_t)q];
            comp_rows[(size_t)fill[(size_t)p.comp[(size_t)r]]++] = r;
        }
        comp_seg.assign((size_t)ncomp, 0);
        std::vector<int64_t> ctiles((size_t)ncomp, 0);
        for (int32_t c = 0; c < ncomp; ++c) {
            int64_t depth = 0, ntl = 0;
            bool ok = true;
            for (int32_t q = comp_ptr[(size_t)c]; q < comp_ptr[(size_t)c + 1] && ok;) {
                const int32_t l = p.level_rw[(size_t)comp_rows[(size_t)q]];
                int32_t e = q;
                int64_t mx = 0;
                for (; e < comp_ptr[(size_t)c + 1] && p.level_rw[(size_t)comp_rows[(size_t)e]] == l; ++e)
                    mx = std::max(mx, len[(size_t)comp_rows[(size_t)e]]);
                const int lg = seg_lanes_log2(mx);
                ok = lg >= 0;
                if (ok) ntl += (e - q + (64 >> lg) - 1) / (64 >> lg);
                ++depth;
                q = e;
            }
            comp_seg[(size_t)c] = ok && depth >= 2 && ntl <= (int64_t)kStageSegTiles * depth;
            ctiles[(size_t)c] = ntl;
            comp_segs += comp_seg[(size_t)c];
        }
        if (comp_segs == 0) {
            comp_rows.clear();
        } else {
            // longest first, so that a wave holding two of them gets short ones
            std::vector<int32_t> order;
            for (int32_t c = 0; c < ncomp; ++c)
                if (comp_seg[(size_t)c]) order.push_back(c);
            std::stable_sort(order.begin(), order.end(),
                             [&](int32_t u, int32_t v) { return ctiles[(size_t)u] > ctiles[(size_t)v]; });
            for (int32_t c : order) {
                open_segment();
                for (int32_t q = comp_ptr[(size_t)c]; q < comp_ptr[(size_t)c + 1];) {
                    const int32_t l = p.level_rw[(size_t)comp_rows[(size_t)q]];
                    int32_t e = q;
                    int64_t mx = 0;
                    for (; e < comp_ptr[(size_t)c + 1] && p.level_rw[(size_t)comp_rows[(size_t)e]] == l; ++e)
                        mx = std::max(mx, len[(size_t)comp_rows[(size_t)e]]);
                    seg_level(comp_rows.data() + q, e - q, seg_lanes_log2(mx), -1);
                    q = e;
                }
                close_segment();
            }
            std::vector<int32_t> rest;
            for (int32_t l = 0; l < L; ++l) {
                rest.clear();
                for (int32_t q = p.sched_ptr[(size_t)l]; q < p.sched_ptr[(size_t)l + 1]; ++q) {
                    const int32_t r = p.sched_rows[(size_t)q];
                    if (!comp_seg[(size_t)p.comp[(size_t)r]]) rest.push_back(r);
                }
                if (!rest.empty()) wide_level(rest.data(), (int32_t)rest.size(), l);
            }
        }
    }
    if (comp_segs == 0) {
        for (int32_t l = 0; l < L; ++l) {
            const int32_t b0 = p.sched_ptr[(size_t)l], b1 = p.sched_ptr[(size_t)l + 1];
            if (!in_seg[(size_t)l]) {
                wide_level(p.sched_rows.data() + b0, b1 - b0, l);
                continue;
            }
            if (l == 0 || !in_seg[(size_t)l - 1]) open_segment();
            seg_level(p.sched_rows.data() + b0, b1 - b0, seg_lg[(size_t)l], l);
            if (l + 1 == L || !in_seg[(size_t)l + 1]) close_segment();
        }
    }
    const int64_t nchain = (int64_t)items.size();
    // work of each queue: 64-lane chunks of terms plus one per tile for the
    // rows (segment tiles: kSegChunks chunks each)
    auto work = [&](const std::vector<Item> &v) {
        int64_t w = 0;
        for (const Item &I : v) w += I.kind == 1 ? I.b * (kSegChunks + 1) : tiles[(size_t)I.a].nch + 1;
        return w;
    };
    p.chain_work = work(items);
    p.sink_work = work(sink_items);
    items.insert(items.end(), sink_items.begin(), sink_items.end());
    sink_items.clear();
    if (nchunks > INT32_MAX || (int64_t)items.size() > INT32_MAX || (int64_t)stiles.size() * 64 > INT32_MAX)
        throw Error{SPTRSV_ERR_OVERFLOW, "device image needs more than INT32_MAX chunks"};
    std::vector<int32_t> slot_of_row((size_t)n);
    for (int32_t s = 0; s < n; ++s) slot_of_row[(size_t)slot_row[(size_t)s]] = s;
    // first slot of every segment (for ring positions)
    std::vector<int32_t> seg_first((size_t)nseg, 0);
    {
        int32_t sid = -1;
        for (const Item &it : items)
            if (it.kind == 1) seg_first[(size_t)++sid] = stiles[(size_t)it.a].row_off;
    }

    // ---- M tiles: every row once, binned by its b-term count, in the order
    // of the caller's indices within a bin (so the pass reads b and writes b'
    // and x in runs of consecutive entries)
    std::vector<int32_t> mslot_row((size_t)n);
    std::vector<Tile> mtiles;
    int64_t mchunks = 0;
    if (rhs_mode == kRhsMPass) {
        int32_t cnt[kBins] = {0};
        auto mlen = [&](int32_t i) { return p.m_ptr[(size_t)i + 1] - p.m_ptr[(size_t)i]; };
        auto row_at = [&](int32_t d) { return p.upper ? n - 1 - d : d; };  // plan row of caller index d
        for (int32_t i = 0; i < n; ++i) ++cnt[bin_of(mlen(i), p.terms_per_lane)];
        int32_t start[kBins], cur[kBins], acc = 0;
        for (int g = 0; g < kBins; ++g) {
            start[g] = cur[g] = acc;
            acc += cnt[g];
        }
        for (int32_t d = 0; d < n; ++d) {
            const int32_t r = row_at(d);
            mslot_row[(size_t)cur[bin_of(mlen(r), p.terms_per_lane)]++] = r;
        }
        for (int g = 0; g < kBins; ++g) {
            const int32_t per = 64 >> g;
            for (int32_t s = start[g]; s < start[g] + cnt[g]; s += per) {
                const int32_t nr = std::min(per, start[g] + cnt[g] - s);
                int64_t mx = 0;
                for (int32_t r = 0; r < nr; ++r) mx = std::max(mx, mlen(mslot_row[(size_t)(s + r)]));
                const int64_t nch = (mx + (1 << g) - 1) >> g;
                mtiles.push_back({mchunks, s, (int32_t)nch, nr, g});
                mchunks += nch;
            }
        }
    }
    if (mchunks > INT32_MAX || (int64_t)mtiles.size() > INT32_MAX)
        throw Error{SPTRSV_ERR_OVERFLOW, "device image needs more than INT32_MAX chunks"};

    // ---- compact columns: a wide tile's terms all read earlier levels, so
    // each column is stored as its distance back from the tile's first
    // slot; when every distance fits in 16 bits (and no copies share terms)
    // the column array is halved.  SPTRSV_COMPACT_COLS=0 keeps 32 bits.
    bool compact = !tiles.empty();
    {
        const char *env = std::getenv("SPTRSV_COMPACT_COLS");
        if (env && env[0] == '0') compact = false;
    }
    int64_t nnz_col16 = 0;
    if (compact) {
        const int threads = hw_threads();
        std::vector<char> fits((size_t)threads, 1);
        std::vector<int64_t> terms((size_t)threads, 0);
        parallel_ranges((int64_t)tiles.size(), threads, [&](int64_t lo, int64_t hi, int w) {
            for (int64_t t = lo; t < hi && fits[(size_t)w]; ++t) {
                const Tile &T = tiles[(size_t)t];
                if (T.lgk != 0 || T.c0 != 0) {
                    fits[(size_t)w] = 0;
                    break;
                }
                for (int32_t r = 0; r < T.nrows; ++r) {
                    const int32_t i = slot_row[(size_t)(T.row_off + r)];
                    for (int64_t q = p.lp_ptr[(size_t)i]; q < p.lp_ptr[(size_t)i + 1] - 1; ++q) {
                        const int64_t dist = (int64_t)T.row_off - slot_of_row[(size_t)p.lp_col[(size_t)q]];
                        if (dist < 1 || dist > 65535) fits[(size_t)w] = 0;
                    }
                    terms[(size_t)w] += p.lp_ptr[(size_t)i + 1] - p.lp_ptr[(size_t)i] - 1;
                }
            }
        });
        for (int w = 0; w < threads; ++w) compact = compact && fits[(size_t)w];
        if (compact)
            for (int64_t t : terms) nnz_col16 += t;
    }

    // ---- layout
    const int64_t nst = (int64_t)stiles.size();
    const bool f32 = p.precision == 32;
    const size_t vb = f32 ? 4 : 8;
    Layout &Ly = p.layout;
    Ly = Layout{};
    Ly.value_bytes = (int)vb;
    // the kernel instance that holds 8 chunks of a wide tile in registers
    // when most tiles need more than 4 (their terms are then gathered before
    // the dependency wait instead of streamed after it)
    {
        int64_t longer = 0;
        for (const Tile &T : tiles) longer += T.nch > 4 ? 1 : -1;
        Ly.reg_chunks = longer > 0 ? 8 : 4;
    }
    size_t off = 0;
    Ly.workspace = off;
    off = align256(off + sizeof(Workspace));
    Ly.tiles = off;
    off = align256(off + items.size() * 16);
    Ly.rows = off;
    off = align256(off + (size_t)n * 4);
    Ly.diag = off;
    off = align256(off + (size_t)n * vb);
    Ly.col16 = compact ? 1 : 0;
    Ly.tcol = off;
    off = align256(off + (size_t)nchunks * 64 * (compact ? 2 : 4));
    Ly.tval = off;
    off = align256(off + (size_t)nchunks * 64 * vb);
    Ly.scol = off;
    off = align256(off + (size_t)nst * kSegChunks * 64 * 4);
    Ly.sval = off;
    off = align256(off + (size_t)nst * kSegChunks * 64 * vb);
    Ly.srow = off;
    off = align256(off + (size_t)nst * 64 * 16);
    Ly.sdiag = off;
    off = align256(off + (size_t)nst * 64 * vb);
    Ly.mtiles = off;
    off = align256(off + mtiles.size() * 16);
    Ly.mrow = off;
    off = align256(off + (size_t)n * 4);
    Ly.mcol = off;
    off = align256(off + (size_t)mchunks * 64 * 4);
    Ly.mval = off;
    off = align256(off + (size_t)mchunks * 64 * vb);
    Ly.bp = off;
    off = align256(off + (size_t)n * vb);
    Ly.xs = off;
    off = align256(off + (size_t)n * vb);
    Ly.nmtiles = (int64_t)mtiles.size();
    Ly.rhs_mode = rhs_mode;
    Ly.nnz_rhs = nnz_rhs;
    if (f32 && !p.is_sub) {
        Ly.nsys = (int32_t)p.sys_n.size();
        for (size_t j = 0; j < p.sys_n.size(); ++j) {
            // a system's block of the union holds k identical copies
            const int64_t nj = p.sys_n[j], kj = p.sys_k[j], r0 = p.sys_base[j];
            Ly.res_rows += nj;
            Ly.res_nnz += ((int64_t)p.rp[(size_t)(r0 + nj * kj)] - p.rp[(size_t)r0]) / kj;
        }
        if (Ly.res_nnz > INT32_MAX) throw Error{SPTRSV_ERR_OVERFLOW, "residual matrix beyond int32 indexing"};
        Ly.sys = off;
        off = align256(off + (size_t)Ly.nsys * 16);
        Ly.res_rp = off;
        off = align256(off + (size_t)(Ly.res_rows + 1) * 4);
        Ly.res_col = off;
        off = align256(off + (size_t)Ly.res_nnz * 4);
        Ly.res_val = off;
        off = align256(off + (size_t)Ly.res_nnz * 8);
        Ly.r32 = off;
        off = align256(off + (size_t)n * 4);
        Ly.d32 = off;
        off = align256(off + (size_t)n * 4);
    }
    if (p.sub) {
        Ly.sub = off;
        Ly.sub_layout = &p.sub->layout;
        off = align256(off + p.sub->layout.total);
    }
    Ly.total = off;

    p.image.clear();
    p.image.resize(Ly.total);  // left uninitialised by its allocator, then cleared in parallel
    parallel_zero(p.image.data(), p.image.size());
    if (p.sub) std::copy(p.sub->image.begin(), p.sub->image.end(), p.image.begin() + (ptrdiff_t)Ly.sub);
    unsigned char *img = p.image.data();
    int32_t *trow = reinterpret_cast<int32_t *>(img + Ly.rows);
    int32_t *tcol = reinterpret_cast<int32_t *>(img + Ly.tcol);
    uint16_t *tcol16 = reinterpret_cast<uint16_t *>(img + Ly.tcol);  // compact: 0 marks a pad
    int32_t *desc = reinterpret_cast<int32_t *>(img + Ly.tiles);
    int32_t *scol = reinterpret_cast<int32_t *>(img + Ly.scol);
    int32_t *srow = reinterpret_cast<int32_t *>(img + Ly.srow);  // {row, meta, slot, 0} per lane
    // value sections: FP64, or rounded to nearest FP32
    auto putv = [&](size_t section, int64_t idx, double v) {
        if (f32)
            reinterpret_cast<float *>(img + section)[idx] = (float)v;
        else
            reinterpret_cast<double *>(img + section)[idx] = v;
    };
    if (!compact)
        parallel_ranges(nchunks * 64, hw_threads(), [&](int64_t lo, int64_t hi, int) {
            std::fill(tcol + lo, tcol + hi, kPad);
        });
    parallel_ranges(nst * kSegChunks * 64, hw_threads(), [&](int64_t lo, int64_t hi, int) {
        std::fill(scol + lo, scol + hi, kPad);
    });
    for (int64_t q = 0; q < nst * 64; ++q) srow[4 * q] = -1;
    // the device image speaks the caller's indices (reversed for upper
    // input; a batched union is numbered like the callers' blocks already)
    auto orig = [&](int32_t i) { return p.upper ? n - 1 - i : i; };
    for (int32_t s = 0; s < n; ++s) {
        const int32_t i = slot_row[(size_t)s];
        trow[s] = orig(i);
        putv(Ly.diag, s, p.lp_val[(size_t)p.lp_ptr[(size_t)i + 1] - 1]);
    }

    // x-terms of row i for a tile with 2^lg lanes per row, written through put(col, val)
    auto row_terms = [&](int32_t i, int32_t seg, int32_t first_slot_of_tile, auto &&put) {
        for (int64_t q = p.lp_ptr[(size_t)i]; q < p.lp_ptr[(size_t)i + 1] - 1; ++q) {
            const int32_t k = p.lp_col[(size_t)q];
            const int32_t sk = slot_of_row[(size_t)k];
            int32_t col = sk;  // x is gathered in slot order
            if (seg >= 0 && seg_of_slot[(size_t)sk] == seg && first_slot_of_tile - sk <= kRing)
                col = n + ((sk - seg_first[(size_t)seg]) & (kRing - 1));
            put(col, -p.lp_val[(size_t)q]);
        }
    };

    int32_t sid = -1;
    int64_t shared_skip = 0;  // off-diagonal terms of copies that read copy 0's
    bool all_ring = true;
    int32_t ring_count = 0;
    for (size_t it = 0; it < items.size(); ++it) {
        const Item &I = items[it];
        if (I.kind == 1) {
            ++sid;
            bool ring_only = true;  // every term read from the LDS ring
            desc[4 * it + 0] = (int32_t)I.a;
            desc[4 * it + 1] = (int32_t)I.b;
            desc[4 * it + 3] = (int32_t)0x80000000u;
            for (int64_t st = I.a; st < I.a + I.b; ++st) {
                const SegTile &T = stiles[(size_t)st];
                const int32_t g = 1 << T.lg;
                for (int32_t lane = 0; lane < 64; ++lane) srow[4 * (st * 64 + lane) + 1] = T.lg;
                for (int32_t r = 0; r < T.nrows; ++r) {
                    const int32_t s = T.row_off + r;
                    const int32_t i = slot_row[(size_t)s];
                    const int64_t lead = st * 64 + r * g;
                    srow[4 * lead] = orig(i);
                    srow[4 * lead + 1] = T.lg | (((s - seg_first[(size_t)sid]) & (kRing - 1)) << 8);
                    srow[4 * lead + 2] = s;
                    putv(Ly.sdiag, lead, p.lp_val[(size_t)p.lp_ptr[(size_t)i + 1] - 1]);
                    int64_t t_ = 0;
                    row_terms(i, sid, T.row_off, [&](int32_t col, double v) {
                        const int64_t ln = st * 64 + r * g + (t_ & (g - 1));
                        const int64_t idx = ln * kSegChunks + (t_ >> T.lg);
                        scol[idx] = col;
                        putv(Ly.sval, idx, v);
                        ring_only = ring_only && col >= n;
                        ++t_;
                    });
                }
            }
            // a segment without gathers: its pads read the ring's zero slot
            desc[4 * it + 2] = ring_only ? 1 : 0;
            all_ring = all_ring && ring_only;
            ring_count += ring_only;
            if (ring_only)
                for (int64_t q = I.a * 64 * kSegChunks; q < (I.a + I.b) * 64 * kSegChunks; ++q)
                    if (scol[q] == kPad) scol[q] = n + kRing;
            continue;
        }
        const Tile &T = tiles[(size_t)I.a];
        desc[4 * it + 0] = (int32_t)T.chunk_off;
        desc[4 * it + 1] = T.row_off;
        desc[4 * it + 2] = T.nch;
        desc[4 * it + 3] = (T.nrows << 16) | (T.c0 << 8) | (T.lgk << 4) | T.lg;
        const int32_t g = 1 << T.lg;
        for (int32_t r = 0; r < T.nrows; ++r)
            if ((r & ((1 << T.lgk) - 1)) || T.c0 > 0) shared_skip += len[(size_t)slot_row[(size_t)(T.row_off + r)]];
        if (T.c0 > 0) continue;  // its terms are those of the tile with copy 0
        // one row of terms per 2^lgk copies: the first copy of each group
        // (or of the tile, when a group spans tiles), its columns moved back
        // by its copy index to those of copy 0
        for (int32_t r0 = 0; r0 < std::max(1, T.nrows >> T.lgk); ++r0) {
            const int32_t i = slot_row[(size_t)(T.row_off + (r0 << T.lgk))];
            const int32_t c = copy_of[(size_t)i];
            int64_t t_ = 0;
            row_terms(i, -1, 0, [&](int32_t col, double v) {
                const int64_t idx = (T.chunk_off + (t_ >> T.lg)) * 64 + r0 * g + (t_ & (g - 1));
                if (compact)
                    tcol16[idx] = (uint16_t)(T.row_off - col);
                else
                    tcol[idx] = col - c;
                putv(Ly.tval, idx, v);
                ++t_;
            });
        }
    }
    Ly.ring_segs = nseg > 0 && all_ring ? 1 : 0;
    if (rhs_mode == kRhsMPass) {
        // M tiles: b-terms (device index of b_j, coefficient M_ij)
        int32_t *mdesc = reinterpret_cast<int32_t *>(img + Ly.mtiles);
        int32_t *mrow = reinterpret_cast<int32_t *>(img + Ly.mrow);
        int32_t *mcol = reinterpret_cast<int32_t *>(img + Ly.mcol);
        std::fill(mcol, mcol + mchunks * 64, kPad);
        for (int32_t s = 0; s < n; ++s) mrow[s] = orig(mslot_row[(size_t)s]);
        for (size_t t = 0; t < mtiles.size(); ++t) {
            const Tile &T = mtiles[t];
            mdesc[4 * t + 0] = (int32_t)T.chunk_off;
            mdesc[4 * t + 1] = T.row_off;
            mdesc[4 * t + 2] = T.nch;
            mdesc[4 * t + 3] = (T.nrows << 8) | T.lg;
            const int32_t g = 1 << T.lg;
            for (int32_t r = 0; r < T.nrows; ++r) {
                const int32_t i = mslot_row[(size_t)(T.row_off + r)];
                int64_t t_ = 0;
                for (int64_t q = p.m_ptr[(size_t)i]; q < p.m_ptr[(size_t)i + 1]; ++q, ++t_) {
                    const int64_t idx = (T.chunk_off + (t_ >> T.lg)) * 64 + r * g + (t_ & (g - 1));
                    mcol[idx] = orig(p.m_col[(size_t)q]);
                    putv(Ly.mval, idx, p.m_val[(size_t)q]);
                }
            }
        }
    }
    if (f32 && !p.is_sub) {
        // the caller's matrices in FP64 (device indices) for the residual
        int32_t *sys = reinterpret_cast<int32_t *>(img + Ly.sys);
        int32_t *rrp = reinterpret_cast<int32_t *>(img + Ly.res_rp);
        int32_t *rcol = reinterpret_cast<int32_t *>(img + Ly.res_col);
        double *rval = reinterpret_cast<double *>(img + Ly.res_val);
        int64_t row = 0, q = 0;
        rrp[0] = 0;
        for (size_t j = 0; j < p.sys_n.size(); ++j) {
            const int32_t nj = p.sys_n[j], kj = p.sys_k[j];
            const int64_t base = p.sys_base[j];
            sys[4 * j + 0] = (int32_t)base;
            sys[4 * j + 1] = nj;
            sys[4 * j + 2] = kj;
            sys[4 * j + 3] = (int32_t)row;
            for (int32_t i = 0; i < nj; ++i) {
                // plan row holding the caller's row i (its copy 0 in a batch)
                const int64_t r = p.upper ? (int64_t)n - 1 - i : base + (int64_t)i * kj;
                for (int32_t t = p.rp[(size_t)r]; t < p.rp[(size_t)r + 1]; ++t) {
                    if (q >= Ly.res_nnz) throw Error{SPTRSV_ERR_STATE, "internal: residual matrix overflow"};
                    const int64_t l = p.upper ? (int64_t)n - 1 - p.ci[(size_t)t] : (p.ci[(size_t)t] - base) / kj;
                    rcol[q] = (int32_t)(base + l * kj);
                    rval[q] = p.val[(size_t)t];
                    ++q;
                }
                rrp[++row] = (int32_t)q;
            }
        }
        if (row != Ly.res_rows || q != Ly.res_nnz)
            throw Error{SPTRSV_ERR_STATE, "internal: residual matrix size mismatch"};
    }
    // executed level of every completion stamp of an instrumented solve
    p.stamp_level.resize(items.size() + stiles.size());
    for (size_t it = 0; it < items.size(); ++it) p.stamp_level[it] = items[it].level;
    for (size_t st = 0; st < stiles.size(); ++st) p.stamp_level[items.size() + st] = stiles[st].level;
    p.ntiles = (int64_t)items.size();
    p.nchain = nchain;
    p.nnz_streamed = (p.lp_ptr.empty() ? 0 : p.lp_ptr.back()) - shared_skip;
    p.nnz_col16 = nnz_col16;
    p.nchunks = nchunks;
    p.nseg = nseg;
    p.nseg_tiles = nst;
    p.comp_segs = comp_segs;
    p.ring_segs = ring_count;
    p.uploaded = false;
}

}  // namespace sptrsv
