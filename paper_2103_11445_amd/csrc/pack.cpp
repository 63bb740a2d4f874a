// pack.cpp -- device image of a plan: the executed schedule (level sets of
// L'), cut into 64-lane work tiles, and the rows' terms in a sliced,
// lane-interleaved layout so that every chunk of a tile is one coalesced
// 64-lane load.
//
// Within a level, rows are binned by term count (b-terms + x-terms): a row
// of `len` terms gets g lanes, the smallest power of two with
// len <= kTermsPerLane * g (capped at 64).  A tile holds 64/g rows of one bin
// of one level; its terms occupy `nchunks` chunks of 64 slots, the t-th term
// of the tile's r-th row at chunk t / g, lane r * g + t % g.  Each row lists
// its b-terms (column ~j, coefficient M_ij) before its x-terms (column k,
// coefficient -L'_ik); unused slots hold INT32_MIN.  Tiles are ordered by
// level, so a tile only depends on tiles before it.
#include <algorithm>
#include <climits>
#include <cstring>
#include <string>

#include "plan.hpp"

namespace sptrsv {

namespace {
constexpr int kTermsPerLane = 4;
constexpr int kBins = 7;  // g = 1, 2, 4, ..., 64
constexpr int32_t kPad = INT32_MIN;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int bin_of(int64_t len) {
    int lg = 0;
    while (lg < kBins - 1 && len > (int64_t)kTermsPerLane << lg) ++lg;
    return lg;
}
}  // namespace

void pack(Plan &p) {
    const int32_t n = p.n;
    std::vector<int64_t> len((size_t)n);
    for (int32_t i = 0; i < n; ++i)
        len[(size_t)i] = (p.lp_ptr[(size_t)i + 1] - p.lp_ptr[(size_t)i] - 1) +
                         (p.m_ptr[(size_t)i + 1] - p.m_ptr[(size_t)i]);

    // ---- order rows inside each level by bin, and cut tiles
    std::vector<int32_t> slot_row((size_t)n);
    struct Tile { int64_t chunk_off; int32_t row_off, nch, nrows, lg; };
    std::vector<Tile> tiles;
    int64_t nchunks = 0;
    int32_t slot = 0;
    for (int32_t l = 0; l < p.nlev_rw; ++l) {
        const int32_t b0 = p.sched_ptr[(size_t)l], b1 = p.sched_ptr[(size_t)l + 1];
        int32_t cnt[kBins] = {0};
        for (int32_t q = b0; q < b1; ++q) ++cnt[bin_of(len[(size_t)p.sched_rows[(size_t)q]])];
        int32_t start[kBins];
        int32_t acc = slot;
        for (int g = 0; g < kBins; ++g) {
            start[g] = acc;
            acc += cnt[g];
        }
        int32_t cur[kBins];
        std::copy(start, start + kBins, cur);
        for (int32_t q = b0; q < b1; ++q) {
            const int32_t r = p.sched_rows[(size_t)q];
            slot_row[(size_t)cur[bin_of(len[(size_t)r])]++] = r;
        }
        for (int g = 0; g < kBins; ++g) {
            const int32_t per = 64 >> g;
            for (int32_t s = start[g]; s < start[g] + cnt[g]; s += per) {
                const int32_t nr = std::min(per, start[g] + cnt[g] - s);
                int64_t mx = 0;
                for (int32_t r = 0; r < nr; ++r) mx = std::max(mx, len[(size_t)slot_row[(size_t)(s + r)]]);
                const int64_t nch = (mx + (1 << g) - 1) >> g;
                tiles.push_back({nchunks, s, (int32_t)nch, nr, g});
                nchunks += nch;
            }
        }
        slot = acc;
    }
    if (nchunks > INT32_MAX || (int64_t)tiles.size() > INT32_MAX)
        throw Error{SPTRSV_ERR_OVERFLOW, "device image needs more than INT32_MAX chunks"};

    // ---- layout
    Layout &L = p.layout;
    size_t off = 0;
    L.workspace = off;
    off = align256(off + sizeof(Workspace));
    L.tiles = off;
    off = align256(off + tiles.size() * 16);
    L.rows = off;
    off = align256(off + (size_t)n * 4);
    L.diag = off;
    off = align256(off + (size_t)n * 8);
    L.tcol = off;
    off = align256(off + (size_t)nchunks * 64 * 4);
    L.tval = off;
    off = align256(off + (size_t)nchunks * 64 * 8);
    L.total = off;

    p.image.assign(L.total, 0);
    unsigned char *img = p.image.data();
    int32_t *trow = reinterpret_cast<int32_t *>(img + L.rows);
    double *tdiag = reinterpret_cast<double *>(img + L.diag);
    int32_t *tcol = reinterpret_cast<int32_t *>(img + L.tcol);
    double *tval = reinterpret_cast<double *>(img + L.tval);
    int32_t *tdesc = reinterpret_cast<int32_t *>(img + L.tiles);
    std::fill(tcol, tcol + nchunks * 64, kPad);
    for (size_t t = 0; t < tiles.size(); ++t) {
        const Tile &T = tiles[t];
        tdesc[4 * t + 0] = (int32_t)T.chunk_off;
        tdesc[4 * t + 1] = T.row_off;
        tdesc[4 * t + 2] = T.nch;
        tdesc[4 * t + 3] = (T.nrows << 8) | T.lg;
        const int32_t g = 1 << T.lg;
        for (int32_t r = 0; r < T.nrows; ++r) {
            const int32_t s = T.row_off + r;
            const int32_t i = slot_row[(size_t)s];
            trow[s] = i;
            tdiag[s] = p.lp_val[(size_t)p.lp_ptr[(size_t)i + 1] - 1];
            int64_t t_ = 0;
            auto put = [&](int32_t col, double v) {
                const int64_t idx = (T.chunk_off + (t_ >> T.lg)) * 64 + r * g + (t_ & (g - 1));
                tcol[idx] = col;
                tval[idx] = v;
                ++t_;
            };
            for (int64_t q = p.m_ptr[(size_t)i]; q < p.m_ptr[(size_t)i + 1]; ++q)
                put(~p.m_col[(size_t)q], p.m_val[(size_t)q]);
            for (int64_t q = p.lp_ptr[(size_t)i]; q < p.lp_ptr[(size_t)i + 1] - 1; ++q)
                put(p.lp_col[(size_t)q], -p.lp_val[(size_t)q]);
        }
    }
    p.ntiles = (int64_t)tiles.size();
    p.nchunks = nchunks;
    p.uploaded = false;
}

}  // namespace sptrsv
