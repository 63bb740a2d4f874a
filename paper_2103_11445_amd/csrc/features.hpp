// features.hpp -- the shape of a group of rows (an executed level of a
// rewritten schedule, or a candidate stage of the rewrite) as the six inputs
// of the learned cost model.  The same function serves the training labels
// (per executed level of a measured solve) and the LEARNED policy (per
// candidate stage), so the model sees the same quantities in both.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

namespace sptrsv {

constexpr int kFeatures = 6;

struct GroupShape {
    int64_t rows = 0;    // rows in the group
    int64_t terms = 0;   // their entries after rewriting: x-terms + b-terms + diagonal
    int64_t orig = 0;    // their entries in L (diagonal included)
    int64_t maxlen = 0;  // largest entry count of one row after rewriting
    int64_t span = 1;    // original levels the group merges
};

// Inputs, each of order one: log2 rows / 16, log2 entries / 24, entries added
// by rewriting per original entry (capped at 16) / 4, log2 longest row / 8,
// entries per row (capped at 256) / 16, log2 merged levels / 8.
inline void group_features(const GroupShape &g, float *f) {
    const double rows = (double)std::max<int64_t>(g.rows, 1);
    f[0] = (float)(std::log2(1.0 + (double)g.rows) / 16.0);
    f[1] = (float)(std::log2(1.0 + (double)g.terms) / 24.0);
    f[2] = (float)(std::min(16.0, (double)std::max<int64_t>(g.terms - g.orig, 0) /
                                      (double)std::max<int64_t>(g.orig, 1)) / 4.0);
    f[3] = (float)(std::log2(1.0 + (double)g.maxlen) / 8.0);
    f[4] = (float)(std::min(256.0, (double)g.terms / rows) / 16.0);
    f[5] = (float)(std::log2((double)std::max<int64_t>(g.span, 1)) / 8.0);
}

}  // namespace sptrsv
