// Host-side planning of collapsed rows (no device code; also compiled on its own by a
// CPU test).
//
// Row i of a view has imaginary part cy0 + ((i + 0.5) - m/2) dy: one rounded product
// and one rounded sum, in the kernels' own order.  Rows with the same c have the same
// counts: when dy is below the spacing of doubles near cy0, neighbouring rows round to
// the same value.  Conjugate points have the same counts too, bit for bit (rounding to
// nearest is symmetric in sign, so the orbit of the conjugate is the conjugate orbit),
// so with `mirror` rows whose imaginary parts differ only in sign are merged as well.
// The plan renders one row per distinct key, in order of first occurrence, each into
// the image row where its key first occurs; every other row then copies the row where
// its key first occurs.  Those source rows are never copy destinations, so the copies
// can run in any order, in place.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>

namespace mandel {

struct RowCollapse {
    std::vector<double> cy;      // imaginary part of each rendered row
    std::vector<int32_t> first;  // image row that each rendered row is written to (ascending)
    std::vector<int32_t> pairs;  // (dst, src) image rows, src a first row, dst ascending
};

// Fills `rc` for a view of m rows; rc.cy.size() == m when every row is distinct (and
// then rc.pairs is empty).  May throw std::bad_alloc.
inline void plan_row_collapse(double cy0, double dy, int32_t m, bool mirror, RowCollapse &rc)
{
    rc.cy.clear();
    rc.first.clear();
    rc.pairs.clear();
    std::vector<int32_t> key_of((size_t)(m > 0 ? m : 0)); // row -> rendered row
    std::unordered_map<uint64_t, int32_t> seen;
    for (int32_t i = 0; i < m; ++i) {
        const double off = ((double)i + 0.5) - 0.5 * (double)m;
        const double py = off * dy;
        const double cy = cy0 + py;
        const double key = mirror ? std::fabs(cy) : cy + 0.0; // + 0.0: -0 and +0 alike
        uint64_t bits;
        std::memcpy(&bits, &key, sizeof bits);
        auto it = seen.find(bits);
        if (it == seen.end()) {
            it = seen.emplace(bits, (int32_t)rc.cy.size()).first;
            rc.cy.push_back(cy);
            rc.first.push_back(i);
        }
        key_of[(size_t)i] = it->second;
    }
    for (int32_t i = 0; i < m; ++i) {
        const int32_t src = rc.first[(size_t)key_of[(size_t)i]];
        if (src != i) {
            rc.pairs.push_back(i);
            rc.pairs.push_back(src);
        }
    }
}

} // namespace mandel
