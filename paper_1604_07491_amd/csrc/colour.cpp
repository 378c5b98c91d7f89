// Host greedy row colouring for the multicolour NE-SOR sweep.
//
// Row i receives the smallest colour that no earlier row i' < i sharing a column with i
// has received.  Rows of one colour then touch disjoint entries of z, so a colour is
// swept in parallel with no write conflicts, and sweeping colour by colour is a
// sequential NE-SOR sweep in colour-major row order (an SOR sweep in a fixed row order,
// Sec. 3.4).  Each column keeps a bitset of the colours already used in it; a row's
// forbidden set is the union of its columns' bitsets.  The bitset of a column grows
// only as far as the largest colour used in it, so memory stays O(nnz) words.
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace lpk {

int32_t greedy_colour(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
                      int32_t* colour, int32_t* perm) {
    std::vector<std::vector<uint64_t>> used((size_t)n);
    std::vector<uint64_t> forb;
    int32_t ncol = 0;
    for (int64_t i = 0; i < m; ++i) {
        size_t words = 0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) words = std::max(words, used[ci[k]].size());
        forb.assign(words + 1, 0);
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const std::vector<uint64_t>& u = used[ci[k]];
            for (size_t w = 0; w < u.size(); ++w) forb[w] |= u[w];
        }
        size_t w = 0;
        while (forb[w] == ~(uint64_t)0) ++w;
        int b = 0;
        while (forb[w] & ((uint64_t)1 << b)) ++b;
        const int32_t c = (int32_t)(w * 64 + b);
        colour[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            std::vector<uint64_t>& u = used[ci[k]];
            if (u.size() <= w) u.resize(w + 1, 0);
            u[w] |= (uint64_t)1 << b;
        }
    }
    // colour-major order, rows ascending inside a colour (stable counting sort)
    std::vector<int64_t> start((size_t)ncol + 1, 0);
    for (int64_t i = 0; i < m; ++i) start[colour[i] + 1]++;
    for (int32_t c = 0; c < ncol; ++c) start[c + 1] += start[c];
    for (int64_t i = 0; i < m; ++i) perm[start[colour[i]]++] = (int32_t)i;
    return ncol;
}

// lanes per row for rows of mean length len: the next power of two, at most 64; rows of
// at most two entries take one lane each (the sub-group sum would cost more than the row)
int lanes_for(double len) {
    if (len <= 2.0) return 1;
    int g = 1;
    while (g < 64 && g < len) g *= 2;
    return g;
}

}  // namespace lpk
