// Presolve of dependent rows, the part the conclusions name first: rows of A that are
// scalar multiples of an earlier row (exact duplicates included).  Such a row adds
// nothing to A x = b when its right-hand side is the same multiple, and makes the LP
// infeasible otherwise.  Rows are grouped by their column pattern; inside a group, row k
// is a multiple of row i when the ratios a_kj / a_k0 and a_ij / a_i0 agree to tol
// (relative), and then lambda = a_k0 / a_i0.  Host code only.
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <unordered_map>
#include <vector>

namespace lpk {

static uint64_t pattern_hash(const int32_t* ci, int64_t len) {
    uint64_t h = 1469598103934665603ull ^ (uint64_t)len;
    for (int64_t q = 0; q < len; ++q) {
        h ^= (uint64_t)(uint32_t)ci[q];
        h *= 1099511628211ull;
    }
    return h;
}

static bool close(double a, double b, double tol) {
    return std::fabs(a - b) <= tol * std::max(1.0, std::max(std::fabs(a), std::fabs(b)));
}

// keep[i] = 1 for the rows to keep; returns false (message in err) when a dropped row's
// right-hand side contradicts the row it repeats
bool presolve_parallel_rows(int64_t m, const int64_t* rp, const int32_t* ci, const double* val,
                            const double* b, double tol, int32_t* keep, int64_t* m_keep, std::string& err) {
    std::unordered_map<uint64_t, std::vector<int64_t>> groups;
    groups.reserve((size_t)m);
    int64_t kept = 0;
    for (int64_t k = 0; k < m; ++k) {
        const int64_t s = rp[k], len = rp[k + 1] - rp[k];
        keep[k] = 1;
        std::vector<int64_t>& g = groups[pattern_hash(ci + s, len)];
        for (int64_t i : g) {
            const int64_t si = rp[i];
            if (rp[i + 1] - si != len || !std::equal(ci + s, ci + s + len, ci + si)) continue;
            if (val[s] == 0.0 || val[si] == 0.0) continue;   // explicit zeros: no ratio
            bool par = true;
            for (int64_t q = 1; q < len && par; ++q)
                par = close(val[s + q] / val[s], val[si + q] / val[si], tol);
            if (!par) continue;
            const double lambda = val[s] / val[si];
            if (!close(b[k], lambda * b[i], tol)) {
                err = "row " + std::to_string(k) + " repeats row " + std::to_string(i) +
                      " with a different right-hand side: the LP is infeasible";
                return false;
            }
            keep[k] = 0;
            break;
        }
        if (keep[k]) {
            g.push_back(k);
            ++kept;
        }
    }
    *m_keep = kept;
    return true;
}

}  // namespace lpk
