// Presolve of dependent rows (the conclusions name it as the preprocessing to add).  First
// the quick pass: rows of A that are scalar multiples of an earlier row (exact duplicates
// included).  Such a row adds
// nothing to A x = b when its right-hand side is the same multiple, and makes the LP
// infeasible otherwise.  Rows are grouped by their column pattern; inside a group, row k
// is a multiple of row i when the ratios a_kj / a_k0 and a_ij / a_i0 agree to tol
// (relative), and then lambda = a_k0 / a_i0.  Host code only.
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <functional>
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

namespace lpk {

// ------------------------------------------------------------------------------------
// General dependent rows.  keep[k] = 1 exactly when row k is not in the span of rows
// 0..k-1 (to tol): the first row basis in the given order.  Rows are taken one at a time
// and reduced against a growing set of basis rows by sparse elimination.  Each basis row
// has a pivot column that no later basis row contains (every row entering the basis was
// reduced against all earlier ones), so eliminating the pivots of a row in the order the
// basis rows entered never brings back an eliminated pivot, and the reduction ends.  A row
// whose remainder is at most tol times its largest entry is dependent: its right-hand side,
// reduced alongside, must vanish to tol relative to the terms that formed it, else the LP
// is infeasible.  Otherwise its pivot is chosen among the remainder's entries within a
// factor 10 of the largest (threshold pivoting), preferring the column that the fewest rows
// still to come contain (few later rows need this basis row), then the column whose later
// rows have been given the fewest pivots so far (the pivots spread over the later rows).
// Elimination fills: on random sparse rows (expanders) and on incidence matrices the
// reduced rows grow towards dense.  Fill is capped at max_fill stored entries; past it the
// caller falls back to presolve_dependent_rows_gram.
// Fill is capped at max_fill stored entries (then false, with the message in err).
bool presolve_dependent_rows(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                             const double* b, double tol, int64_t max_fill, int32_t* keep, int64_t* m_keep,
                             std::string& err) {
    // columns' counts of rows not yet taken
    std::vector<int32_t> rest((size_t)n, 0);
    for (int64_t q = 0; q < rp[m]; ++q) rest[(size_t)ci[q]] += 1;
    // the rows of each column, ascending (CSC pattern), and the pivots given to each row
    std::vector<int64_t> cp((size_t)n + 1, 0);
    for (int64_t q = 0; q < rp[m]; ++q) cp[(size_t)ci[q] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) cp[(size_t)j + 1] += cp[(size_t)j];
    std::vector<int32_t> crow((size_t)rp[m]);
    {
        std::vector<int64_t> fillp(cp.begin(), cp.end() - 1);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t q = rp[i]; q < rp[i + 1]; ++q) crow[(size_t)fillp[(size_t)ci[q]]++] = (int32_t)i;
    }
    std::vector<int32_t> load((size_t)m, 0);

    auto later_load = [&](int32_t j, int64_t k) {
        int64_t sum = 0;
        for (int64_t q = cp[(size_t)j + 1] - 1; q >= cp[(size_t)j] && crow[(size_t)q] > k; --q)
            sum += load[(size_t)crow[(size_t)q]];
        return sum;
    };
    std::vector<int32_t> piv_of((size_t)n, -1);        // basis row whose pivot is this column
    std::vector<int64_t> bs;                           // basis rows: start in bcol / bval
    std::vector<int32_t> bcol;
    std::vector<double> bval, bpiv, bb;                // pivot value and right-hand side
    bs.push_back(0);
    std::vector<double> acc((size_t)n, 0.0);           // the row being reduced, scattered
    std::vector<char> on((size_t)n, 0);
    std::vector<int32_t> nz;                           // its nonzero columns
    std::vector<int32_t> heap;                         // basis rows to eliminate, earliest first
    int64_t kept = 0;
    for (int64_t k = 0; k < m; ++k) {
        nz.clear();
        heap.clear();
        double amax = 0.0;
        for (int64_t q = rp[k]; q < rp[k + 1]; ++q) {
            const int32_t j = ci[q];
            rest[(size_t)j] -= 1;
            if (!on[(size_t)j]) {
                on[(size_t)j] = 1;
                nz.push_back(j);
            }
            acc[(size_t)j] += val[q];
            amax = std::max(amax, std::fabs(val[q]));
        }
        for (int32_t j : nz)
            if (piv_of[(size_t)j] >= 0) heap.push_back(piv_of[(size_t)j]);
        std::make_heap(heap.begin(), heap.end(), std::greater<int32_t>());
        double rb = b[k], bscale = std::fabs(b[k]);
        while (!heap.empty()) {
            std::pop_heap(heap.begin(), heap.end(), std::greater<int32_t>());
            const int32_t r = heap.back();
            heap.pop_back();
            const int32_t pc = bcol[(size_t)bs[(size_t)r]];   // the pivot is stored first
            const double v = acc[(size_t)pc];
            if (v == 0.0) continue;
            const double f = v / bpiv[(size_t)r];
            for (int64_t q = bs[(size_t)r]; q < bs[(size_t)r + 1]; ++q) {
                const int32_t j = bcol[(size_t)q];
                if (!on[(size_t)j]) {
                    on[(size_t)j] = 1;
                    nz.push_back(j);
                    if (piv_of[(size_t)j] >= 0 && piv_of[(size_t)j] != r) {
                        heap.push_back(piv_of[(size_t)j]);
                        std::push_heap(heap.begin(), heap.end(), std::greater<int32_t>());
                    }
                }
                acc[(size_t)j] -= f * bval[(size_t)q];
            }
            acc[(size_t)pc] = 0.0;
            rb -= f * bb[(size_t)r];
            bscale += std::fabs(f * bb[(size_t)r]);
        }
        // the remainder: dependent, or a new basis row
        double rmax = 0.0;
        for (int32_t j : nz) rmax = std::max(rmax, std::fabs(acc[(size_t)j]));
        if (rmax <= tol * amax) {
            if (std::fabs(rb) > tol * std::max(1.0, bscale)) {
                err = "row " + std::to_string(k) +
                      " is a combination of earlier rows with a different right-hand side: the LP is infeasible";
                for (int32_t j : nz) {
                    acc[(size_t)j] = 0.0;
                    on[(size_t)j] = 0;
                }
                return false;
            }
            keep[k] = 0;
        } else {
            int32_t pc = -1;
            int64_t pc_load = 0;
            for (int32_t j : nz) {
                const double a = std::fabs(acc[(size_t)j]);
                if (a < 0.1 * rmax || a <= tol * amax) continue;
                if (pc >= 0 && rest[(size_t)j] > rest[(size_t)pc]) continue;
                const int64_t ld = rest[(size_t)j] > 0 ? later_load(j, k) : 0;
                if (pc < 0 || rest[(size_t)j] < rest[(size_t)pc] || ld < pc_load ||
                    (ld == pc_load && a > std::fabs(acc[(size_t)pc]))) {
                    pc = j;
                    pc_load = ld;
                }
            }
            for (int64_t q = cp[(size_t)pc + 1] - 1; q >= cp[(size_t)pc] && crow[(size_t)q] > k; --q)
                load[(size_t)crow[(size_t)q]] += 1;
            const int32_t r = (int32_t)(bs.size() - 1);
            piv_of[(size_t)pc] = r;
            bcol.push_back(pc);
            bval.push_back(acc[(size_t)pc]);
            for (int32_t j : nz)
                if (j != pc && std::fabs(acc[(size_t)j]) > tol * amax) {
                    bcol.push_back(j);
                    bval.push_back(acc[(size_t)j]);
                }
            bpiv.push_back(acc[(size_t)pc]);
            bb.push_back(rb);
            bs.push_back((int64_t)bcol.size());
            keep[k] = 1;
            ++kept;
            if ((int64_t)bcol.size() > max_fill) {
                err = "the dependency search exceeded its fill limit of " + std::to_string(max_fill) + " entries";
                for (int32_t j : nz) {
                    acc[(size_t)j] = 0.0;
                    on[(size_t)j] = 0;
                }
                return false;
            }
        }
        for (int32_t j : nz) {
            acc[(size_t)j] = 0.0;
            on[(size_t)j] = 0;
        }
    }
    *m_keep = kept;
    return true;
}

}  // namespace lpk

namespace lpk {

// ------------------------------------------------------------------------------------
// The same decision on the Gram matrix G = A A^T (dense, m x m), for problems whose
// elimination fills past its cap.  Rows are taken in order; a Cholesky factor is built over
// the kept rows only: for row k, y = L^-1 G[K, k] over the kept rows K before it, and the
// squared distance of row k from their span is d = G_kk - ||y||^2.  Squared norms resolve
// that distance only to about sqrt(eps) of the row's norm, so d serves as a screen: a row
// with d <= 1e-6 G_kk (within an angle of about 1e-3 of the span) gets its combination
// lambda = L^-T y, refined once against the explicit residual r = A_k - lambda^T A_K, and is
// dependent when max|r| <= tol max|A_k| (the elimination's test).  Its right-hand side must
// then equal lambda^T b_K to tol relative to the terms.  O(m^3 / 3) time, 8 m^2 bytes.
bool presolve_dependent_rows_gram(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
                                  const double* val, const double* b, double tol, int32_t* keep,
                                  int64_t* m_keep, std::string& err) {
    std::vector<double> G((size_t)m * (size_t)m, 0.0);   // lower triangle, row-major
    std::vector<double> dense((size_t)n, 0.0);
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) dense[(size_t)ci[q]] += val[q];
        for (int64_t j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int64_t q = rp[j]; q < rp[j + 1]; ++q) s += val[q] * dense[(size_t)ci[q]];
            G[(size_t)i * m + j] = s;
        }
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) dense[(size_t)ci[q]] = 0.0;
    }
    auto gram = [&](int64_t i, int64_t j) { return i >= j ? G[(size_t)i * m + j] : G[(size_t)j * m + i]; };
    // L over the kept rows: row t of L (t-th kept row) holds t + 1 entries, packed
    std::vector<int64_t> kept_rows;
    std::vector<double> L;
    std::vector<int64_t> lstart;
    std::vector<double> y;
    for (int64_t k = 0; k < m; ++k) {
        const size_t r = kept_rows.size();
        y.assign(r, 0.0);
        double d = G[(size_t)k * m + k];
        for (size_t t = 0; t < r; ++t) {
            const double* Lt = &L[(size_t)lstart[t]];
            double s = gram(k, kept_rows[t]);
            for (size_t u = 0; u < t; ++u) s -= Lt[u] * y[u];
            y[t] = s / Lt[t];
            d -= y[t] * y[t];
        }
        const double gkk = G[(size_t)k * m + k];
        bool dependent = false;
        std::vector<double> lam;
        if (d <= 1e-6 * gkk) {
            // lambda = G_KK^-1 G[K, k] = L^-T y, refined once: lambda += G_KK^-1 A_K r
            auto solve_lt = [&](std::vector<double>& v) {   // v <- L^-T v
                for (size_t t = r; t-- > 0;) {
                    v[t] /= L[(size_t)lstart[t] + t];
                    const double vt = v[t];
                    const double* Lt = &L[(size_t)lstart[t]];
                    for (size_t u = 0; u < t; ++u) v[u] -= Lt[u] * vt;
                }
            };
            auto solve_l = [&](std::vector<double>& v) {    // v <- L^-1 v
                for (size_t t = 0; t < r; ++t) {
                    const double* Lt = &L[(size_t)lstart[t]];
                    double s = v[t];
                    for (size_t u = 0; u < t; ++u) s -= Lt[u] * v[u];
                    v[t] = s / Lt[t];
                }
            };
            auto residual = [&]() {   // dense = A_k - lambda^T A_K; returns max|A_k|
                double amax = 0.0;
                for (int64_t q = rp[k]; q < rp[k + 1]; ++q) {
                    dense[(size_t)ci[q]] += val[q];
                    amax = std::max(amax, std::fabs(val[q]));
                }
                for (size_t t = 0; t < r; ++t)
                    for (int64_t q = rp[kept_rows[t]]; q < rp[kept_rows[t] + 1]; ++q)
                        dense[(size_t)ci[q]] -= lam[t] * val[q];
                return amax;
            };
            auto clear_rows = [&]() {
                for (int64_t q = rp[k]; q < rp[k + 1]; ++q) dense[(size_t)ci[q]] = 0.0;
                for (size_t t = 0; t < r; ++t)
                    for (int64_t q = rp[kept_rows[t]]; q < rp[kept_rows[t] + 1]; ++q) dense[(size_t)ci[q]] = 0.0;
            };
            lam = y;
            solve_lt(lam);
            residual();
            std::vector<double> g(r, 0.0);
            for (size_t t = 0; t < r; ++t) {
                double s = 0.0;
                for (int64_t q = rp[kept_rows[t]]; q < rp[kept_rows[t] + 1]; ++q) s += val[q] * dense[(size_t)ci[q]];
                g[t] = s;
            }
            clear_rows();
            solve_l(g);
            solve_lt(g);
            for (size_t t = 0; t < r; ++t) lam[t] += g[t];
            const double amax = residual();
            double rmax = 0.0;
            for (int64_t q = rp[k]; q < rp[k + 1]; ++q) rmax = std::max(rmax, std::fabs(dense[(size_t)ci[q]]));
            for (size_t t = 0; t < r; ++t)
                for (int64_t q = rp[kept_rows[t]]; q < rp[kept_rows[t] + 1]; ++q)
                    rmax = std::max(rmax, std::fabs(dense[(size_t)ci[q]]));
            clear_rows();
            dependent = rmax <= tol * amax;
        }
        if (dependent) {
            double rb = b[k], sc = std::fabs(b[k]);
            for (size_t t = 0; t < r; ++t) {
                rb -= lam[t] * b[kept_rows[t]];
                sc += std::fabs(lam[t] * b[kept_rows[t]]);
            }
            if (std::fabs(rb) > tol * std::max(1.0, sc)) {
                err = "row " + std::to_string(k) +
                      " is a combination of earlier rows with a different right-hand side: the LP is infeasible";
                return false;
            }
            keep[k] = 0;
            continue;
        }
        keep[k] = 1;
        lstart.push_back((int64_t)L.size());
        for (size_t t = 0; t < r; ++t) L.push_back(y[t]);
        L.push_back(std::sqrt(d));
        kept_rows.push_back(k);
    }
    *m_keep = (int64_t)kept_rows.size();
    return true;
}

}  // namespace lpk
