// Bounded variables: the reduction to the standard form.  Per variable x_j:
//   lower  (l finite, u = +inf):  x_j = l_j + x'_j
//   box    (l < u, both finite):  x_j = l_j + x'_j, and a new row x'_j + w_j = u_j - l_j
//   upper  (l = -inf, u finite):  x_j = u_j - x'_j (column and cost negated)
//   free   (both infinite):       x_j = x+_j - x-_j (an extra column -a_j with cost -c_j)
//   fixed  (l = u):               x_j = l_j, the column is removed
// Standard-form columns: the kept variables in their order, then the negative parts of
// the free variables, then the box slacks; rows: the original rows, then the box rows.
// Inside a row the kept columns come in the original order and the negative parts after
// them, so column indices stay strictly increasing.  b' = b - A s with s the shifts,
// accumulated in the row's CSR order.
#include "bounds.h"

#include <cmath>

namespace lpk {

bool bounds_to_standard(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                        const double* b, const double* c, const double* lo, const double* hi, StdForm& out,
                        BoundMap& map, std::string& err) {
    map = BoundMap{};
    map.m0 = m;
    map.n0 = n;
    map.kind.resize((size_t)n);
    map.shift.assign((size_t)n, 0.0);
    map.col.assign((size_t)n, -1);
    map.col2.assign((size_t)n, -1);
    map.c0.assign(c, c + n);
    int64_t nkept = 0, nfree = 0, nbox = 0;
    for (int64_t j = 0; j < n; ++j) {
        const double l = lo[j], u = hi[j];
        if (std::isnan(l) || std::isnan(u) || l == INFINITY || u == -INFINITY || l > u) {
            err = "invalid bounds for variable " + std::to_string(j);
            return false;
        }
        const bool lf = std::isfinite(l), uf = std::isfinite(u);
        BoundKind k;
        if (lf && uf) k = l == u ? BK_FIXED : BK_BOX;
        else if (lf) k = BK_LOWER;
        else if (uf) k = BK_UPPER;
        else k = BK_FREE;
        map.kind[(size_t)j] = k;
        if (k == BK_LOWER || k == BK_BOX || k == BK_FIXED) map.shift[(size_t)j] = l;
        if (k == BK_UPPER) map.shift[(size_t)j] = u;
        if (k != BK_FIXED) map.col[(size_t)j] = nkept++;
        nfree += k == BK_FREE;
        nbox += k == BK_BOX;
    }
    int64_t t = 0;
    for (int64_t j = 0; j < n; ++j)
        if (map.kind[(size_t)j] == BK_FREE) map.col2[(size_t)j] = nkept + t++;
    double off = 0.0;
    for (int64_t j = 0; j < n; ++j) off += c[j] * map.shift[(size_t)j];
    map.offset = off;

    out = StdForm{};
    out.m = m + nbox;
    out.n = nkept + nfree + nbox;
    out.rp.reserve((size_t)out.m + 1);
    out.rp.push_back(0);
    out.b.resize((size_t)out.m);
    out.c.assign((size_t)out.n, 0.0);
    for (int64_t i = 0; i < m; ++i) {
        double bi = b[i];
        const size_t before = out.ci.size();
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int32_t j = ci[q];
            const int8_t k = map.kind[(size_t)j];
            bi -= val[q] * map.shift[(size_t)j];
            if (k == BK_FIXED) continue;
            out.ci.push_back((int32_t)map.col[(size_t)j]);
            out.val.push_back(k == BK_UPPER ? -val[q] : val[q]);
        }
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int32_t j = ci[q];
            if (map.kind[(size_t)j] != BK_FREE) continue;
            out.ci.push_back((int32_t)map.col2[(size_t)j]);
            out.val.push_back(-val[q]);
        }
        if (out.ci.size() == before) {
            err = "row " + std::to_string(i) + " has only fixed variables";
            return false;
        }
        out.b[(size_t)i] = bi;
        out.rp.push_back((int64_t)out.ci.size());
    }
    t = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (map.kind[(size_t)j] != BK_BOX) continue;
        out.ci.push_back((int32_t)map.col[(size_t)j]);
        out.val.push_back(1.0);
        out.ci.push_back((int32_t)(nkept + nfree + t));
        out.val.push_back(1.0);
        out.b[(size_t)(m + t)] = hi[j] - lo[j];
        out.rp.push_back((int64_t)out.ci.size());
        ++t;
    }
    for (int64_t j = 0; j < n; ++j) {
        const int8_t k = map.kind[(size_t)j];
        if (k == BK_FIXED) continue;
        out.c[(size_t)map.col[(size_t)j]] = k == BK_UPPER ? -c[j] : c[j];
        if (k == BK_FREE) out.c[(size_t)map.col2[(size_t)j]] = -c[j];
    }
    return true;
}

void bounds_recover(const BoundMap& map, const double* xs, double* x) {
    for (int64_t j = 0; j < map.n0; ++j) {
        const size_t u = (size_t)j;
        switch (map.kind[u]) {
            case BK_LOWER:
            case BK_BOX: x[j] = map.shift[u] + xs[map.col[u]]; break;
            case BK_UPPER: x[j] = map.shift[u] - xs[map.col[u]]; break;
            case BK_FREE: x[j] = xs[map.col[u]] - xs[map.col2[u]]; break;
            default: x[j] = map.shift[u]; break;
        }
    }
}

}  // namespace lpk
