// Bounded variables lo <= x <= hi, brought to the standard form of the introduction
// (min c^T x, A x = b, x >= 0) the way the experiments on typical LPs (Sec. 4.3) do, after
// LIPSOL.  Host code only.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace lpk {

enum BoundKind : int8_t { BK_LOWER = 0, BK_BOX = 1, BK_UPPER = 2, BK_FREE = 3, BK_FIXED = 4 };

// How the original variables sit in the standard form.
struct BoundMap {
    int64_t m0 = 0, n0 = 0;            // original rows and variables
    std::vector<int8_t> kind;          // BoundKind per variable
    std::vector<double> shift;         // l (lower, box, fixed), u (upper); 0 for free
    std::vector<int64_t> col;          // standard-form column of x'_j (x+_j if free); -1 if fixed
    std::vector<int64_t> col2;         // free: column of x-_j; else -1
    std::vector<double> c0;            // the original costs
    double offset = 0.0;               // sum_j c_j shift_j
};

struct StdForm {
    int64_t m = 0, n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> val, b, c;
};

// The reduction; returns false with a message in err on invalid bounds (NaN, l = +inf,
// u = -inf, l > u) or when a row keeps no entry (all of its variables fixed).  The CSR
// input is assumed validated.
bool bounds_to_standard(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                        const double* b, const double* c, const double* lo, const double* hi, StdForm& out,
                        BoundMap& map, std::string& err);

// x (n0) from a standard-form point xs.
void bounds_recover(const BoundMap& map, const double* xs, double* x);

// Presolve: rows that are scalar multiples of an earlier row (keep[i] = 0 for those);
// false with a message when such a row's right-hand side contradicts (infeasible LP).
bool presolve_parallel_rows(int64_t m, const int64_t* rp, const int32_t* ci, const double* val,
                            const double* b, double tol, int32_t* keep, int64_t* m_keep, std::string& err);

// Presolve: every row in the span of the rows before it (to tol) gets keep = 0; false with
// a message when such a row's right-hand side contradicts, or when the elimination would
// store more than max_fill entries.
bool presolve_dependent_rows(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                             const double* b, double tol, int64_t max_fill, int32_t* keep, int64_t* m_keep,
                             std::string& err);
// The same on the dense Gram matrix (m^2 doubles), when the elimination fills.
bool presolve_dependent_rows_gram(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
                                  const double* val, const double* b, double tol, int32_t* keep,
                                  int64_t* m_keep, std::string& err);

}  // namespace lpk
