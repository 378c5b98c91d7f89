// Per-launch kernel timing with HIP events on a batch's stream.  A launch of an
// enabled class is bracketed by two events; statistics are folded in when they are read
// (or when the record list grows long), keeping only launches that did work: loop
// kernels enqueued after a solve had converged return at once and are discarded by
// their iteration index.
#include <string.h>

#include "lpk_impl.h"

namespace lpk {

static const char* kClassName[LP_K_COUNT] = {"sweep", "spmv_csr", "spmv_csc", "gs_dots", "gs_update", "gram",
                                              "cg_vec"};

static hipEvent_t take_event(Batch* p) {
    if (!p->prof_pool.empty()) {
        hipEvent_t e = p->prof_pool.back();
        p->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

Prof::Prof(Batch* pp, int cls, int64_t iter, double bytes, double flops) : B(pp) {
    Batch* p = B;
    if (p->count_launch && cls == p->count_cls) {
        *p->count_launch += 1;
        *p->count_bytes += bytes;
        *p->count_flops += flops;
    }
    if (!(p->prof_mask & (1u << cls))) return;
    ProfRec r;
    r.cls = cls;
    r.solve = p->cur_solve;
    r.iter = iter;
    r.bytes = bytes;
    r.flops = flops;
    r.a = take_event(p);
    r.b = take_event(p);
    if (!r.a || !r.b) return;
    (void)hipEventRecord(r.a, p->L.st);
    idx = (int)p->prof_recs.size();
    p->prof_recs.push_back(r);
}

Prof::~Prof() {
    if (idx >= 0) (void)hipEventRecord(B->prof_recs[idx].b, B->L.st);
}

lp_status prof_collect(Batch& B) {
    Batch* p = &B;
    if (p->prof_recs.empty()) return LP_OK;
    LPK_HIP(hipStreamSynchronize(p->st));
    for (ProfRec& r : p->prof_recs) {
        bool keep = true;
        if (r.iter >= 0) {
            const int64_t s = r.solve;
            keep = s >= 0 && s < (int64_t)p->solve_iters.size() && r.iter < p->solve_iters[s];
        }
        if (keep) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                p->prof_launch[r.cls] += 1;
                p->prof_ms[r.cls] += ms;
                p->prof_bytes[r.cls] += r.bytes;
                p->prof_flops[r.cls] += r.flops;
            }
        }
        p->prof_pool.push_back(r.a);
        p->prof_pool.push_back(r.b);
    }
    p->prof_recs.clear();
    return LP_OK;
}

void prof_release(Batch& B) {
    Batch* p = &B;
    if (p->st) (void)hipStreamSynchronize(p->st);
    for (ProfRec& r : p->prof_recs) {
        p->prof_pool.push_back(r.a);
        p->prof_pool.push_back(r.b);
    }
    p->prof_recs.clear();
    for (hipEvent_t e : p->prof_pool)
        if (e) (void)hipEventDestroy(e);
    p->prof_pool.clear();
}

}  // namespace lpk

using namespace lpk;

extern "C" {

lp_status lp_profile(lp_problem* pr, uint32_t mask) {
    if (!pr) return LP_EINVAL;
    Batch* p = nullptr;
    lp_status rc = solo_batch(pr, &p);
    if (rc != LP_OK) return rc;
    rc = prof_collect(*p);
    if (rc != LP_OK) return rc;
    p->prof_mask = mask;
    for (int c = 0; c < LP_K_COUNT; ++c) {
        p->prof_launch[c] = 0;
        p->prof_ms[c] = 0.0;
        p->prof_bytes[c] = 0.0;
        p->prof_flops[c] = 0.0;
    }
    return LP_OK;
}

lp_status lp_profile_read(lp_problem* pr, lp_kernel_stat* st, int32_t cap, int32_t* n_out) {
    if (!pr || !n_out) return LP_EINVAL;
    Batch* p = nullptr;
    lp_status rc = solo_batch(pr, &p);
    if (rc != LP_OK) return rc;
    rc = prof_collect(*p);
    if (rc != LP_OK) return rc;
    *n_out = LP_K_COUNT;
    for (int c = 0; c < LP_K_COUNT && st && c < cap; ++c) {
        memset(&st[c], 0, sizeof(st[c]));
        st[c].cls = c;
        st[c].launches = p->prof_launch[c];
        st[c].ms_total = p->prof_ms[c];
        st[c].bytes_total = p->prof_bytes[c];
        st[c].flops_total = p->prof_flops[c];
        strncpy(st[c].name, kClassName[c], sizeof(st[c].name) - 1);
    }
    return LP_OK;
}

}  // extern "C"
