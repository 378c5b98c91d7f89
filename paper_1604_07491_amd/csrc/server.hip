// Concurrent solves: lp_solve_batch over created problems, and the request-driven server
// (HBM-footprint admission, FIFO with bounded skip, continuous admission as slots free).
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/lpk_server.h"
#include "lpk_impl.h"

using namespace lpk;

extern "C" lp_status lp_solve_batch(lp_problem** problems, int32_t count, int32_t workers,
                                    lp_result* results) {
    if (!problems || !results || count < 0 || workers < 1) return LP_EINVAL;
    if (count == 0) return LP_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LP_EDEVICE;
    std::atomic<int32_t> next{0};
    std::atomic<int> first_err{LP_OK};
    const int32_t nw = workers < count ? workers : count;
    std::vector<std::thread> th;
    for (int32_t w = 0; w < nw; ++w) {
        th.emplace_back([&, dev]() {
            if (hipSetDevice(dev) != hipSuccess) {
                first_err.store(LP_EDEVICE);
                return;
            }
            hipStream_t st = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                first_err.store(LP_EDEVICE);
                return;
            }
            for (;;) {
                const int32_t i = next.fetch_add(1);
                if (i >= count) break;
                lp_problem* p = problems[i];
                hipStream_t keep = p->st;
                p->st = st;
                const lp_status rc = lp_solve(p, &results[i]);
                p->st = keep;
                if (rc != LP_OK && rc != LP_NOT_CONVERGED && rc != LP_DIVERGED) {
                    int expect = LP_OK;
                    first_err.compare_exchange_strong(expect, (int)rc);
                }
            }
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        });
    }
    for (auto& t : th) t.join();
    return (lp_status)first_err.load();
}

namespace {

struct Request {
    uint64_t ticket = 0;
    int64_t m = 0, n = 0, nnz = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> val, b, c;
    uint64_t footprint = 0;
    int32_t skipped = 0;
    double t_submit = 0.0;
};

struct Solution {
    std::vector<double> x, y, s;
};

}  // namespace

struct lp_server {
    lp_server_options opt{};
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<Request>> queue;
    std::deque<lp_completion> done;
    std::map<uint64_t, Solution> solutions;
    uint64_t next_ticket = 1;
    uint64_t in_use = 0;
    int32_t running = 0;
    int64_t outstanding = 0;   // submitted and not completed
    bool stop = false;
    std::vector<std::thread> workers;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

// next request that fits the budget: the head if it fits; otherwise a later one that fits,
// while the head has been overtaken fewer than max_skip times (caller holds the lock)
static std::unique_ptr<Request> take_admissible(lp_server* s) {
    if (s->queue.empty()) return nullptr;
    const uint64_t budget = s->opt.hbm_budget;
    auto fits = [&](const Request& r) { return s->in_use + r.footprint <= budget; };
    if (fits(*s->queue.front())) {
        std::unique_ptr<Request> r = std::move(s->queue.front());
        s->queue.pop_front();
        return r;
    }
    if (s->queue.front()->skipped >= s->opt.max_skip) return nullptr;
    for (size_t i = 1; i < s->queue.size(); ++i) {
        if (fits(*s->queue[i])) {
            s->queue.front()->skipped += 1;
            std::unique_ptr<Request> r = std::move(s->queue[i]);
            s->queue.erase(s->queue.begin() + (long)i);
            return r;
        }
    }
    return nullptr;
}

static void worker_main(lp_server* s) {
    if (hipSetDevice(s->device) != hipSuccess) return;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        std::unique_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                if (s->stop && s->queue.empty()) return true;
                return !s->queue.empty() && (r = take_admissible(s)) != nullptr;
            });
            if (!r) break;   // stopping and nothing queued
            s->in_use += r->footprint;
            s->running += 1;
        }
        lp_completion cpl;
        memset(&cpl, 0, sizeof(cpl));
        cpl.ticket = r->ticket;
        cpl.t_submit = r->t_submit;
        cpl.t_start = s->now();
        cpl.footprint = r->footprint;
        lp_options o = s->opt.solver;
        o.device_io = 0;
        o.stream = st;
        lp_problem* p = nullptr;
        Solution sol;
        lp_status rc = lp_create(r->m, r->n, r->nnz, r->rp.data(), r->ci.data(), r->val.data(),
                                 r->b.data(), r->c.data(), &o, &p);
        if (rc == LP_OK) {
            lp_result res;
            rc = lp_solve(p, &res);
            cpl.iters = res.iters;
            cpl.pobj = res.pobj;
            cpl.dobj = res.dobj;
            cpl.gamma_rel = res.gamma_rel;
            cpl.krylov_iters = res.krylov_iters;
            sol.x.resize((size_t)r->n);
            sol.y.resize((size_t)r->m);
            sol.s.resize((size_t)r->n);
            lp_status rc2 = lp_get_state(p, sol.x.data(), sol.y.data(), sol.s.data(), nullptr);
            if (rc2 != LP_OK && (rc == LP_OK || rc == LP_NOT_CONVERGED)) rc = rc2;
            lp_destroy(p);
        }
        cpl.status = rc;
        cpl.t_done = s->now();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->in_use -= r->footprint;
            s->running -= 1;
            s->outstanding -= 1;
            s->solutions[r->ticket] = std::move(sol);
            s->done.push_back(cpl);
        }
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    (void)hipStreamDestroy(st);
}

extern "C" {

lp_status lp_server_options_default(lp_server_options* o) {
    if (!o) return LP_EINVAL;
    memset(o, 0, sizeof(*o));
    o->slots = 8;
    o->max_skip = 8;
    o->hbm_budget = 0;
    return lp_options_default(&o->solver);
}

lp_status lp_server_create(const lp_server_options* o, lp_server** out) {
    if (!o || !out) return LP_EINVAL;
    *out = nullptr;
    if (o->slots < 1 || o->slots > 256 || o->max_skip < 0) {
        set_error("slots must be in [1, 256] and max_skip >= 0");
        return LP_EINVAL;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        set_error("no HIP device available");
        return LP_EDEVICE;
    }
    lp_server* s = new lp_server();
    s->opt = *o;
    (void)hipGetDevice(&s->device);
    if (s->opt.hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            set_error("hipMemGetInfo failed");
            return LP_EDEVICE;
        }
        s->opt.hbm_budget = (uint64_t)(0.8 * (double)fr);
    }
    s->t0 = std::chrono::steady_clock::now();
    for (int32_t w = 0; w < s->opt.slots; ++w) s->workers.emplace_back(worker_main, s);
    *out = s;
    return LP_OK;
}

lp_status lp_server_submit(lp_server* s, int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                           const int32_t* col_idx, const double* val, const double* b,
                           const double* c, uint64_t* ticket) {
    if (!s || !ticket) return LP_EINVAL;
    if (m < 1 || n < 1 || !row_ptr) return LP_EDIM;
    lp_status rc = validate_inputs(m, n, nnz, row_ptr, col_idx, val, b, c);
    if (rc != LP_OK) return rc;
    std::unique_ptr<Request> r(new Request());
    r->m = m;
    r->n = n;
    r->nnz = nnz;
    r->rp.assign(row_ptr, row_ptr + m + 1);
    r->ci.assign(col_idx, col_idx + nnz);
    r->val.assign(val, val + nnz);
    r->b.assign(b, b + m);
    r->c.assign(c, c + n);
    r->footprint = footprint(m, n, nnz, s->opt.solver);
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = s->now();
    *ticket = r->ticket;
    s->outstanding += 1;
    if (r->footprint > s->opt.hbm_budget) {
        // can never fit: rejected at once
        lp_completion cpl;
        memset(&cpl, 0, sizeof(cpl));
        cpl.ticket = r->ticket;
        cpl.status = LP_ETOOBIG;
        cpl.t_submit = cpl.t_start = cpl.t_done = r->t_submit;
        cpl.footprint = r->footprint;
        s->done.push_back(cpl);
        s->outstanding -= 1;
        s->cv_done.notify_all();
        return LP_OK;
    }
    s->queue.push_back(std::move(r));
    s->cv_work.notify_all();
    return LP_OK;
}

lp_status lp_server_poll(lp_server* s, lp_completion* out, int32_t cap, int32_t* n_out) {
    if (!s || !n_out || (cap > 0 && !out)) return LP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = k;
    return LP_OK;
}

lp_status lp_server_wait(lp_server* s, int32_t count, double timeout_s) {
    if (!s) return LP_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] {
        return (int64_t)s->done.size() >= count || s->outstanding == 0;
    });
    return ok ? LP_OK : LP_NOT_CONVERGED;
}

lp_status lp_server_result(lp_server* s, uint64_t ticket, double* x, double* y, double* s_out) {
    if (!s) return LP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->solutions.find(ticket);
    if (it == s->solutions.end()) {
        set_error("unknown or unfinished ticket");
        return LP_EINVAL;
    }
    const Solution& sol = it->second;
    if (x && !sol.x.empty()) memcpy(x, sol.x.data(), sizeof(double) * sol.x.size());
    if (y && !sol.y.empty()) memcpy(y, sol.y.data(), sizeof(double) * sol.y.size());
    if (s_out && !sol.s.empty()) memcpy(s_out, sol.s.data(), sizeof(double) * sol.s.size());
    s->solutions.erase(it);
    return LP_OK;
}

lp_status lp_server_stats(lp_server* s, uint64_t* bytes_in_use, int32_t* queued, int32_t* running) {
    if (!s) return LP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (bytes_in_use) *bytes_in_use = s->in_use;
    if (queued) *queued = (int32_t)s->queue.size();
    if (running) *running = s->running;
    return LP_OK;
}

lp_status lp_server_destroy(lp_server* s) {
    if (!s) return LP_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    delete s;
    return LP_OK;
}

}  // extern "C"
