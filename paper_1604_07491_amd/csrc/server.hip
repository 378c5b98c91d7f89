// Many LPs on one MI355X: lp_solve_batch over created problems, and the request-driven
// server.  Both run the batched engine: up to `width` LPs share every launch, each in its
// own phase of its own interior-point iteration.  A finished LP leaves the batch after any
// round and a waiting one joins at once, so the batch stays full while work remains.
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

// one group of compatible problems through one batch of width `width`
static lp_status solve_group(lp_problem** problems, const std::vector<int32_t>& idx, int32_t width,
                             lp_result* results) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return LP_EDEVICE;
    for (int32_t i : idx)
        if (hipStreamSynchronize(problems[i]->st) != hipSuccess) {
            (void)hipStreamDestroy(st);
            return LP_EDEVICE;
        }
    Batch B;
    lp_status rc = B.init(std::min<int32_t>(width, (int32_t)idx.size()), st, true);
    if (rc != LP_OK) return rc;
    Engine E;
    E.attach(&B);
    std::vector<int32_t> who((size_t)B.cap, -1);
    size_t next = 0;
    auto refill = [&]() {
        while (next < idx.size()) {
            const int slot = B.free_slot();
            if (slot < 0) break;
            const int32_t i = idx[next++];
            lp_problem* p = problems[i];
            bool from_point = false;
            if (p->opt.start != 0) {
                if (!p->have_point) {
                    memset(&results[i], 0, sizeof(lp_result));
                    results[i].status = LP_EINVAL;
                    continue;
                }
                p->ist.eps_in = p->opt.eps_in0;
                p->ist.k = 0;
                p->ist.fail_prev = 0;
                from_point = true;
            }
            p->log.clear();
            p->krylov_total = 0;
            who[E.join(p, from_point, p->opt.ipm_max_iter)] = i;
        }
    };
    refill();
    while (E.any_live()) {
        rc = E.round();
        if (rc != LP_OK) break;
        for (int s = 0; s < B.cap; ++s) {
            if (E.mem[s].state != Engine::DONE) continue;
            fill_result(E.mem[s], &results[who[s]]);
            E.leave(s);
            who[s] = -1;
        }
        refill();
    }
    (void)hipStreamSynchronize(st);
    return rc;
}

extern "C" lp_status lp_solve_batch(lp_problem** problems, int32_t count, int32_t width,
                                    lp_result* results) {
    if (!problems || !results || count < 0 || width < 1) {
        set_error("NULL arrays, count < 0 or width < 1");
        return LP_EINVAL;
    }
    for (int32_t i = 0; i < count; ++i)
        if (!problems[i]) {
            set_error("NULL problem");
            return LP_EINVAL;
        }
    // groups of problems that can share launches, in order of first appearance
    std::vector<std::vector<int32_t>> groups;
    for (int32_t i = 0; i < count; ++i) {
        bool placed = false;
        for (auto& g : groups)
            if (batch_compatible(problems[g[0]], problems[i])) {
                g.push_back(i);
                placed = true;
                break;
            }
        if (!placed) groups.push_back({i});
    }
    lp_status first = LP_OK;
    for (auto& g : groups) {
        const lp_status rc = solve_group(problems, g, width, results);
        if (rc != LP_OK && first == LP_OK) first = rc;
    }
    return first;
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

// a created problem waiting to join the batch
struct Ready {
    std::unique_ptr<Request> req;
    lp_problem* p = nullptr;
};

}  // namespace

struct lp_server {
    lp_server_options opt{};
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_ready, cv_done;
    std::deque<std::unique_ptr<Request>> queue;   // submitted, not admitted
    std::deque<Ready> ready;                      // admitted and created, not joined
    std::deque<std::pair<lp_problem*, uint64_t>> retire;   // finished: destroy, then release
    bool engine_done = false;
    int32_t preparing = 0;
    std::deque<lp_completion> done;
    std::map<uint64_t, Solution> solutions;
    uint64_t next_ticket = 1;
    uint64_t in_use = 0;
    int32_t running = 0;
    int64_t outstanding = 0;   // submitted and not completed
    bool stop = false;
    std::thread prep, engine;

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

// publish a completion; fp is released from the budget now, or (fp = 0 here) by the
// preparer once it has destroyed the problem
static void complete(lp_server* s, lp_completion cpl, uint64_t fp, Solution sol, bool was_running) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->in_use -= fp;
        if (was_running) s->running -= 1;
        s->outstanding -= 1;
        s->solutions[cpl.ticket] = std::move(sol);
        s->done.push_back(cpl);
    }
    s->cv_work.notify_all();
    s->cv_ready.notify_all();
    s->cv_done.notify_all();
}

// admission and host-side set-up (validation was done at submit; colouring, CSC, copies)
static void prep_main(lp_server* s) {
    if (hipSetDevice(s->device) != hipSuccess) return;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        std::unique_ptr<Request> r;
        std::deque<std::pair<lp_problem*, uint64_t>> retire;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                if (!s->retire.empty()) return true;
                if (s->stop && s->queue.empty() && s->engine_done) return true;
                return !s->queue.empty() && (r = take_admissible(s)) != nullptr;
            });
            retire.swap(s->retire);
            if (r) {
                s->in_use += r->footprint;
                s->preparing += 1;
            }
        }
        // Finished problems are destroyed here, not on the engine thread: freeing device
        // memory waits for the work queued on the device, and the engine keeps the other
        // lanes' rounds queued meanwhile.  Their memory returns to the budget afterwards.
        if (!retire.empty()) {
            uint64_t freed = 0;
            for (auto& q : retire) {
                lp_destroy(q.first);
                freed += q.second;
            }
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->in_use -= freed;
            }
            s->cv_work.notify_all();
        }
        if (!r) {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->retire.empty() && s->stop && s->queue.empty() && s->engine_done) break;
            continue;
        }
        lp_options o = s->opt.solver;
        o.device_io = 0;
        o.stream = st;
        lp_problem* p = nullptr;
        const lp_status rc = lp_create(r->m, r->n, r->nnz, r->rp.data(), r->ci.data(), r->val.data(),
                                       r->b.data(), r->c.data(), &o, &p);
        if (rc != LP_OK) {
            lp_completion cpl;
            memset(&cpl, 0, sizeof(cpl));
            cpl.ticket = r->ticket;
            cpl.status = rc;
            cpl.t_submit = r->t_submit;
            cpl.t_start = cpl.t_done = s->now();
            cpl.footprint = r->footprint;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->preparing -= 1;
            }
            complete(s, cpl, r->footprint, Solution(), false);
            continue;
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->preparing -= 1;
            Ready rd;
            rd.req = std::move(r);
            rd.p = p;
            s->ready.push_back(std::move(rd));
        }
        s->cv_ready.notify_all();
    }
    (void)hipStreamSynchronize(st);
    // problems created here now run on the engine's stream
    (void)hipStreamDestroy(st);
}

// One lane: a lockstep batch on a stream of its own, and the requests of its members.
struct Lane {
    hipStream_t st = nullptr;
    Batch B;
    Engine E;
    std::vector<Ready> held;
    std::vector<double> t_start;
};

// Complete the lane's members that finished (or, after a device error, every member;
// nothing of the lane is in flight when this runs):
// copy the solution out, publish the completion, and hand the problem to the preparer to
// destroy (its budget is released then).
static void drain_lane(lp_server* s, Lane& L, lp_status trc) {
    for (int slot = 0; slot < L.B.cap; ++slot) {
        Engine::Member& mb = L.E.mem[slot];
        if (mb.state != Engine::DONE && !(trc != LP_OK && mb.state != Engine::EMPTY)) continue;
        Ready& rd = L.held[slot];
        lp_completion cpl;
        memset(&cpl, 0, sizeof(cpl));
        cpl.ticket = rd.req->ticket;
        cpl.t_submit = rd.req->t_submit;
        cpl.t_start = L.t_start[slot];
        cpl.footprint = rd.req->footprint;
        Solution sol;
        if (trc != LP_OK) {
            cpl.status = trc;
        } else {
            lp_result res;
            fill_result(mb, &res);
            cpl.status = res.status;
            cpl.iters = res.iters;
            cpl.pobj = res.pobj;
            cpl.dobj = res.dobj;
            cpl.gamma_rel = res.gamma_rel;
            cpl.krylov_iters = res.krylov_iters;
            sol.x.resize((size_t)rd.req->n);
            sol.y.resize((size_t)rd.req->m);
            sol.s.resize((size_t)rd.req->n);
            const lp_status rc2 = lp_get_state(rd.p, sol.x.data(), sol.y.data(), sol.s.data(), nullptr);
            if (rc2 != LP_OK) cpl.status = rc2;
        }
        cpl.t_done = s->now();
        L.E.leave(slot);
        // the lane's stream is idle here and outlives no retired problem: the problem is
        // destroyed without it
        rd.p->st = nullptr;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->retire.emplace_back(rd.p, rd.req->footprint);
        }
        L.held[slot] = Ready();
        complete(s, cpl, 0, std::move(sol), true);
    }
}

// A lane's stream on a hardware queue of its own.  Streams otherwise share the process's few
// hardware queues (GPU_MAX_HW_QUEUES) with every other stream, the preparer's and the graph
// captures' included, and two lanes on one queue run their rounds in turn.  A stream created
// with a CU mask gets a queue of its own; the mask here covers every compute unit.
static hipError_t create_lane_stream(int device, hipStream_t* st) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0) {
        std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0xFFFFFFFFu);
        if (cus % 32) mask.back() = (1u << (cus % 32)) - 1u;
        if (hipExtStreamCreateWithCUMask(st, (uint32_t)mask.size(), mask.data()) == hipSuccess) return hipSuccess;
    }
    return hipStreamCreateWithFlags(st, hipStreamNonBlocking);
}

// The lanes: join ready problems into a lane's free slots whenever its previous round has
// completed, queue its next round, and complete the members that finished.  All launches
// come from this one thread.  While one lane's round runs on the GPU the others' rounds
// are queued on their streams, so their kernels overlap.
static void engine_main(lp_server* s) {
    bool ok = hipSetDevice(s->device) == hipSuccess;
    const int nl = std::max(1, std::min<int>(s->opt.lanes, s->opt.slots));
    std::vector<std::unique_ptr<Lane>> lanes;
    for (int l = 0; ok && l < nl; ++l) {
        std::unique_ptr<Lane> L(new Lane());
        if (create_lane_stream(s->device, &L->st) != hipSuccess) {
            ok = false;
            break;
        }
        // slots split as evenly as they go, the first lanes taking the remainder
        const int cap = s->opt.slots / nl + (l < s->opt.slots % nl ? 1 : 0);
        if (L->B.init(cap, L->st, true) != LP_OK) {
            ok = false;
            break;
        }
        L->E.attach(&L->B);
        L->held.resize((size_t)L->B.cap);
        L->t_start.assign((size_t)L->B.cap, 0.0);
        lanes.push_back(std::move(L));
    }
    auto busy = [&]() {
        for (auto& L : lanes)
            if (L->E.issued || L->E.any_live()) return true;
        return false;
    };
    while (ok) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_ready.wait(lk, [&] {
                if (busy()) return true;
                if (!s->ready.empty()) return true;
                return s->stop && s->queue.empty() && s->ready.empty() && s->preparing == 0;
            });
            if (!busy() && s->ready.empty()) break;
        }
        bool progressed = false;
        for (auto& Lp : lanes) {
            Lane& L = *Lp;
            if (L.E.issued) {
                if (!L.E.ready()) continue;
                const lp_status trc = L.E.complete();
                drain_lane(s, L, trc);
                progressed = true;
            }
            std::vector<Ready> joining;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                int free = 0;
                for (int i = 0; i < L.B.cap; ++i) free += L.B.mem[i] == nullptr;
                while (free > 0 && !s->ready.empty()) {
                    joining.push_back(std::move(s->ready.front()));
                    s->ready.pop_front();
                    --free;
                    s->running += 1;
                }
            }
            for (Ready& rd : joining) {
                // the problem was created (and synchronised) on the preparer's stream
                rd.p->st = L.st;
                const int slot = L.E.join(rd.p, false, rd.p->opt.ipm_max_iter);
                L.t_start[slot] = s->now();
                L.held[slot] = std::move(rd);
            }
            if (!L.E.any_live()) continue;
            const lp_status trc = L.E.issue();
            if (trc != LP_OK) {
                // what was queued before the error ends before the members leave
                (void)hipStreamSynchronize(L.st);
                L.E.issued = false;
                drain_lane(s, L, trc);
            }
            progressed = true;
        }
        // every queued round still running: wait a little before looking again
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (auto& L : lanes) (void)hipStreamSynchronize(L->st);
    lanes.clear();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->engine_done = true;
    }
    s->cv_work.notify_all();
}

extern "C" {

lp_status lp_server_options_default(lp_server_options* o) {
    if (!o) return LP_EINVAL;
    memset(o, 0, sizeof(*o));
    o->slots = 32;
    o->max_skip = 8;
    o->lanes = 1;
    o->hbm_budget = 0;
    return lp_options_default(&o->solver);
}

lp_status lp_server_create(const lp_server_options* o, lp_server** out) {
    if (!o || !out) return LP_EINVAL;
    *out = nullptr;
    if (o->slots < 1 || o->slots > 256 || o->max_skip < 0 || o->lanes < 1 || o->lanes > 8) {
        set_error("slots must be in [1, 256], lanes in [1, 8] and max_skip >= 0");
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
    s->prep = std::thread(prep_main, s);
    s->engine = std::thread(engine_main, s);
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
    s->cv_ready.notify_all();
    // the engine first: it may still wait for problems the preparer creates, and the
    // preparer destroys what the engine retires until the engine is done
    s->engine.join();
    s->prep.join();
    delete s;
    return LP_OK;
}

}  // extern "C"
