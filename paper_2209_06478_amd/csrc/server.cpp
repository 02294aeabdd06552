// Serving loop: CG solves submitted one by one are admitted under a slot and
// HBM budget and run with continuous batching.
//
// Each worker thread owns one HIP stream and its own workspaces.  A free
// worker takes the oldest queued request.  A large one is solved by the
// device-wide CG on the worker's stream; a small one is batched with every
// other queued small request that fits (up to batch_max, in arrival order)
// into one persistent launch where each workgroup solves one system.
// Requests that arrive while other work is on the GPU are admitted as soon
// as a worker, a slot and budget are free, so their kernels overlap with the
// ones already running.  The budget counts the matrices of the requests in
// flight and the workspaces the workers hold (admission.hpp); a request that
// can never fit is refused at submit.  A workspace allocation that fails on
// the device (another user of the context's budget, or hipMalloc) sends the
// request back to the head of the queue while other requests are in flight,
// and fails it with DSM_E_NOMEM when none is.
//
// Every path is deterministic per request, so a request's iterate and
// iteration count are the same whether it ran alone or in a mix.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.hpp"
#include "core.hpp"

struct dsm_server_s {
    struct Req {
        dsm_matrix m;
        const double *b;
        double *x;
        dsm_cg_opts o;
        dsm::Admission::Item item;
        bool done = false;
        dsm_status error = DSM_OK;
        dsm_cg_result res{};
        dsm_timestamps ts{};
    };
    // With no budget of its own the server takes the context's, and then
    // counts what the context really holds (its bytes in use) instead of
    // the matrices in flight.
    dsm_server_s(const dsm_server_opts &o, dsm_ctx c)
        : ctx(c), opts(o), budget(o.hbm_budget ? o.hbm_budget : c->budget),
          ctx_mode(o.hbm_budget == 0 && c->budget != 0),
          adm(o.slots, budget, o.batch_max, o.streams, dsm::batch_arena_fixed(), !ctx_mode) {}
    dsm_ctx ctx = nullptr;
    dsm_server_opts opts{};
    size_t budget = 0;
    bool ctx_mode = false;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    dsm::Admission adm;  // queue, slots and budget (guarded by mu)
    std::unordered_map<uint64_t, Req> reqs;
    bool stopping = false;
    uint64_t next_ticket = 1;
    uint64_t requeued = 0;  // units sent back to the queue after a failed allocation
    uint64_t submitted = 0, completed = 0, budget_waits = 0, last_blocked = 0;
    int running = 0;        // units of work between their start and their result
    double busy_since = 0, busy_s = 0;

    // Device bytes the workers' workspaces hold at this moment, updated by
    // the allocations themselves (a workspace grown during a unit of work is
    // counted before the unit settles).  Allocation adds before and freeing
    // subtracts after the context's own count changes, so the difference
    // below can only undercount the bytes held by others, never count a
    // workspace twice (which would refuse requests that fit).
    std::atomic<size_t> ws_live{0};

    // guarded by mu
    void refresh() {
        if (!ctx_mode) return;
        const size_t in = ctx->in_use.load(), ws = ws_live.load();
        adm.set_external(in > ws ? in - ws : 0);
    }
    void settle(int w, const size_t *cap) { adm.settle(w, cap); }
    void unit_started(double t) {
        if (running++ == 0) busy_since = t;
    }
    void unit_ended(double t) {
        if (--running == 0) busy_s += t - busy_since;
    }
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace dsm {

static void held_caps(const Workspace &arena, const Workspace &cgws, const Workspace &spws, size_t *cap) {
    cap[WS_BATCH] = arena.p ? arena.bytes : 0;
    cap[WS_CG] = cgws.p ? cgws.bytes : 0;
    cap[WS_SPMV] = spws.p ? spws.bytes : 0;
}

static void worker_main(dsm_server s, int w) {
    (void)hipSetDevice(s->ctx->device);
    hipStream_t stream = nullptr;
    (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    Workspace arena, cgws, spws;
    arena.grow_pow2 = cgws.grow_pow2 = spws.grow_pow2 = true;  // sizes the admission predicts
    arena.live = cgws.live = spws.live = &s->ws_live;
    size_t cap[WS_KINDS];
    for (;;) {
        std::vector<Admission::Item> take;
        bool small = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                s->refresh();
                take = s->adm.take(w, &small);
                if (!take.empty()) {
                    const double t = s->now();
                    for (const auto &it : take) s->reqs[it.id].ts.start_s = t;
                    s->unit_started(t);
                    break;
                }
                if (s->stopping && s->adm.empty()) break;
                if (s->adm.head_blocked_by_budget(w) && s->adm.head_id() != s->last_blocked) {
                    s->budget_waits++;
                    s->last_blocked = s->adm.head_id();
                }
                if (s->adm.head_stuck(w)) {
                    // nothing in flight or held can make room: fail it
                    const Admission::Item it = s->adm.pop_head();
                    auto &r = s->reqs[it.id];
                    r.res = dsm_cg_result{};
                    r.res.status = DSM_E_NOMEM;
                    r.error = DSM_E_NOMEM;
                    r.ts.start_s = r.ts.finish_s = s->now();
                    r.done = true;
                    s->completed++;
                    s->cv_done.notify_all();
                    s->cv_work.notify_all();  // a new head, maybe for another worker
                    continue;
                }
                if (s->adm.should_shrink(w)) {
                    // idle, and what this worker holds keeps the head out:
                    // give it back (nothing of this worker is in flight)
                    lk.unlock();
                    (void)hipStreamSynchronize(stream);
                    ws_release(s->ctx, arena);
                    ws_release(s->ctx, cgws);
                    ws_release(s->ctx, spws);
                    lk.lock();
                    held_caps(arena, cgws, spws, cap);
                    s->settle(w, cap);
                    s->cv_work.notify_all();
                    continue;
                }
                s->cv_work.wait(lk);
            }
            if (take.empty()) break;  // stopping and drained
        }
        // run outside the lock
        std::vector<dsm_cg_result> res(take.size());
        dsm_status err = DSM_OK;
        std::string msg;
        try {
            if (small) {
                BatchJob job;
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    for (const auto &it : take) {
                        auto &r = s->reqs[it.id];
                        job.mats.push_back(r.m);
                        job.b.push_back(r.b);
                        job.x.push_back(r.x);
                        job.opts.push_back(r.o);
                    }
                }
                run_batch(s->ctx, job, res.data(), arena, stream);
            } else {
                dsm_matrix m;
                const double *b;
                double *x;
                dsm_cg_opts o;
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    auto &r = s->reqs[take[0].id];
                    m = r.m;
                    b = r.b;
                    x = r.x;
                    o = r.o;
                }
                cg_solve_ws(m, b, x, o, &res[0], stream, cgws, spws, false);
            }
        } catch (const Error &e) {
            err = e.status;
            msg = e.msg;
            (void)hipStreamSynchronize(stream);
        } catch (...) {
            err = DSM_E_DEVICE;
            (void)hipStreamSynchronize(stream);
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            held_caps(arena, cgws, spws, cap);
            s->settle(w, cap);
            // a workspace that could not be allocated: the solve had not
            // started (workspaces are sized before the first launch), so
            // the request can wait for memory at the head of the queue
            const double t = s->now();
            s->unit_ended(t);
            if (err == DSM_E_NOMEM && s->adm.requeue(take)) {
                s->requeued++;
            } else {
                s->completed += take.size();
                for (const auto &it : take) {
                    auto &r = s->reqs[it.id];
                    r.res = res[&it - &take[0]];
                    if (err != DSM_OK) r.res.status = err;
                    r.error = err;
                    r.ts.finish_s = t;
                    r.done = true;
                    s->adm.release(it);
                }
            }
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
    ws_release(s->ctx, arena);
    ws_release(s->ctx, cgws);
    ws_release(s->ctx, spws);
    if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace dsm

using namespace dsm;

DSM_API void dsm_server_opts_default(dsm_server_opts *o) {
    if (!o) return;
    o->slots = 64;
    o->hbm_budget = 0;
    o->streams = 4;
    // one-workgroup batching raises throughput a little (5% at saturation on
    // the mixed stream) but holds every system of a batch until its slowest
    // member finishes: past a few thousand rows the device-wide solver's
    // latency is far lower (p50 1.6 vs 19.5 ms at 400 requests/s)
    o->small_rows = 4096;
    o->batch_max = 256;
}

DSM_API dsm_status dsm_server_create(dsm_ctx ctx, const dsm_server_opts *opts, dsm_server *out) {
    return guard([&] {
        DSM_CHECK(ctx && out, DSM_E_INVALID, "null argument");
        dsm_server_opts o;
        dsm_server_opts_default(&o);
        if (opts) o = *opts;
        DSM_CHECK(o.slots >= 1 && o.streams >= 1 && o.streams <= 16 && o.batch_max >= 1, DSM_E_INVALID,
                  "slots, streams (1..16) and batch_max must be positive");
        DSM_CHECK(o.small_rows >= 0 && o.small_rows <= 40000, DSM_E_INVALID,
                  "small_rows must be in [0, 40000] (the one-workgroup solver's limit)");
        auto *s = new dsm_server_s(o, ctx);
        s->t0 = std::chrono::steady_clock::now();
        for (int i = 0; i < o.streams; i++) s->workers.emplace_back(worker_main, s, i);
        *out = s;
    });
}

DSM_API dsm_status dsm_server_submit(dsm_server s, dsm_matrix m, const double *b, double *x, const dsm_cg_opts *opts,
                                     uint64_t *ticket) {
    return guard([&] {
        DSM_CHECK(s && m && m->ctx == s->ctx && ticket, DSM_E_INVALID, "null argument or foreign matrix");
        DSM_CHECK(m->nrows == m->ncols, DSM_E_UNSUPPORTED, "CG needs a square matrix");
        DSM_CHECK((b && x) || m->nrows == 0, DSM_E_INVALID, "null vector");
        dsm_cg_opts o;
        dsm_cg_opts_default(&o);
        if (opts) o = *opts;
        DSM_CHECK(o.tol >= 0, DSM_E_INVALID, "negative tolerance");
        dsm_server_s::Req r;
        r.m = m;
        r.b = b;
        r.x = x;
        r.o = o;
        Admission::Item &it = r.item;
        it.small = o.mode == DSM_CG_F64 && batch_eligible(m, s->opts.small_rows);
        it.matrix = m->P.bytes;
        it.ws[WS_BATCH] = it.small ? batch_request_bytes(m->nrows) : 0;
        it.ws[WS_CG] = it.small ? 0 : cg_workspace_bytes(m->nrows, o.mode == DSM_CG_IR || o.mode == DSM_CG_IR_CONT);
        it.ws[WS_SPMV] = it.small ? 0 : spmv_scratch_bytes(m, m->P, DSM_F64);
        std::lock_guard<std::mutex> lk(s->mu);
        s->refresh();
        DSM_CHECK(s->adm.could_fit_alone(it), DSM_E_NOMEM, "request footprint exceeds the server's HBM budget");
        DSM_CHECK(!s->stopping, DSM_E_INVALID, "server is shutting down");
        r.ts.arrival_s = s->now();
        const uint64_t id = s->next_ticket++;
        it.id = id;
        s->reqs.emplace(id, r);
        s->adm.push(it);
        s->submitted++;
        *ticket = id;
        // every idle worker looks: the head may fit only on a worker that
        // already holds large enough workspaces, and a worker that cannot
        // take it waits without waking the others
        s->cv_work.notify_all();
    });
}

static dsm_status fill(dsm_server_s::Req &r, dsm_cg_result *res, dsm_timestamps *ts) {
    if (res) *res = r.res;
    if (ts) *ts = r.ts;
    return r.error;
}

DSM_API dsm_status dsm_server_poll(dsm_server s, uint64_t ticket, dsm_cg_result *result, dsm_timestamps *ts) {
    dsm_status inner = DSM_OK;
    dsm_status st = guard([&] {
        DSM_CHECK(s, DSM_E_INVALID, "null server");
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        DSM_CHECK(it != s->reqs.end(), DSM_E_INVALID, "unknown ticket");
        if (!it->second.done) {
            inner = DSM_E_PENDING;
            return;
        }
        inner = fill(it->second, result, ts);
    });
    return st != DSM_OK ? st : inner;
}

DSM_API dsm_status dsm_server_wait(dsm_server s, uint64_t ticket, dsm_cg_result *result, dsm_timestamps *ts) {
    dsm_status inner = DSM_OK;
    dsm_status st = guard([&] {
        DSM_CHECK(s, DSM_E_INVALID, "null server");
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        DSM_CHECK(it != s->reqs.end(), DSM_E_INVALID, "unknown ticket");
        s->cv_done.wait(lk, [&] { return it->second.done; });
        inner = fill(it->second, result, ts);
    });
    return st != DSM_OK ? st : inner;
}

DSM_API double dsm_server_now(dsm_server s) { return s ? s->now() : 0.0; }

DSM_API dsm_status dsm_server_get_stats(dsm_server s, dsm_server_stats *out) {
    return guard([&] {
        DSM_CHECK(s && out, DSM_E_INVALID, "null argument");
        std::lock_guard<std::mutex> lk(s->mu);
        const double t = s->now();
        dsm_server_stats st{};
        st.submitted = s->submitted;
        st.completed = s->completed;
        st.budget_waits = s->budget_waits;
        st.requeued = s->requeued;
        st.peak_charged_bytes = s->adm.peak_charged();
        st.workspace_bytes = s->adm.held_bytes();
        st.busy_s = s->busy_s + (s->running > 0 ? t - s->busy_since : 0.0);
        st.elapsed_s = t;
        *out = st;
    });
}

DSM_API dsm_status dsm_server_destroy(dsm_server s) {
    return guard([&] {
        if (!s) return;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stopping = true;
        }
        s->cv_work.notify_all();
        for (auto &t : s->workers) t.join();
        delete s;
    });
}
