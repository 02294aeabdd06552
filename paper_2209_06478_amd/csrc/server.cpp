// Serving loop: CG solves submitted one by one are admitted under a slot and
// HBM budget and run with continuous batching.
//
// Each worker thread owns one HIP stream and its own scratch.  A free
// worker takes the oldest queued request.  A large one is solved by the
// device-wide CG on the worker's stream; a small one is batched with every
// other queued small request that fits (up to batch_max, in arrival order)
// into one persistent launch where each workgroup solves one system.  Requests that arrive while other work is on the GPU
// are admitted as soon as a worker, a slot and budget are free, so their
// kernels overlap with the ones already running.  The footprint charged per
// request is its matrix payload plus its solver vectors; a request that can
// never fit is refused at submit.
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
        size_t footprint;
        bool small;
        bool done = false;
        dsm_status error = DSM_OK;
        dsm_cg_result res{};
        dsm_timestamps ts{};
    };
    dsm_server_s(const dsm_server_opts &o, size_t budget_bytes)
        : opts(o), budget(budget_bytes), adm(o.slots, budget_bytes, o.batch_max) {}
    dsm_ctx ctx = nullptr;
    dsm_server_opts opts{};
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    dsm::Admission adm;  // queue, slots and budget (guarded by mu)
    std::unordered_map<uint64_t, Req> reqs;
    bool stopping = false;
    uint64_t next_ticket = 1;
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace dsm {

static void worker_main(dsm_server s) {
    (void)hipSetDevice(s->ctx->device);
    hipStream_t stream = nullptr;
    (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    Workspace arena, cgws, spws;
    for (;;) {
        std::vector<uint64_t> take;
        bool small = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                const auto items = s->adm.take(&small);
                if (!items.empty()) {
                    const double t = s->now();
                    for (const auto &it : items) {
                        s->reqs[it.id].ts.start_s = t;
                        take.push_back(it.id);
                    }
                    break;
                }
                if (s->stopping && s->adm.empty()) break;
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
                    for (uint64_t id : take) {
                        auto &r = s->reqs[id];
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
                    auto &r = s->reqs[take[0]];
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
            const double t = s->now();
            for (size_t i = 0; i < take.size(); i++) {
                auto &r = s->reqs[take[i]];
                r.res = res[i];
                if (err != DSM_OK) r.res.status = err;
                r.error = err;
                r.ts.finish_s = t;
                r.done = true;
                s->adm.release(r.footprint);
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
        auto *s = new dsm_server_s(o, o.hbm_budget ? o.hbm_budget : ctx->budget);
        s->ctx = ctx;
        s->t0 = std::chrono::steady_clock::now();
        for (int i = 0; i < o.streams; i++) s->workers.emplace_back(worker_main, s);
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
        r.small = o.mode == DSM_CG_F64 && batch_eligible(m, s->opts.small_rows);
        r.footprint = m->P.bytes + (r.small ? batch_request_bytes(m->nrows) : cg_workspace_bytes(m->nrows, o.mode == DSM_CG_IR));
        DSM_CHECK(s->budget == 0 || r.footprint <= s->budget, DSM_E_NOMEM,
                  "request footprint exceeds the server's HBM budget");
        std::lock_guard<std::mutex> lk(s->mu);
        DSM_CHECK(!s->stopping, DSM_E_INVALID, "server is shutting down");
        r.ts.arrival_s = s->now();
        const uint64_t id = s->next_ticket++;
        s->reqs.emplace(id, r);
        s->adm.push(id, r.footprint, r.small);
        *ticket = id;
        s->cv_work.notify_one();
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
