// Scripted scenarios for the serving loop's admission queue (host logic
// only, no HIP): FIFO order, cross-queue batching of small requests,
// head-of-line blocking on the budget, slot and batch limits, workspaces
// kept by idle workers and charged to the budget, growth charged to the
// worker that grows, giving workspaces back when they keep the head out,
// requeueing after a failed allocation.  Prints "admission driver ok" and
// exits 0 when every check holds; otherwise reports the failed check and
// exits 1.
#include <cstdio>
#include <vector>

#include "../../paper_2209_06478_amd/csrc/admission.hpp"

using dsm::Admission;
using dsm::ws_round;
using dsm::WS_BATCH;
using dsm::WS_CG;
using dsm::WS_KINDS;
using dsm::WS_SPMV;

static int fails = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);   \
            fails++;                                                     \
        }                                                                \
    } while (0)

static std::vector<uint64_t> ids(const std::vector<Admission::Item> &v) {
    std::vector<uint64_t> r;
    for (auto &i : v) r.push_back(i.id);
    return r;
}

// a large request: matrix bytes and CG workspace bytes
static Admission::Item large(uint64_t id, size_t matrix, size_t cg, size_t spmv = 0) {
    Admission::Item it{id, matrix, {0, cg, spmv}, false};
    return it;
}

// a small request: matrix bytes and its share of a batch arena
static Admission::Item smallr(uint64_t id, size_t matrix, size_t share) {
    Admission::Item it{id, matrix, {share, 0, 0}, true};
    return it;
}

static void settle(Admission &a, int w, size_t batch, size_t cg, size_t spmv) {
    const size_t cap[WS_KINDS] = {batch, cg, spmv};
    a.settle(w, cap);
}

static void finish(Admission &a, const std::vector<Admission::Item> &items) {
    for (auto &i : items) a.release(i);
}

int main() {
    const size_t K = 1 << 16;  // the smallest workspace size (ws_round)
    bool small = false;
    CHECK(ws_round(1) == K && ws_round(K) == K && ws_round(K + 1) == 2 * K && ws_round(3 * K) == 4 * K);
    {  // arrival order; smalls gathered across the queue, larges left in place
        Admission a(64, 0, 256, 2);
        a.push(large(1, 100, 10));
        a.push(smallr(2, 10, 1));
        a.push(large(3, 100, 10));
        a.push(smallr(4, 10, 1));
        a.push(smallr(5, 10, 1));
        auto u1 = a.take(0, &small);
        CHECK(ids(u1) == std::vector<uint64_t>({1}) && !small);
        auto u2 = a.take(1, &small);
        CHECK(ids(u2) == std::vector<uint64_t>({2, 4, 5}) && small);
        auto u3 = a.take(0, &small);
        CHECK(ids(u3) == std::vector<uint64_t>({3}) && !small);
        CHECK(a.take(1, &small).empty() && a.empty());
        CHECK(a.in_flight() == 5 && a.matrix_bytes_in_flight() == 230);
        finish(a, u1);
        finish(a, u2);
        finish(a, u3);
        CHECK(a.in_flight() == 0 && a.matrix_bytes_in_flight() == 0);
    }
    {  // budget: a head that does not fit blocks the queue (no overtaking);
       // workspace growth is part of what must fit
        Admission a(64, 2 * K + 250, 256, 1);
        a.push(large(1, 200, K));
        a.push(large(2, 100, K));
        a.push(smallr(3, 10, 100));
        auto u1 = a.take(0, &small);
        CHECK(ids(u1) == std::vector<uint64_t>({1}));
        CHECK(a.charged() == 200 + K && a.held_bytes(0) == K);
        settle(a, 0, 0, K, 0);
        // 200 + K + 100 (no growth: the worker holds K) fits, but the
        // second request needs a slot only; it is admitted
        auto u2 = a.take(0, &small);
        CHECK(ids(u2) == std::vector<uint64_t>({2}) && a.charged() == 300 + K);
        // the small needs an arena of K: 300 + 2K + 10 > budget, it waits
        CHECK(a.take(0, &small).empty() && a.head_blocked_by_budget(0));
        finish(a, u1);
        auto u3 = a.take(0, &small);
        CHECK(ids(u3) == std::vector<uint64_t>({3}) && small && a.charged() == 110 + 2 * K);
    }
    {  // an idle worker keeps its workspace charged; reuse charges no growth
        Admission a(64, 0, 256, 2);
        a.push(large(1, 1000, 3 * K, 5));
        auto u = a.take(0, &small);
        CHECK(a.held_bytes(0) == 4 * K + K && a.held_bytes() == 5 * K);  // CG 3K -> 4K, SpMV 5 -> K
        settle(a, 0, 0, 4 * K, K);
        finish(a, u);
        CHECK(a.charged() == 5 * K && a.in_flight() == 0);
        a.push(large(2, 1000, 2 * K));
        u = a.take(0, &small);
        CHECK(a.held_bytes() == 5 * K && a.charged() == 1000 + 5 * K);  // fits in what worker 0 holds
        finish(a, u);
        a.push(large(3, 1000, 2 * K));
        u = a.take(1, &small);  // worker 1 holds nothing: it grows by 2K
        CHECK(a.held_bytes(1) == 2 * K && a.held_bytes() == 7 * K);
        CHECK(a.peak_charged() == 1000 + 7 * K);
        finish(a, u);
    }
    {  // the worker's actual holdings replace the prediction (a failed
       // allocation leaves nothing)
        Admission a(64, 0, 256, 1);
        a.push(large(1, 10, 2 * K));
        auto u = a.take(0, &small);
        CHECK(a.held_bytes(0) == 2 * K);
        settle(a, 0, 0, 0, 0);
        CHECK(a.held_bytes() == 0);
        finish(a, u);
    }
    {  // idle workspace that keeps the head out is given back
        Admission a(64, 8 * K, 256, 2);
        a.push(smallr(1, 0, 3 * K));
        auto u = a.take(1, &small);
        settle(a, 1, 4 * K, 0, 0);  // worker 1 keeps a 4K arena
        finish(a, u);
        a.push(large(2, 3 * K, 2 * K));  // 4K held + 3K + 2K > 8K on either worker
        CHECK(a.take(0, &small).empty() && a.take(1, &small).empty());
        CHECK(a.head_blocked_by_budget(0) && a.head_blocked_by_budget(1));
        CHECK(!a.should_shrink(0) && a.should_shrink(1));
        settle(a, 1, 0, 0, 0);  // worker 1 gave it back
        CHECK(!a.should_shrink(1));
        u = a.take(0, &small);
        CHECK(ids(u) == std::vector<uint64_t>({2}) && a.charged() == 5 * K);
        finish(a, u);
    }
    {  // the head fits only on the worker already holding its workspace:
       // an empty worker cannot take it and has nothing to give back, so
       // the server must wake every worker when a request arrives
        Admission a(64, 100 + 4 * K, 256, 2);
        a.push(large(1, 100, 3 * K));
        auto u = a.take(1, &small);
        settle(a, 1, 0, 4 * K, 0);
        finish(a, u);
        a.push(large(2, 100, 3 * K));
        CHECK(a.take(0, &small).empty() && a.head_blocked_by_budget(0));
        CHECK(!a.should_shrink(0) && !a.head_stuck(0));
        u = a.take(1, &small);
        CHECK(ids(u) == std::vector<uint64_t>({2}) && a.held_bytes() == 4 * K);
        finish(a, u);
    }
    {  // a failed allocation sends the unit back to the head while others
       // run; the queue waits for one of them to finish
        Admission a(64, 0, 256, 2);
        a.push(large(1, 10, K));
        a.push(large(2, 10, K));
        a.push(large(3, 10, K));
        auto u1 = a.take(0, &small);
        auto u2 = a.take(1, &small);
        CHECK(a.requeue(u2) && a.stalled() && a.queued() == 2 && a.in_flight() == 1);
        CHECK(a.take(1, &small).empty() && !a.should_shrink(1));
        finish(a, u1);
        CHECK(!a.stalled());
        auto again = a.take(1, &small);
        CHECK(ids(again) == std::vector<uint64_t>({2}));
        // nothing else in flight: the unit stays admitted and is failed
        CHECK(!a.requeue(again) && a.in_flight() == 1);
        finish(a, again);
        auto u3 = a.take(0, &small);
        CHECK(ids(u3) == std::vector<uint64_t>({3}));
        finish(a, u3);
    }
    {  // a batch goes back whole, in its order
        Admission a(64, 0, 256, 2);
        a.push(large(1, 10, K));
        a.push(smallr(2, 1, 1));
        a.push(smallr(3, 1, 1));
        auto u1 = a.take(0, &small);
        auto u2 = a.take(1, &small);
        CHECK(ids(u2) == std::vector<uint64_t>({2, 3}));
        CHECK(a.requeue(u2));
        finish(a, u1);
        CHECK(ids(a.take(1, &small)) == std::vector<uint64_t>({2, 3}));
    }
    {  // a gathered small is skipped while it does not fit, and stays queued
        Admission a(64, 3 * K + 100, 256, 1);
        a.push(smallr(1, 40, K / 2));
        a.push(smallr(2, 70, 3 * K));
        a.push(smallr(3, 30, K / 4));
        auto u = a.take(0, &small);
        CHECK(ids(u) == std::vector<uint64_t>({1, 3}));
        CHECK(a.queued() == 1 && a.take(0, &small).empty());
        settle(a, 0, K, 0, 0);
        finish(a, u);
        // the arena must grow to 4K: 4K + 70 > 3K + 100 even on an idle
        // server; submit refuses such a request up front
        CHECK(a.alone_bytes(smallr(9, 70, 3 * K)) == 70 + 4 * K);
    }
    {  // slots bound every batch and every admission
        Admission a(2, 0, 256, 1);
        for (uint64_t i = 1; i <= 3; i++) a.push(smallr(i, 1, 1));
        auto u = a.take(0, &small);
        CHECK(ids(u) == std::vector<uint64_t>({1, 2}));
        CHECK(a.take(0, &small).empty() && !a.head_blocked_by_budget(0));
        a.release(u[0]);
        CHECK(ids(a.take(0, &small)) == std::vector<uint64_t>({3}));
    }
    {  // batch_max splits a run of smalls
        Admission a(64, 0, 3, 1);
        for (uint64_t i = 1; i <= 5; i++) a.push(smallr(i, 1, 1));
        CHECK(ids(a.take(0, &small)) == std::vector<uint64_t>({1, 2, 3}));
        CHECK(ids(a.take(0, &small)) == std::vector<uint64_t>({4, 5}));
    }
    {  // an empty queue admits nothing; a request that fits an idle server alone is admitted
        Admission a(1, 50 + K, 8, 1);
        CHECK(a.take(0, &small).empty());
        a.push(large(9, 50, 10));
        CHECK(a.alone_bytes(large(9, 50, 10)) == 50 + K);
        CHECK(ids(a.take(0, &small)) == std::vector<uint64_t>({9}));
    }
    {  // the context's budget: what the context holds besides the workers'
       // workspaces is counted (resident matrices), not the matrices in flight
        Admission a(64, 10 * K, 256, 2, 0, false);
        a.set_external(6 * K);
        a.push(large(1, 5 * K, 2 * K));
        a.push(large(2, 5 * K, 2 * K));
        a.push(large(3, 5 * K, 4 * K));
        CHECK(a.could_fit_alone(large(3, 5 * K, 4 * K)) && !a.could_fit_alone(large(4, 0, 5 * K)));
        auto u1 = a.take(0, &small);
        CHECK(ids(u1) == std::vector<uint64_t>({1}) && a.charged() == 8 * K);
        auto u2 = a.take(1, &small);
        CHECK(ids(u2) == std::vector<uint64_t>({2}) && a.charged() == 10 * K);
        finish(a, u1);
        finish(a, u2);
        CHECK(a.charged() == 10 * K);  // the workspaces stay held
        CHECK(a.take(0, &small).empty() && a.should_shrink(0) && a.should_shrink(1));
        settle(a, 1, 0, 0, 0);
        // worker 0 holds 2K and needs 4K: 6K + 2K + 2K growth fits
        auto u3 = a.take(0, &small);
        CHECK(ids(u3) == std::vector<uint64_t>({3}) && a.charged() == 10 * K);
        finish(a, u3);
    }
    {  // a head that cannot get in while nothing runs and nothing is held
        Admission a(8, 4 * K, 8, 1, 0, false);
        a.set_external(K);
        a.push(large(1, 0, 2 * K));
        CHECK(!a.head_stuck(0));
        a.set_external(3 * K);  // the context filled up after the submit
        CHECK(a.head_stuck(0) && a.take(0, &small).empty());
        CHECK(a.pop_head().id == 1 && a.empty() && !a.head_stuck(0));
    }
    if (fails) return 1;
    std::printf("admission driver ok\n");
    return 0;
}
