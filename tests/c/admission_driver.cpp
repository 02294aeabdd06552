// Scripted scenarios for the serving loop's admission queue (host logic
// only, no HIP): FIFO order, cross-queue batching of small requests,
// head-of-line blocking on the budget, slot and batch limits, release
// accounting.  Prints "admission driver ok" and exits 0 when every check
// holds; otherwise reports the failed check and exits 1.
#include <cstdio>
#include <vector>

#include "../../paper_2209_06478_amd/csrc/admission.hpp"

using dsm::Admission;

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

int main() {
    bool small = false;
    {  // arrival order; smalls gathered across the queue, larges left in place
        Admission a(64, 0, 256);
        a.push(1, 100, false);
        a.push(2, 10, true);
        a.push(3, 100, false);
        a.push(4, 10, true);
        a.push(5, 10, true);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({1}) && !small);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({2, 4, 5}) && small);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({3}) && !small);
        CHECK(a.take(&small).empty() && a.empty());
        CHECK(a.in_flight() == 5 && a.bytes_in_flight() == 230);
        for (size_t f : {100, 10, 100, 10, 10}) a.release(f);
        CHECK(a.in_flight() == 0 && a.bytes_in_flight() == 0);
    }
    {  // budget: a head that does not fit blocks the queue (no overtaking)
        Admission a(64, 250, 256);
        a.push(1, 200, false);
        a.push(2, 100, false);
        a.push(3, 10, true);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({1}));
        CHECK(a.take(&small).empty());  // 200 + 100 > 250; the small behind waits
        a.release(200);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({2}));
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({3}) && small);
        CHECK(a.bytes_in_flight() == 110);
    }
    {  // a gathered small is skipped while it does not fit, and stays queued
        Admission a(64, 100, 256);
        a.push(1, 40, true);
        a.push(2, 70, true);
        a.push(3, 30, true);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({1, 3}));
        CHECK(a.queued() == 1 && a.take(&small).empty());
        a.release(40);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({2}));
    }
    {  // slots bound every batch and every admission
        Admission a(2, 0, 256);
        for (uint64_t i = 1; i <= 3; i++) a.push(i, 1, true);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({1, 2}));
        CHECK(a.take(&small).empty());
        a.release(1);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({3}));
    }
    {  // batch_max splits a run of smalls
        Admission a(64, 0, 3);
        for (uint64_t i = 1; i <= 5; i++) a.push(i, 1, true);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({1, 2, 3}));
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({4, 5}));
    }
    {  // an empty queue admits nothing; a single request always fits an idle server
        Admission a(1, 50, 8);
        CHECK(a.take(&small).empty());
        a.push(9, 50, false);
        CHECK(ids(a.take(&small)) == std::vector<uint64_t>({9}));
    }
    if (fails) return 1;
    std::printf("admission driver ok\n");
    return 0;
}
