// Checks of the diagonal grouping used by the LDS-staged DIA sweep (host
// logic only, no HIP).  Prints "clusters driver ok" and exits 0 when every
// check holds; otherwise reports the failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2209_06478_amd/csrc/clusters.hpp"

using dsm::diagonal_clusters;

static int fails = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);   \
            fails++;                                                     \
        }                                                                \
    } while (0)

// every diagonal once, in order; each run within the limits and tight
static void check_invariants(const std::vector<int32_t> &offs, const std::vector<int32_t> &c, int max_k, long span) {
    const int R = dsm::CLU_REC;
    CHECK(c.size() % R == 0);
    if (max_k > dsm::CLU_MAXK) max_k = dsm::CLU_MAXK;
    int32_t next = 0;
    for (size_t r = 0; r + R - 1 < c.size(); r += R) {
        const int32_t kb = c[r], ke = c[r + 1], lo = c[r + 2], hi = c[r + 3];
        CHECK(kb == next);
        CHECK(ke > kb && ke - kb <= max_k);
        // relative offsets of the run's diagonals, zero past its end
        for (int u = 0; u < dsm::CLU_MAXK; u++) CHECK(c[r + 4 + u] == (kb + u < ke ? offs[kb + u] - lo : 0));
        CHECK(lo == offs[kb] && hi == offs[ke - 1]);
        CHECK((long)hi - lo <= span);
        // maximal: the next diagonal could not have joined this run
        if (ke < (int32_t)offs.size() && ke - kb < max_k) CHECK((long)offs[ke] - lo > span);
        next = ke;
    }
    CHECK(next == (int32_t)offs.size());
}

int main() {
    {  // 27-point stencil on an n^3 grid: 9 runs of 3
        const int n = 104;
        std::vector<int32_t> offs;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) offs.push_back(dx + n * dy + n * n * dz);
        const int R = dsm::CLU_REC;
        auto c = diagonal_clusters(offs, 3, 64);
        CHECK(c.size() == (size_t)9 * R);
        for (size_t r = 0; r < c.size(); r += R)
            CHECK(c[r + 1] - c[r] == 3 && c[r + 3] - c[r + 2] == 2 && c[r + 4] == 0 && c[r + 5] == 1 &&
                  c[r + 6] == 2 && c[r + 7] == 0);
        check_invariants(offs, c, 3, 64);
        // the sweep's limits: one run per z-plane, offsets n^2 dz + {-n-1 .. n+1}
        auto c9 = diagonal_clusters(offs, 9, 256);
        CHECK(c9.size() == (size_t)3 * R);
        for (size_t r = 0; r < c9.size(); r += R) {
            CHECK(c9[r + 1] - c9[r] == 9 && c9[r + 3] - c9[r + 2] == 2 * n + 2);
            const int rel[9] = {0, 1, 2, n, n + 1, n + 2, 2 * n, 2 * n + 1, 2 * n + 2};
            for (int u = 0; u < 9; u++) CHECK(c9[r + 4 + u] == rel[u]);
            for (int u = 9; u < dsm::CLU_MAXK; u++) CHECK(c9[r + 4 + u] == 0);
        }
        check_invariants(offs, c9, 9, 256);
    }
    {  // 7-point operator: -n^2, -n, {-1, 0, 1}, n, n^2
        const int n = 128;
        std::vector<int32_t> offs{-n * n, -n, -1, 0, 1, n, n * n};
        const int R = dsm::CLU_REC;
        auto c = diagonal_clusters(offs, 3, 64);
        CHECK(c.size() == (size_t)5 * R);
        CHECK(c[2 * R] == 2 && c[2 * R + 1] == 5);
        check_invariants(offs, c, 3, 64);
        // span 256: -n .. n (span 2n = 256) is one run
        auto c9 = diagonal_clusters(offs, 9, 256);
        CHECK(c9.size() == (size_t)3 * R);
        CHECK(c9[R] == 1 && c9[R + 1] == 6);
        check_invariants(offs, c9, 9, 256);
    }
    {  // banded: 129 consecutive diagonals -> 43 runs of 3
        std::vector<int32_t> offs;
        for (int d = -64; d <= 64; d++) offs.push_back(d);
        auto c = diagonal_clusters(offs, 3, 64);
        CHECK(c.size() == (size_t)43 * dsm::CLU_REC);
        check_invariants(offs, c, 3, 64);
        auto c9 = diagonal_clusters(offs, 9, 256);  // 14 runs of 9, one of 3
        CHECK(c9.size() == (size_t)15 * dsm::CLU_REC);
        check_invariants(offs, c9, 9, 256);
    }
    {  // scattered offsets: span limit splits runs
        std::vector<int32_t> offs{-1000, -900, -100, -99, -36, 0, 28, 29, 200, 264, 265, 5000};
        auto c = diagonal_clusters(offs, 3, 64);
        check_invariants(offs, c, 3, 64);
        const int R = dsm::CLU_REC;
        CHECK(c[0] == 0 && c[1] == 1);             // -1000 alone
        CHECK(c[R] == 1 && c[R + 1] == 2);         // -900 alone
        CHECK(c[2 * R] == 2 && c[2 * R + 1] == 5); // -100, -99, -36 (span 64)
        CHECK(c[2 * R + 4] == 0 && c[2 * R + 5] == 1 && c[2 * R + 6] == 64 && c[2 * R + 7] == 0);
    }
    {  // random ascending offsets, several limits
        std::srand(7);
        for (int trial = 0; trial < 200; trial++) {
            std::vector<int32_t> offs;
            int32_t o = -(std::rand() % 5000);
            const int nd = 1 + std::rand() % 60;
            for (int k = 0; k < nd; k++) {
                offs.push_back(o);
                o += 1 + std::rand() % 90;
            }
            const int max_k = 1 + std::rand() % 14;  // past CLU_MAXK too (capped)
            const long span = std::rand() % 300;
            check_invariants(offs, diagonal_clusters(offs, max_k, span), max_k, span);
        }
    }
    {  // no diagonals
        CHECK(diagonal_clusters({}, 3, 64).empty());
    }
    if (fails) return 1;
    std::printf("clusters driver ok\n");
    return 0;
}
