// Grouping of a DIA matrix's diagonals for the LDS-staged sweep: pure host
// logic (no HIP), so it can be checked on the CPU.
//
// Diagonals (offsets ascending) are cut into consecutive runs of at most
// `max_k` (<= CLU_MAXK) diagonals whose offsets lie within `max_span` of the
// run's first offset.  The result is a flat array of CLU_REC-int records,
// one per run, covering every diagonal once, in order: {first diagonal, one
// past the last, lowest offset, highest offset, then for u < CLU_MAXK the
// offset of diagonal first + u minus the lowest offset (0 past the last)}.
// A sweep reads a run's record in one 64-byte load and needs no other
// index.  With the sweep's limits (9 diagonals, span 256) a 27-point
// stencil on a grid of side n <= 127 gives 3 runs of 9 (the offsets of one
// z-plane, d-n-1 .. d+n+1).
#pragma once

#include <cstdint>
#include <vector>

namespace dsm {

constexpr int CLU_MAXK = 12;  // relative offsets a record holds
constexpr int CLU_REC = 16;   // ints per record

inline std::vector<int32_t> diagonal_clusters(const std::vector<int32_t> &offs, int max_k, int64_t max_span) {
    std::vector<int32_t> out;
    if (max_k > CLU_MAXK) max_k = CLU_MAXK;
    const int64_t nd = (int64_t)offs.size();
    for (int64_t k = 0; k < nd;) {
        int64_t e = k + 1;
        while (e < nd && e - k < max_k && (int64_t)offs[e] - offs[k] <= max_span) e++;
        out.insert(out.end(), {(int32_t)k, (int32_t)e, offs[k], offs[e - 1]});
        for (int64_t u = 0; u < CLU_MAXK; u++) out.push_back(k + u < e ? offs[k + u] - offs[k] : 0);
        k = e;
    }
    return out;
}

}  // namespace dsm
