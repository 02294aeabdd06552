// Device prefix sums and reductions used by the format conversions
// (row pointers, diagonal slot maps, compaction offsets).
//
// Exclusive scan is reduce-then-scan: per-tile totals, a scan of the
// totals (recursively), then a tile-local scan plus the tile's offset.  All
// sums are formed in 64-bit integers, so results are exact and independent
// of the launch shape.
#include "core.hpp"

namespace dsm {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = threadIdx.x % WAVE;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        T t = __shfl_up(v, off, WAVE);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over the workgroup; returns the
// exclusive prefix and writes the workgroup total to *total.
__device__ __forceinline__ i64 block_excl_scan(i64 v, i64 *lds, i64 *total) {
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    i64 incl = wave_incl_scan(v);
    __syncthreads();
    if (lane == WAVE - 1) lds[w] = incl;
    __syncthreads();
    i64 off = 0, tot = 0;
    for (int i = 0; i < nw; i++) {
        if (i < w) off += lds[i];
        tot += lds[i];
    }
    *total = tot;
    return incl - v + off;
}

template <class InT>
__global__ void __launch_bounds__(SCAN_BLOCK) k_tile_sums(const InT *in, i64 n, i64 *sums) {
    __shared__ i64 lds[SCAN_BLOCK / WAVE];
    i64 base = (i64)blockIdx.x * SCAN_TILE + (i64)threadIdx.x * SCAN_ITEMS;
    i64 s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++)
        if (base + k < n) s += (i64)in[base + k];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

template <class InT, class OutT>
__global__ void __launch_bounds__(SCAN_BLOCK) k_tile_scan(const InT *in, OutT *out, i64 n,
                                                          const i64 *tile_off) {
    __shared__ i64 lds[SCAN_BLOCK / WAVE];
    i64 base = (i64)blockIdx.x * SCAN_TILE + (i64)threadIdx.x * SCAN_ITEMS;
    i64 v[SCAN_ITEMS];
    i64 s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        v[k] = base + k < n ? (i64)in[base + k] : 0;
        s += v[k];
    }
    i64 tot;
    i64 pre = block_excl_scan(s, lds, &tot) + (tile_off ? tile_off[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        if (base + k < n) out[base + k] = (OutT)pre;
        pre += v[k];
    }
    // the last element writes the grand total at out[n]
    if (base + SCAN_ITEMS >= n && base < n) out[n] = (OutT)pre;
}

template <class T>
__global__ void k_store_total(T *out, i64 n) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && n == 0) out[0] = 0;
}

template <class InT, class OutT>
static i64 scan_impl(dsm_ctx ctx, const InT *in, OutT *out, i64 n, hipStream_t s, bool want_total) {
    if (n == 0) {
        hipLaunchKernelGGL(k_store_total<OutT>, dim3(1), dim3(64), 0, s, out, (i64)0);
        DSM_HIP(hipGetLastError());
        return 0;
    }
    i64 ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    i64 *offs = nullptr;
    size_t obytes = 0;
    if (ntiles > 1) {
        obytes = sizeof(i64) * (size_t)(2 * ntiles + 1);
        offs = (i64 *)dev_alloc(ctx, obytes);
        i64 *sums = offs + ntiles + 1;
        hipLaunchKernelGGL(k_tile_sums<InT>, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, s, in, n, sums);
        DSM_HIP(hipGetLastError());
        try {
            scan_impl<i64, i64>(ctx, sums, offs, ntiles, s, false);
        } catch (...) {
            dev_free(ctx, offs, obytes);
            throw;
        }
    }
    hipLaunchKernelGGL((k_tile_scan<InT, OutT>), dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, s, in, out, n,
                       offs);
    DSM_HIP(hipGetLastError());
    i64 total = 0;
    if (want_total) {
        OutT t;
        DSM_HIP(hipMemcpyAsync(&t, out + n, sizeof(OutT), hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
        total = (i64)t;
    }
    if (offs) {
        if (!want_total) DSM_HIP(hipStreamSynchronize(s));
        dev_free(ctx, offs, obytes);
    }
    return total;
}

i64 exclusive_scan_i32(dsm_ctx ctx, const i32 *in, i32 *out, i64 n, hipStream_t s, bool want_total) {
    return scan_impl<i32, i32>(ctx, in, out, n, s, want_total);
}

i64 exclusive_scan_i64(dsm_ctx ctx, const i64 *in, i64 *out, i64 n, hipStream_t s, bool want_total) {
    return scan_impl<i64, i64>(ctx, in, out, n, s, want_total);
}

__global__ void __launch_bounds__(256) k_reduce_max(const i32 *in, i64 n, i32 *partial) {
    __shared__ i32 lds[256 / WAVE];
    i32 m = INT32_MIN;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        m = max(m, in[i]);
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, WAVE));
    if (threadIdx.x % WAVE == 0) lds[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256 / WAVE; i++) m = max(m, lds[i]);
        partial[blockIdx.x] = m;
    }
}

i32 reduce_max_i32(dsm_ctx ctx, const i32 *in, i64 n, hipStream_t s) {
    if (n == 0) return 0;
    unsigned g = (unsigned)std::min<i64>(1024, (n + 255) / 256);
    i32 *part = (i32 *)dev_alloc(ctx, sizeof(i32) * (g + 1));
    i32 h = 0;
    try {
        hipLaunchKernelGGL(k_reduce_max, dim3(g), dim3(256), 0, s, in, n, part);
        hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(256), 0, s, part, (i64)g, part + g);
        DSM_HIP(hipGetLastError());
        DSM_HIP(hipMemcpyAsync(&h, part + g, sizeof(i32), hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
    } catch (...) {
        dev_free(ctx, part, sizeof(i32) * (g + 1));
        throw;
    }
    dev_free(ctx, part, sizeof(i32) * (g + 1));
    return h;
}

}  // namespace dsm
