// Streaming probes: the practical HBM ceiling that SpMV kernels are measured
// against.  A read-reduce (the access pattern of a matrix sweep: read only,
// a few bytes written), a copy and a write-only fill, each moving 16 B per
// lane per access.
#include "core.hpp"

namespace dsm {

constexpr int PB = 256;
constexpr int PU = 16;

struct alignas(16) d2 {
    double a, b;
};

// Each workgroup streams one contiguous chunk (1/gridDim of the buffer),
// PU loads of 16 B per lane in flight; contiguous chunks keep DRAM pages
// open (a grid-stride walk measured about 10% slower on MI355X).
__device__ __forceinline__ void chunk_of(i64 n, i64 &b0, i64 &b1) {
    const i64 per = (n + gridDim.x - 1) / gridDim.x;
    b0 = min((i64)blockIdx.x * per, n);
    b1 = min(b0 + per, n);
}

__global__ void __launch_bounds__(PB) k_probe_read(const d2 *__restrict__ src, i64 n, double *__restrict__ part) {
    i64 b0, b1;
    chunk_of(n, b0, b1);
    double s = 0.0;
    i64 i = b0 + threadIdx.x;
    for (; i + (PU - 1) * PB < b1; i += PU * PB) {
        d2 v[PU];
#pragma unroll
        for (int u = 0; u < PU; u++) v[u] = src[i + u * PB];
#pragma unroll
        for (int u = 0; u < PU; u++) s += v[u].a + v[u].b;
    }
    for (; i < b1; i += PB) s += src[i].a + src[i].b;
    __shared__ double lds[PB / WAVE];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(PB) k_probe_copy(const d2 *__restrict__ src, d2 *__restrict__ dst, i64 n) {
    i64 b0, b1;
    chunk_of(n, b0, b1);
    i64 i = b0 + threadIdx.x;
    for (; i + (PU - 1) * PB < b1; i += PU * PB) {
        d2 v[PU];
#pragma unroll
        for (int u = 0; u < PU; u++) v[u] = src[i + u * PB];
#pragma unroll
        for (int u = 0; u < PU; u++) dst[i + u * PB] = v[u];
    }
    for (; i < b1; i += PB) dst[i] = src[i];
}

__global__ void __launch_bounds__(PB) k_probe_write(d2 *__restrict__ dst, i64 n) {
    i64 b0, b1;
    chunk_of(n, b0, b1);
    const d2 z{0.0, 0.0};
    for (i64 i = b0 + threadIdx.x; i < b1; i += PB) dst[i] = z;
}

// Random-gather probe: the x-operand traffic of an irregular SpMV without
// the rest of it.  Lane-contiguous index loads (PU per lane in flight), then
// one 8-byte gather per index; an index outside [0, xlen) reads nothing.
__global__ void __launch_bounds__(PB) k_probe_gather(const double *__restrict__ x, i64 xlen,
                                                     const i32 *__restrict__ idx, i64 n, double *__restrict__ part) {
    i64 b0, b1;
    chunk_of(n, b0, b1);
    double s = 0.0;
    i64 i = b0 + threadIdx.x;
    for (; i + (PU - 1) * PB < b1; i += PU * PB) {
        i32 j[PU];
#pragma unroll
        for (int u = 0; u < PU; u++) j[u] = idx[i + u * PB];
        double v[PU];
#pragma unroll
        for (int u = 0; u < PU; u++) v[u] = (u64)(i64)j[u] < (u64)xlen ? x[j[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < PU; u++) s += v[u];
    }
    for (; i < b1; i += PB) {
        const i32 j = idx[i];
        s += (u64)(i64)j < (u64)xlen ? x[j] : 0.0;
    }
    __shared__ double lds[PB / WAVE];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void flush_read(const void *buf, i64 bytes, double *part, hipStream_t s) {
    hipLaunchKernelGGL(k_probe_read, dim3(DSM_PROBE_PARTIALS), dim3(PB), 0, s, (const d2 *)buf, bytes / 16, part);
    DSM_HIP(hipGetLastError());
}

}  // namespace dsm

using namespace dsm;

DSM_API dsm_status dsm_gather_probe(const double *x, int64_t xlen, const int32_t *idx, int64_t n, double *part,
                                    void *stream) {
    return guard([&] {
        DSM_CHECK(n >= 0 && xlen >= 0, DSM_E_INVALID, "negative length");
        DSM_CHECK(part && (idx || n == 0) && (x || xlen == 0), DSM_E_INVALID, "null buffer");
        hipLaunchKernelGGL(k_probe_gather, dim3(DSM_PROBE_PARTIALS), dim3(PB), 0, (hipStream_t)stream, x, xlen,
                           idx, n, part);
        DSM_HIP(hipGetLastError());
    });
}

DSM_API dsm_status dsm_stream_probe(int32_t mode, const void *src, void *dst, int64_t bytes, void *stream) {
    return guard([&] {
        DSM_CHECK(mode >= DSM_PROBE_READ && mode <= DSM_PROBE_WRITE, DSM_E_INVALID, "unknown probe mode");
        DSM_CHECK(bytes >= 0 && bytes % 16 == 0, DSM_E_INVALID, "bytes must be a non-negative multiple of 16");
        DSM_CHECK((mode == DSM_PROBE_WRITE || src) && dst, DSM_E_INVALID, "null buffer");
        DSM_CHECK(((uintptr_t)src % 16) == 0 && ((uintptr_t)dst % 16) == 0, DSM_E_INVALID,
                  "buffers must be 16-byte aligned");
        const i64 n = bytes / 16;
        hipStream_t s = (hipStream_t)stream;
        const dim3 g(DSM_PROBE_PARTIALS), b(PB);
        if (mode == DSM_PROBE_READ)
            hipLaunchKernelGGL(k_probe_read, g, b, 0, s, (const d2 *)src, n, (double *)dst);
        else if (n == 0)
            return;
        else if (mode == DSM_PROBE_COPY)
            hipLaunchKernelGGL(k_probe_copy, g, b, 0, s, (const d2 *)src, (d2 *)dst, n);
        else
            hipLaunchKernelGGL(k_probe_write, g, b, 0, s, (d2 *)dst, n);
        DSM_HIP(hipGetLastError());
    });
}
