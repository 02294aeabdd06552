// Device-resident solver state shared by the CG loops (plain, mixed
// precision, Jacobi and multigrid preconditioned): the state block, the
// deterministic reduction of per-workgroup partials, the done-flag
// broadcast and the chunked (optionally graph-replayed) host driver.
#pragma once

#include <string>

#include "core.hpp"

namespace dsm {

constexpr int CGB = 512;    // threads per workgroup in the vector kernels
constexpr int CGG = 512;    // workgroups in the vector kernels (= partials)

struct CgState {
    double rho[2];   // r.r (r.z when preconditioned) before iteration k is rho[(k-1) & 1]
    double nr0;      // ||r0||
    double pq;
    double relres;
    double tol;
    long long iters; // SpMVs done inside the loop
    long long maxit;
    int done;        // 0 running, 1 converged, 2 iteration limit, 3 breakdown
    int pad;
};

// Contiguous slice [slice_lo(n), slice_hi(n)) of [0, n) for this workgroup,
// a whole number of blockDim.x-element rows long: each workgroup of a
// vector kernel streams one run of consecutive elements, which keeps DRAM
// pages open (a grid-stride walk streamed about 10% slower on MI355X).
__device__ __forceinline__ i64 slice_len(i64 n) {
    const i64 per = (n + gridDim.x - 1) / gridDim.x;
    return (per + blockDim.x - 1) / blockDim.x * blockDim.x;
}
__device__ __forceinline__ i64 slice_lo(i64 n) { return min((i64)blockIdx.x * slice_len(n), n); }
__device__ __forceinline__ i64 slice_hi(i64 n) { return min(slice_lo(n) + slice_len(n), n); }

// Every workgroup reduces the same `count` partials in the same order.
__device__ __forceinline__ double reduce_partials(const double *part, double *lds, int count = CGG) {
    double v = 0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) v += part[i];
    return block_sum(v, lds);
}

// Reads the solve's done flag once per workgroup and shares it through LDS,
// so every wave of the workgroup takes the same early exit even while
// workgroup 0 of the same launch is writing the flag (the barriers later in
// the kernel must see all waves).
__device__ __forceinline__ bool wg_done(const int *flag) {
    __shared__ int s_done;
    if (threadIdx.x == 0) s_done = *(volatile const int *)flag;
    __syncthreads();
    return s_done != 0;
}

bool cg_graphs_enabled();

// Host driver of a device-resident loop: enqueues `enqueue(j, stream)` for
// j = 0 .. every-1 per chunk and reads the state back after each chunk,
// until its done flag is set or `cap` steps have been enqueued.  With
// use_graph the chunk is captured once per `key` into gws (replayed on
// gws's private stream after `s` has drained); if capture fails the chunk
// runs eagerly on `s`.
template <class Enq>
CgState run_chunks(Workspace &gws, const std::string &key, bool use_graph, int every, long long cap,
                   const CgState *st, hipStream_t s, Enq &&enqueue) {
    CgState h{};
    hipGraphExec_t exec = nullptr;
    if (use_graph && cg_graphs_enabled()) {
        // private replay stream (default priority, non-blocking)
        if (!gws.stream) DSM_HIP(hipStreamCreateWithFlags(&gws.stream, hipStreamNonBlocking));
        if (gws.graph_key != key) {
            if (gws.graph) (void)hipGraphExecDestroy((hipGraphExec_t)gws.graph);
            gws.graph = nullptr;
            gws.graph_key.clear();
            hipGraph_t g = nullptr;
            bool ok = hipStreamBeginCapture(gws.stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                // the capture is always closed, also when enqueueing fails
                try {
                    for (int j = 0; j < every; j++) enqueue(j, gws.stream);
                } catch (...) {
                    ok = false;
                }
                hipError_t ec = hipStreamEndCapture(gws.stream, &g);
                ok = ok && ec == hipSuccess && g != nullptr;
            }
            hipGraphExec_t ex = nullptr;
            if (ok) ok = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            if (ok) {
                gws.graph = ex;
                gws.graph_key = key;
            }
        }
        exec = (hipGraphExec_t)gws.graph;
    }
    if (exec) {
        DSM_HIP(hipStreamSynchronize(s));  // set-up work done before the replays
        long long done_steps = 0;
        for (;;) {
            DSM_HIP(hipGraphLaunch(exec, gws.stream));
            done_steps += every;
            DSM_HIP(hipMemcpyAsync(&h, st, sizeof(CgState), hipMemcpyDeviceToHost, gws.stream));
            DSM_HIP(hipStreamSynchronize(gws.stream));
            if (h.done || done_steps >= cap) break;
        }
        return h;
    }
    long long enq = 0;
    for (;;) {
        for (int j = 0; j < every && enq < cap; j++, enq++) enqueue(j, s);
        DSM_HIP(hipGetLastError());
        DSM_HIP(hipMemcpyAsync(&h, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
        if (h.done || enq >= cap) break;
    }
    return h;
}

}  // namespace dsm
