// Device-resident solver state shared by the CG loops (plain, mixed
// precision, Jacobi and multigrid preconditioned): the state block, the
// deterministic reduction of per-workgroup partials, the done-flag
// broadcast and the chunked (optionally graph-replayed) host driver.
#pragma once

#include <atomic>
#include <cstring>
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
    int pad;         // sequence number of the state copies to the host
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

// wg_done and reduce_partials in one round trip: the flag and the partials
// are loaded together before the first barrier.  *sum is valid only when the
// result is false.
__device__ __forceinline__ bool wg_done_sum(const int *flag, const double *part, int count, double *lds,
                                            double *sum) {
    __shared__ int s_done;
    int f = 0;
    if (threadIdx.x == 0) f = *(volatile const int *)flag;
    double v = 0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) v += part[i];
    if (threadIdx.x == 0) s_done = f;
    *sum = block_sum(v, lds);  // its barriers also publish s_done
    return s_done != 0;
}

bool cg_graphs_enabled();

// Enqueue the copy of *st into host slot (seq & 1) of a two-slot coherent
// pinned buffer (device-side address host_dev), seq counting the copies
// since the last enqueue_state_seq_reset.
void enqueue_state_out(CgState *st, CgState *host_dev, hipStream_t s);
void enqueue_state_seq_reset(CgState *st, hipStream_t s);

// Predicted relative residual one chunk ahead from the last two read back
// (geometric extrapolation); the last one when there is no decrease to
// extrapolate.
inline double next_relres(double older, double last) {
    return (older > 0 && last < older) ? last * (last / older) : last;
}

// Host driver of a device-resident loop: enqueues `enqueue(j, stream)` for
// j = 0 .. every-1 per chunk, each chunk followed by a kernel that copies
// the state to pinned host memory, until a chunk's state has its done flag set or `cap`
// steps have been enqueued.  While a chunk runs, the next one is enqueued
// before the host waits, unless the residual trend predicts convergence
// within the running chunk: the device then never idles between chunks,
// and a chunk enqueued past convergence only pays its launches (every
// kernel of the loop checks the done flag first).  With use_graph the chunk
// is captured once per `key` into gws (replayed on gws's private stream,
// which first waits for the work already queued on `s`); if capture fails
// the chunk runs eagerly on `s`.
// Returns after every enqueued chunk has finished, with the last state.
template <class Enq>
CgState run_chunks(Workspace &gws, const std::string &key, bool use_graph, int every, long long cap,
                   CgState *st, hipStream_t s, Enq &&enqueue) {
    if (!gws.host)
        DSM_HIP(hipHostMalloc(&gws.host, 2 * sizeof(CgState), hipHostMallocCoherent | hipHostMallocMapped));
    for (auto &e : gws.events)
        if (!e) DSM_HIP(hipEventCreateWithFlags((hipEvent_t *)&e, hipEventDisableTiming));
    CgState *slot = (CgState *)gws.host;
    CgState *slot_dev = nullptr;
    DSM_HIP(hipHostGetDevicePointer((void **)&slot_dev, gws.host, 0));

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
                    enqueue_state_out(st, slot_dev, gws.stream);
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
    hipStream_t rs = exec ? gws.stream : s;
    if (exec) {
        // the replays wait for the set-up work on `s` on the device (an
        // event, not a host round trip)
        DSM_HIP(hipEventRecord((hipEvent_t)gws.events[0], s));
        DSM_HIP(hipStreamWaitEvent(rs, (hipEvent_t)gws.events[0], 0));
    }
    enqueue_state_seq_reset(st, rs);

    long long steps = 0;
    long long issued = 0, read = 0;  // chunks enqueued / read back; chunk c lands in slot c & 1
    auto launch = [&]() {
        if (exec) {
            DSM_HIP(hipGraphLaunch(exec, rs));
            steps += every;
        } else {
            for (int j = 0; j < every && steps < cap; j++, steps++) enqueue(j, rs);
            enqueue_state_out(st, slot_dev, rs);
        }
        DSM_HIP(hipGetLastError());
        DSM_HIP(hipEventRecord((hipEvent_t)gws.events[issued & 1], rs));
        issued++;
    };
    auto wait_next = [&]() {
        const int k = (int)(read & 1);
        DSM_HIP(hipEventSynchronize((hipEvent_t)gws.events[k]));
        read++;
        std::atomic_thread_fence(std::memory_order_acquire);
        CgState h;
        std::memcpy(&h, &slot[k], sizeof h);
        DSM_CHECK(h.pad == (int)(read - 1), DSM_E_DEVICE, "solver state copy out of sequence");
        return h;
    };
    CgState h{};
    double older = -1, last = -1;  // relres of the last two chunks read
    launch();
    for (;;) {
        // one chunk in flight: enqueue the next unless it is predicted idle
        if (issued == read + 1 && steps < cap && read >= 2 && next_relres(older, last) > h.tol) launch();
        h = wait_next();
        older = last;
        last = h.relres;
        if (h.done) break;
        if (issued == read) {
            if (steps >= cap) break;
            launch();
        }
    }
    while (read < issued) h = wait_next();  // the chunk enqueued past convergence
    return h;
}

}  // namespace dsm
