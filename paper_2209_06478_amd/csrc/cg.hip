// Conjugate gradients on the device: HPCG's solver with the preconditioner
// switched off, as in the paper's port (Sections II-B and IV-B).
//
//   r = b - A x0, p = r, rho = r.r, stop when ||r|| <= tol ||r0||
//   loop: q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q;
//         rho' = r.r; test; beta = rho'/rho; p = r + beta p
//
// The whole loop stays on the GPU.  Scalars live in a small device state
// block; every workgroup that needs a dot product reduces the same array of
// per-workgroup partials in the same order, so all workgroups agree on alpha
// and beta bit for bit without a separate reduction launch, and the result
// does not depend on scheduling.  A device flag stops every later kernel once
// the solve has converged, broken down or hit maxit; the host reads the
// state back only every few iterations.
//
// Mixed precision (iterative refinement): the outer loop keeps x, the
// residual b - A x, its norm and the update x += d in FP64 (the residual
// SpMV accumulates the stored FP32/BF16 values in FP64); the inner CG solves
// A d = r/||r|| with FP32 vectors and FP32-accumulated SpMV, while its dot
// products are accumulated in FP64.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "core.hpp"

namespace dsm {

constexpr int CGB = 512;    // threads per workgroup in the vector kernels
constexpr int CGG = 512;    // workgroups in the vector kernels (= partials)

struct CgState {
    double rho[2];   // r.r before iteration k is rho[(k-1) & 1]
    double nr0;      // ||r0||
    double pq;
    double relres;
    double tol;
    long long iters; // SpMVs done inside the loop
    long long maxit;
    int done;        // 0 running, 1 converged, 2 iteration limit, 3 breakdown
    int pad;
};

// Every workgroup reduces the same CGG partials in the same order.
__device__ __forceinline__ double reduce_partials(const double *part, double *lds) {
    double v = 0;
    for (int i = threadIdx.x; i < CGG; i += blockDim.x) v += part[i];
    return block_sum(v, lds);
}

template <class X>
__global__ void __launch_bounds__(CGB) k_cg_init(i64 n, const X *b, const X *q, X *r, X *p, double *part) {
    __shared__ double lds[CGB / WAVE];
    double acc = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        X ri = b[i] - q[i];
        r[i] = ri;
        p[i] = ri;
        acc += (double)ri * (double)ri;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(CGB) k_cg_init_state(const double *part, CgState *st, double tol, long long maxit) {
    __shared__ double lds[CGB / WAVE];
    double rho = reduce_partials(part, lds);
    if (threadIdx.x == 0) {
        st->rho[0] = rho;
        st->rho[1] = 0;
        st->nr0 = sqrt(rho);
        st->pq = 0;
        st->relres = rho > 0 ? 1.0 : 0.0;
        st->tol = tol;
        st->iters = 0;
        st->maxit = maxit;
        st->done = rho == 0 ? 1 : (!isfinite(rho) ? 3 : (maxit <= 0 ? 2 : 0));
    }
}

template <class X>
__global__ void __launch_bounds__(CGB) k_cg_dot_pq(i64 n, const X *p, const X *q, double *part, CgState *st) {
    __shared__ double lds[CGB / WAVE];
    if (st->done) return;
    double acc = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        acc += (double)p[i] * (double)q[i];
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc;
        if (blockIdx.x == 0) st->iters += 1;
    }
}

template <class X>
__global__ void __launch_bounds__(CGB) k_cg_update_xr(i64 n, X *x, X *r, const X *p, const X *q,
                                                       const double *part_pq, double *part_rr, CgState *st) {
    __shared__ double lds[CGB / WAVE];
    if (st->done) return;
    const double pq = reduce_partials(part_pq, lds);
    const long long k = st->iters;
    const double rho = st->rho[(k - 1) & 1];
    if (!(pq > 0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->done = 3;
        }
        return;
    }
    const double alpha = rho / pq;
    const X a = (X)alpha;
    double acc = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        x[i] = x[i] + a * p[i];
        X ri = r[i] - a * q[i];
        r[i] = ri;
        acc += (double)ri * (double)ri;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = acc;
        if (blockIdx.x == 0) st->pq = pq;
    }
}

template <class X>
__global__ void __launch_bounds__(CGB) k_cg_update_p(i64 n, const X *r, X *p, const double *part_rr, CgState *st) {
    __shared__ double lds[CGB / WAVE];
    if (st->done) return;
    const double rho1 = reduce_partials(part_rr, lds);
    const long long k = st->iters;
    const double rho = st->rho[(k - 1) & 1];
    const double nr = sqrt(rho1);
    int done = 0;
    if (!isfinite(rho1)) done = 3;
    else if (nr <= st->tol * st->nr0) done = 1;
    else if (k >= st->maxit) done = 2;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->relres = st->nr0 > 0 ? nr / st->nr0 : 0.0;
        st->rho[k & 1] = rho1;
        if (done) st->done = done;
    }
    if (done) return;
    const X beta = (X)(rho1 / rho);
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        p[i] = r[i] + beta * p[i];
}

// ---------------------------------------------------------------- IR helpers
// r = b - q (FP64) and partial sums of r.r and b.b
__global__ void __launch_bounds__(CGB) k_residual(i64 n, const double *b, const double *q, double *r, double *part_rr,
                                                  double *part_bb) {
    __shared__ double lds[CGB / WAVE];
    double a = 0, c = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        double ri = b[i] - q[i];
        r[i] = ri;
        a += ri * ri;
        c += b[i] * b[i];
    }
    a = block_sum(a, lds);
    c = block_sum(c, lds);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = a;
        part_bb[blockIdx.x] = c;
    }
}

// two norms from partials -> out[0] = sqrt(sum rr), out[1] = sqrt(sum bb)
__global__ void __launch_bounds__(CGB) k_norms(const double *part_rr, const double *part_bb, double *out) {
    __shared__ double lds[CGB / WAVE];
    double a = reduce_partials(part_rr, lds);
    double c = reduce_partials(part_bb, lds);
    if (threadIdx.x == 0) {
        out[0] = sqrt(a);
        out[1] = sqrt(c);
    }
}

// r32 = r / ||r|| (FP32), d32 = 0
__global__ void __launch_bounds__(CGB) k_scale_down(i64 n, const double *r, const double *nrm, float *r32, float *d32) {
    const double inv = nrm[0] > 0 ? 1.0 / nrm[0] : 0.0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        r32[i] = (float)(r[i] * inv);
        d32[i] = 0.0f;
    }
}

// x += ||r|| * d32 (FP64)
__global__ void __launch_bounds__(CGB) k_apply_update(i64 n, double *x, const float *d32, const double *nrm) {
    const double s = nrm[0];
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        x[i] = x[i] + s * (double)d32[i];
}

// ================================================================ host side
struct CgBuffers {
    // FP64 part
    double *r = nullptr, *p = nullptr, *q = nullptr;
    double *part_a = nullptr, *part_b = nullptr, *norms = nullptr;
    CgState *st = nullptr, *st2 = nullptr;
    // FP32 inner part (IR)
    float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr, *ri32 = nullptr;
};

static CgBuffers cg_buffers(dsm_matrix m, bool ir, Workspace &cgws) {
    const size_t n = (size_t)std::max<i64>(m->nrows, 1);
    size_t bytes = 3 * ((n * 8 + 255) & ~(size_t)255) + 8 * 256 + 2 * CGG * 8;
    if (ir) bytes += 5 * ((n * 4 + 255) & ~(size_t)255);
    char *base = (char *)ws_get(m->ctx, cgws, bytes);
    CgBuffers B;
    auto take = [&](size_t sz) {
        char *p = base;
        base += (sz + 255) & ~(size_t)255;
        return (void *)p;
    };
    B.r = (double *)take(n * 8);
    B.p = (double *)take(n * 8);
    B.q = (double *)take(n * 8);
    B.part_a = (double *)take(CGG * 8);
    B.part_b = (double *)take(CGG * 8);
    B.norms = (double *)take(64);
    B.st = (CgState *)take(sizeof(CgState));
    B.st2 = (CgState *)take(sizeof(CgState));
    if (ir) {
        B.r32 = (float *)take(n * 4);
        B.p32 = (float *)take(n * 4);
        B.q32 = (float *)take(n * 4);
        B.d32 = (float *)take(n * 4);
        B.ri32 = (float *)take(n * 4);
    }
    return B;
}

// Workspace bytes a solve of this matrix needs (for admission control).
size_t cg_workspace_bytes(i64 n, bool ir) {
    const size_t nn = (size_t)std::max<i64>(n, 1);
    size_t bytes = 3 * ((nn * 8 + 255) & ~(size_t)255) + 8 * 256 + 2 * CGG * 8;
    if (ir) bytes += 5 * ((nn * 4 + 255) & ~(size_t)255);
    return bytes;
}

static unsigned vec_grid(i64 n) { return (unsigned)std::max<i64>(1, std::min<i64>(CGG, (n + CGB - 1) / CGB)); }

// One CG iteration: SpMV, p.q, x/r update, p update.  Every kernel checks
// the state's done flag first, so iterations enqueued past convergence cost
// only their launches.
template <class X>
static void enqueue_iteration(dsm_matrix m, X *x, X *r, X *p, X *q, double *part_a, double *part_b, CgState *st,
                              int vdt, hipStream_t s, Workspace &spws) {
    const i64 n = m->nrows;
    spmv(m, m->P, p, q, vdt, m->variant, s, &spws, &st->done);
    hipLaunchKernelGGL((k_cg_dot_pq<X>), dim3(CGG), dim3(CGB), 0, s, n, p, q, part_a, st);
    hipLaunchKernelGGL((k_cg_update_xr<X>), dim3(CGG), dim3(CGB), 0, s, n, x, r, p, q, part_a, part_b, st);
    hipLaunchKernelGGL((k_cg_update_p<X>), dim3(CGG), dim3(CGB), 0, s, n, r, p, part_b, st);
}

static bool graphs_enabled() {
    const char *e = getenv("DSM_CG_GRAPH");
    return !(e && e[0] == '0');
}

// Runs CG on (b, x) with vectors of type X.  Uses buffers r, p, q, part_*.
// The loop is replayed in chunks of `check_every` iterations from a HIP
// graph captured once per (matrix payload, buffers, chunk) and kept in
// `cgws`; the host reads the device state back once per chunk.  Returns the
// final state.
template <class X>
static CgState run_cg(dsm_matrix m, const X *b, X *x, X *r, X *p, X *q, double *part_a, double *part_b,
                      CgState *st, int vdt, double tol, long long maxit, int check_every, hipStream_t s,
                      Workspace &spws, Workspace &cgws, bool use_graph) {
    const i64 n = m->nrows;
    spmv(m, m->P, x, q, vdt, m->variant, s, &spws);
    hipLaunchKernelGGL((k_cg_init<X>), dim3(CGG), dim3(CGB), 0, s, n, b, q, r, p, part_a);
    hipLaunchKernelGGL(k_cg_init_state, dim3(1), dim3(CGB), 0, s, part_a, st, tol, maxit);
    DSM_HIP(hipGetLastError());
    CgState h{};
    hipStream_t gs = nullptr;
    hipGraphExec_t exec = nullptr;
    if (use_graph && graphs_enabled()) {
        const Payload &P = m->P;
        char key[512];
        snprintf(key, sizeof key, "%p|%d|%d|%d|%lld|%lld|%lld|%lld|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%d|%d|%p|%lld",
                 (void *)m, P.fmt, P.vdt, m->variant, (long long)P.ndiag, (long long)P.K, (long long)P.csr_nnz,
                 (long long)P.coo_nnz, (void *)P.rp, (void *)P.dval, (void *)P.evl, (void *)P.cval, (void *)x,
                 (void *)r, (void *)p, (void *)q, (void *)part_a, (void *)part_b, vdt, check_every, spws.p,
                 (long long)n);
        // private replay stream (default priority, non-blocking)
        if (!cgws.stream) DSM_HIP(hipStreamCreateWithFlags(&cgws.stream, hipStreamNonBlocking));
        gs = cgws.stream;
        // the scratch the SpMV needs is sized by the eager SpMV above
        if (cgws.graph_key != std::string(key) + "|" + std::to_string((uintptr_t)st)) {
            if (cgws.graph) (void)hipGraphExecDestroy((hipGraphExec_t)cgws.graph);
            cgws.graph = nullptr;
            cgws.graph_key.clear();
            hipGraph_t g = nullptr;
            bool ok = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                // the capture is always closed, also when enqueueing fails
                try {
                    for (int j = 0; j < check_every; j++)
                        enqueue_iteration<X>(m, x, r, p, q, part_a, part_b, st, vdt, gs, spws);
                } catch (...) {
                    ok = false;
                }
                hipError_t ec = hipStreamEndCapture(gs, &g);
                ok = ok && ec == hipSuccess && g != nullptr;
            }
            hipGraphExec_t ex = nullptr;
            if (ok) ok = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            if (ok) {
                cgws.graph = ex;
                cgws.graph_key = std::string(key) + "|" + std::to_string((uintptr_t)st);
            }
        }
        exec = (hipGraphExec_t)cgws.graph;
    }
    if (exec) {
        DSM_HIP(hipStreamSynchronize(s));  // init work done before the replays
        long long done_iters = 0;
        for (;;) {
            DSM_HIP(hipGraphLaunch(exec, gs));
            done_iters += check_every;
            DSM_HIP(hipMemcpyAsync(&h, st, sizeof(CgState), hipMemcpyDeviceToHost, gs));
            DSM_HIP(hipStreamSynchronize(gs));
            if (h.done || done_iters >= maxit) break;
        }
        return h;
    }
    long long enq = 0;
    for (;;) {
        for (int j = 0; j < check_every && enq < maxit; j++, enq++)
            enqueue_iteration<X>(m, x, r, p, q, part_a, part_b, st, vdt, s, spws);
        DSM_HIP(hipGetLastError());
        DSM_HIP(hipMemcpyAsync(&h, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
        if (h.done || enq >= maxit) break;
    }
    return h;
}

// ||b - A x|| / ||b|| in FP64 on the device (A with its stored values)
static double true_relres(dsm_matrix m, const double *b, const double *x, CgBuffers &B, hipStream_t s,
                          Workspace &spws) {
    const i64 n = m->nrows;
    spmv(m, m->P, x, B.q, DSM_F64, m->variant, s, &spws);
    hipLaunchKernelGGL(k_residual, dim3(CGG), dim3(CGB), 0, s, n, b, B.q, B.r, B.part_a, B.part_b);
    hipLaunchKernelGGL(k_norms, dim3(1), dim3(CGB), 0, s, B.part_a, B.part_b, B.norms);
    DSM_HIP(hipGetLastError());
    double h[2];
    DSM_HIP(hipMemcpyAsync(h, B.norms, sizeof(h), hipMemcpyDeviceToHost, s));
    DSM_HIP(hipStreamSynchronize(s));
    return h[1] > 0 ? h[0] / h[1] : h[0];
}

static int default_check_every(i64 n) { return n < 100000 ? 32 : 8; }

void cg_solve_ws(dsm_matrix m, const double *b, double *x, const dsm_cg_opts &o, dsm_cg_result *res, hipStream_t s,
                 Workspace &cgws, Workspace &spws, bool use_graph) {
    DSM_CHECK(m->nrows == m->ncols, DSM_E_UNSUPPORTED, "CG needs a square matrix");
    const i64 n = m->nrows;
    long long maxit = o.maxit > 0 ? o.maxit : std::min<long long>(10 * std::max<i64>(n, 1), 20000);
    int every = o.check_every > 0 ? o.check_every : default_check_every(n);
    dsm_cg_result R{};
    const bool ir = o.mode == DSM_CG_IR;
    DSM_CHECK(o.mode == DSM_CG_F64 || o.mode == DSM_CG_IR, DSM_E_INVALID, "unknown CG mode");
    DSM_CHECK(!ir || m->P.vdt != DSM_F64, DSM_E_UNSUPPORTED,
              "iterative refinement needs F32 or BF16 matrix values (convert with value_dtype)");
    CgBuffers B = cg_buffers(m, ir, cgws);
    if (n == 0) {
        R.status = DSM_OK;
        *res = R;
        return;
    }
    if (!ir) {
        CgState h = run_cg<double>(m, b, x, B.r, B.p, B.q, B.part_a, B.part_b, B.st, DSM_F64, o.tol, maxit, every, s,
                                   spws, cgws, use_graph);
        R.iters = h.iters;
        R.relres = h.relres;
        R.status = h.done == 1 ? DSM_OK : h.done == 3 ? DSM_E_BREAKDOWN : DSM_E_NOT_CONVERGED;
        R.relres_true = true_relres(m, b, x, B, s, spws);
        *res = R;
        return;
    }
    // iterative refinement
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-4;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 50;
    long long inner_total = 0;
    int status = DSM_E_NOT_CONVERGED;
    double relres = 1.0;
    for (int outer = 0;; outer++) {
        // r = b - A x in FP64, norms
        spmv(m, m->P, x, B.q, DSM_F64, m->variant, s, &spws);
        hipLaunchKernelGGL(k_residual, dim3(CGG), dim3(CGB), 0, s, n, b, B.q, B.r, B.part_a, B.part_b);
        hipLaunchKernelGGL(k_norms, dim3(1), dim3(CGB), 0, s, B.part_a, B.part_b, B.norms);
        DSM_HIP(hipGetLastError());
        double nrm[2];
        DSM_HIP(hipMemcpyAsync(nrm, B.norms, sizeof(nrm), hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
        relres = nrm[1] > 0 ? nrm[0] / nrm[1] : nrm[0];
        R.outer_iters = outer;
        if (!std::isfinite(relres)) {
            status = DSM_E_BREAKDOWN;
            break;
        }
        if (nrm[0] == 0 || relres <= o.tol) {
            status = DSM_OK;
            break;
        }
        if (outer >= max_outer || inner_total >= maxit) break;
        // inner FP32 solve of A d = r / ||r||
        hipLaunchKernelGGL(k_scale_down, dim3(CGG), dim3(CGB), 0, s, n, B.r, B.norms, B.r32, B.d32);
        DSM_HIP(hipGetLastError());
        // the scaled residual r32 is the inner right-hand side, d32 the inner iterate
        CgState h = run_cg<float>(m, B.r32, B.d32, B.ri32, B.p32, B.q32, B.part_a, B.part_b, B.st2, DSM_F32,
                                  inner_tol, std::max<long long>(1, maxit - inner_total), every, s, spws,
                                  cgws, use_graph);
        inner_total += h.iters;
        if (h.done == 3 && h.iters <= 1) {
            status = DSM_E_BREAKDOWN;
            break;
        }
        hipLaunchKernelGGL(k_apply_update, dim3(CGG), dim3(CGB), 0, s, n, x, B.d32, B.norms);
        DSM_HIP(hipGetLastError());
    }
    R.iters = inner_total;
    R.relres = relres;
    R.status = status;
    R.relres_true = true_relres(m, b, x, B, s, spws);
    *res = R;
}

}  // namespace dsm

using namespace dsm;

DSM_API void dsm_cg_opts_default(dsm_cg_opts *o) {
    if (!o) return;
    o->tol = 1e-10;
    o->maxit = 0;
    o->mode = DSM_CG_F64;
    o->inner_tol = 1e-4;
    o->check_every = 0;
    o->max_outer = 50;
}

DSM_API dsm_status dsm_cg_solve(dsm_matrix m, const double *b, double *x, const dsm_cg_opts *opts,
                                dsm_cg_result *result, void *stream) {
    dsm_cg_result R{};
    dsm_status st = guard([&] {
        DSM_CHECK(m && m->ctx, DSM_E_INVALID, "null matrix handle");
        DSM_CHECK((b && x) || m->nrows == 0, DSM_E_INVALID, "null vector");
        DSM_CHECK(result, DSM_E_INVALID, "result is null");
        DSM_HIP(hipSetDevice(m->ctx->device));
        dsm_cg_opts o;
        dsm_cg_opts_default(&o);
        if (opts) o = *opts;
        DSM_CHECK(o.tol >= 0, DSM_E_INVALID, "negative tolerance");
        hipStream_t s = (hipStream_t)stream;
        cg_solve_ws(m, b, x, o, &R, s, m->cgws, m->ws, true);
        m->last_stream = s;
    });
    if (result) *result = R;
    if (st != DSM_OK) return st;
    return R.status;
}
