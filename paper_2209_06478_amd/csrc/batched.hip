// Batched CG: many independent small systems in one persistent launch.
//
// A fixed grid of workgroups pulls request indices from an integer counter;
// each workgroup then runs one request's whole CG loop by itself, with
// workgroup barriers as the only synchronisation (no inter-workgroup waits,
// so every workgroup finishes once the counter passes the request count).
// Every reduction inside a request uses the same thread-to-element map and
// the same fixed combination order, so a request's iterates and iteration
// count do not depend on which workgroup runs it or on what else is in the
// batch.
//
// Supported in-workgroup formats: CSR (a power-of-two lane group per row,
// the "tile" the batched tuner picks), DIA and ELL, with FP64 values.
// Anything else, or systems above the size threshold, is solved by the
// device-wide solver on a side stream while the batch kernel runs.
#include <algorithm>
#include <thread>
#include <vector>

#include "core.hpp"

namespace dsm {

constexpr int BB = 512;  // threads per workgroup of the batched kernel
constexpr i64 BATCH_SMALL_ROWS = 40000;  // largest system solved by one workgroup

struct BReq {
    int fmt;
    int lanes;
    i64 n;
    const i32 *rp;
    const i32 *col;
    const double *val;
    const i32 *offs;
    i64 ndiag;
    i64 pitch;
    const double *dval;
    const i32 *ecol;
    const double *evl;
    i64 K;
    const double *b;
    double *x;
    double *r;
    double *p;
    double *q;
    double tol;
    i64 maxit;
};

struct BRes {
    i64 iters;
    double relres;
    double relres_true;
    int status;
    int pad;
};

// y = A x by one workgroup.  Every lane issues a batch of index/value loads
// (WB entries or diagonals) before the dependent x loads, and padding
// entries take their x operand from the zero word (+0 products, which leave
// the sums unchanged), so no load waits behind a branch.  Sums run in the
// same entry / diagonal order as one entry at a time.
constexpr int WB = 8;

__device__ __forceinline__ void wg_spmv(const BReq &R, const double *__restrict__ xin, double *__restrict__ yout) {
    const int tid = threadIdx.x;
    if (R.fmt == DSM_CSR) {
        const int L = R.lanes;
        const int per = BB / L;
        const int lane = tid % L;
        for (i64 row0 = 0; row0 < R.n; row0 += per) {
            const i64 row = row0 + tid / L;
            double s = 0;
            if (row < R.n) {
                const i64 e1 = R.rp[row + 1];
                for (i64 e0 = R.rp[row] + lane; e0 < e1; e0 += (i64)WB * L) {
                    i32 c[WB];
                    double v[WB];
#pragma unroll
                    for (int u = 0; u < WB; u++) {
                        const i64 e = e0 + (i64)u * L;
                        c[u] = *(e < e1 ? R.col + e : sentinel_ptr<i32>());
                        v[u] = *(e < e1 ? R.val + e : zero_ptr<double>());
                    }
#pragma unroll
                    for (int u = 0; u < WB; u++) s += v[u] * *(c[u] >= 0 ? xin + c[u] : zero_ptr<double>());
                }
            }
            for (int off = L >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
            if (row < R.n && lane == 0) yout[row] = s;
        }
    } else if (R.fmt == DSM_DIA) {
        // the offsets are zero-padded to a multiple of 16 entries
        for (i64 i = tid; i < R.n; i += BB) {
            double s = 0;
            for (i64 k0 = 0; k0 < R.ndiag; k0 += WB) {
                double v[WB], xv[WB];
#pragma unroll
                for (int u = 0; u < WB; u++) {
                    const i64 k = k0 + u;
                    const i64 j = i + R.offs[k];
                    const bool kin = k < R.ndiag;
                    v[u] = *(kin ? R.dval + k * R.pitch + i : zero_ptr<double>());
                    xv[u] = *(kin && j >= 0 && j < R.n ? xin + j : zero_ptr<double>());
                }
                // zero slots are no entries (as in the device-wide sweep);
                // the x operands are pinned as loaded so the select stays a
                // register select
#pragma unroll
                for (int u = 0; u < WB; u++) asm volatile("" : "+v"(xv[u]));
#pragma unroll
                for (int u = 0; u < WB; u++) s += v[u] * (v[u] != 0.0 ? xv[u] : 0.0);
            }
            yout[i] = s;
        }
    } else {  // ELL
        for (i64 i = tid; i < R.n; i += BB) {
            double s = 0;
            for (i64 k0 = 0; k0 < R.K; k0 += WB) {
                i32 c[WB];
                double v[WB];
#pragma unroll
                for (int u = 0; u < WB; u++) {
                    const i64 k = k0 + u;
                    c[u] = *(k < R.K ? R.ecol + k * R.pitch + i : sentinel_ptr<i32>());
                    v[u] = *(k < R.K ? R.evl + k * R.pitch + i : zero_ptr<double>());
                }
#pragma unroll
                for (int u = 0; u < WB; u++) s += v[u] * *(c[u] >= 0 ? xin + c[u] : zero_ptr<double>());
            }
            yout[i] = s;
        }
    }
}

__device__ void solve_one(const BReq &R, BRes *out, double *lds) {
    const int tid = threadIdx.x;
    const i64 n = R.n;
    wg_spmv(R, R.x, R.q);
    __syncthreads();
    double a = 0, c = 0;
    for (i64 i = tid; i < n; i += BB) {
        const double ri = R.b[i] - R.q[i];
        R.r[i] = ri;
        R.p[i] = ri;
        a += ri * ri;
        c += R.b[i] * R.b[i];
    }
    double rho = block_sum(a, lds);
    const double nb = sqrt(block_sum(c, lds));
    const double nr0 = sqrt(rho);
    int status = rho == 0 ? DSM_OK : (!isfinite(rho) ? DSM_E_BREAKDOWN : 1);  // 1 = running
    double relres = rho > 0 ? 1.0 : 0.0;
    i64 k = 0;
    while (status == 1) {
        if (k >= R.maxit) {
            status = DSM_E_NOT_CONVERGED;
            break;
        }
        __syncthreads();
        wg_spmv(R, R.p, R.q);
        __syncthreads();
        k++;
        a = 0;
        for (i64 i = tid; i < n; i += BB) a += R.p[i] * R.q[i];
        const double pq = block_sum(a, lds);
        if (!(pq > 0) || !isfinite(pq)) {
            status = DSM_E_BREAKDOWN;
            break;
        }
        const double alpha = rho / pq;
        a = 0;
        for (i64 i = tid; i < n; i += BB) {
            R.x[i] = R.x[i] + alpha * R.p[i];
            const double ri = R.r[i] - alpha * R.q[i];
            R.r[i] = ri;
            a += ri * ri;
        }
        const double rho1 = block_sum(a, lds);
        relres = nr0 > 0 ? sqrt(rho1) / nr0 : 0.0;
        if (!isfinite(rho1)) {
            status = DSM_E_BREAKDOWN;
            break;
        }
        if (sqrt(rho1) <= R.tol * nr0) {
            status = DSM_OK;
            break;
        }
        const double beta = rho1 / rho;
        for (i64 i = tid; i < n; i += BB) R.p[i] = R.r[i] + beta * R.p[i];
        rho = rho1;
    }
    __syncthreads();
    wg_spmv(R, R.x, R.q);
    __syncthreads();
    a = 0;
    for (i64 i = tid; i < n; i += BB) {
        const double ri = R.b[i] - R.q[i];
        a += ri * ri;
    }
    const double nrt = sqrt(block_sum(a, lds));
    if (tid == 0) {
        out->iters = k;
        out->relres = relres;
        out->relres_true = nb > 0 ? nrt / nb : nrt;
        out->status = status;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(BB) k_cg_batched(const BReq *__restrict__ reqs, BRes *__restrict__ res, int count,
                                                   int *next) {
    __shared__ double lds[BB / WAVE];
    __shared__ int sidx;
    for (;;) {
        if (threadIdx.x == 0) sidx = atomicAdd(next, 1);
        __syncthreads();
        const int idx = sidx;
        __syncthreads();
        if (idx >= count) return;
        const BReq R = reqs[idx];
        solve_one(R, &res[idx], lds);
    }
}

// ---------------------------------------------------------------- host side
bool batch_eligible(const dsm_matrix_s *m, i64 small_rows) {
    const Payload &P = m->P;
    return m->nrows == m->ncols && m->nrows <= small_rows && P.vdt == DSM_F64 &&
           (P.fmt == DSM_CSR || P.fmt == DSM_DIA || P.fmt == DSM_ELL);
}

static int default_lanes(const dsm_matrix_s *m, const Payload &P) {
    if (P.fmt != DSM_CSR) return 1;
    const double mean = m->nrows ? (double)P.csr_nnz / (double)m->nrows : 1.0;
    int L = 1;
    while (L < 32 && L < mean) L <<= 1;
    return L;
}

static size_t vec_bytes(i64 n) { return ((size_t)std::max<i64>(n, 1) * 8 + 255) & ~(size_t)255; }

// Arena bytes of one batch: a fixed part (the work counter and the 256-byte
// rounding of the descriptor and result arrays) plus one share per request.
size_t batch_request_bytes(i64 n) { return 3 * vec_bytes(n) + sizeof(BReq) + sizeof(BRes); }
size_t batch_arena_fixed() { return 1536; }

static BReq make_req(const dsm_matrix_s *m, const Payload &P, int lanes) {
    BReq R{};
    R.fmt = P.fmt;
    R.lanes = lanes;
    R.n = m->nrows;
    R.rp = P.rp;
    R.col = P.col;
    R.val = (const double *)P.val;
    R.offs = P.offs;
    R.ndiag = P.ndiag;
    R.pitch = P.pitch;
    R.dval = (const double *)P.dval;
    R.ecol = P.ecol;
    R.evl = (const double *)P.evl;
    R.K = P.K;
    return R;
}

// Lays out descriptors, results, counter and per-request vectors in `arena`,
// launches the persistent kernel on s and waits.
static void launch_reqs(dsm_ctx ctx, std::vector<BReq> &hreq, std::vector<BRes> &hres, Workspace &arena,
                        hipStream_t s) {
    const int count = (int)hreq.size();
    if (count == 0) return;
    size_t bytes = batch_arena_fixed();
    for (auto &R : hreq) bytes += batch_request_bytes(R.n);
    char *base = (char *)ws_get(ctx, arena, bytes, s);
    auto take = [&](size_t sz) {
        char *p = base;
        base += (sz + 255) & ~(size_t)255;
        return (void *)p;
    };
    int *next = (int *)take(sizeof(int));
    BReq *dreq = (BReq *)take(sizeof(BReq) * count);
    BRes *dres = (BRes *)take(sizeof(BRes) * count);
    for (auto &R : hreq) {
        R.r = (double *)take(vec_bytes(R.n));
        R.p = (double *)take(vec_bytes(R.n));
        R.q = (double *)take(vec_bytes(R.n));
    }
    hres.resize(count);
    DSM_HIP(hipMemcpyAsync(dreq, hreq.data(), sizeof(BReq) * count, hipMemcpyHostToDevice, s));
    DSM_HIP(hipMemsetAsync(next, 0, sizeof(int), s));
    int ncu = 256;
    DSM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const unsigned grid = (unsigned)std::min(count, ncu * 4);
    hipLaunchKernelGGL(k_cg_batched, dim3(grid), dim3(BB), 0, s, dreq, dres, count, next);
    DSM_HIP(hipGetLastError());
    DSM_HIP(hipMemcpyAsync(hres.data(), dres, sizeof(BRes) * count, hipMemcpyDeviceToHost, s));
    DSM_HIP(hipStreamSynchronize(s));
}

static void to_result(const BRes &r, dsm_cg_result *out) {
    dsm_cg_result R{};
    R.iters = r.iters;
    R.outer_iters = 0;
    R.relres = r.relres;
    R.relres_true = r.relres_true;
    R.status = r.status;
    *out = R;
}

void run_batch(dsm_ctx ctx, const BatchJob &job, dsm_cg_result *results, Workspace &arena, hipStream_t s) {
    const size_t count = job.mats.size();
    // longest first, so the tail of the batch is short systems
    std::vector<size_t> order(count);
    for (size_t k = 0; k < count; k++) order[k] = k;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t c) { return job.mats[a]->nrows > job.mats[c]->nrows; });
    std::vector<BReq> hreq;
    for (size_t k : order) {
        dsm_matrix m = job.mats[k];
        BReq R = make_req(m, m->P, m->P.fmt == DSM_CSR && m->batch_lanes > 0 ? m->batch_lanes
                                                                             : default_lanes(m, m->P));
        R.b = job.b[k];
        R.x = job.x[k];
        R.tol = job.opts[k].tol;
        R.maxit = job.opts[k].maxit > 0 ? job.opts[k].maxit : std::min<i64>(10 * std::max<i64>(m->nrows, 1), 20000);
        hreq.push_back(R);
    }
    std::vector<BRes> hres;
    launch_reqs(ctx, hreq, hres, arena, s);
    for (size_t i = 0; i < count; i++) to_result(hres[i], &results[order[i]]);
}

__global__ void k_ones(i64 n, double *v) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = 1.0;
}

double time_batched_solve(dsm_matrix m, const Payload &P, int lanes, int iters, hipStream_t s) {
    dsm_ctx ctx = m->ctx;
    const i64 n = m->nrows;
    void *v = dev_alloc(ctx, 2 * vec_bytes(n));
    double *b = (double *)v, *x = (double *)((char *)v + vec_bytes(n));
    Workspace arena;
    double us = 0;
    try {
        hipLaunchKernelGGL(k_ones, dim3(grid_for(n, 256)), dim3(256), 0, s, n, b);
        std::vector<BReq> hreq(1, make_req(m, P, lanes));
        hreq[0].b = b;
        hreq[0].x = x;
        hreq[0].tol = 0.0;  // run exactly `iters` iterations
        hreq[0].maxit = iters;
        std::vector<BRes> hres;
        hipEvent_t e0, e1;
        DSM_HIP(hipEventCreate(&e0));
        DSM_HIP(hipEventCreate(&e1));
        for (int rep = 0; rep < 3; rep++) {
            DSM_HIP(hipMemsetAsync(x, 0, 8 * (size_t)n, s));
            std::vector<BReq> r = hreq;
            DSM_HIP(hipEventRecord(e0, s));
            launch_reqs(ctx, r, hres, arena, s);
            DSM_HIP(hipEventRecord(e1, s));
            DSM_HIP(hipEventSynchronize(e1));
            float ms = 0;
            DSM_HIP(hipEventElapsedTime(&ms, e0, e1));
            us = rep == 0 ? ms * 1e3 : std::min(us, (double)ms * 1e3);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    } catch (...) {
        ws_release(ctx, arena);
        dev_free(ctx, v, 2 * vec_bytes(n));
        throw;
    }
    ws_release(ctx, arena);
    dev_free(ctx, v, 2 * vec_bytes(n));
    return us;
}

}  // namespace dsm

using namespace dsm;

DSM_API dsm_status dsm_cg_solve_batched(int32_t count, const dsm_matrix *mats, const double *const *b,
                                        double *const *x, const dsm_cg_opts *opts, dsm_cg_result *results,
                                        void *stream) {
    return guard([&] {
        DSM_CHECK(count >= 0, DSM_E_INVALID, "negative count");
        if (count == 0) return;
        DSM_CHECK(mats && b && x && opts && results, DSM_E_INVALID, "null argument");
        dsm_ctx ctx = nullptr;
        for (int k = 0; k < count; k++) {
            DSM_CHECK(mats[k] && mats[k]->ctx, DSM_E_INVALID, "null matrix handle");
            DSM_CHECK(mats[k]->nrows == mats[k]->ncols, DSM_E_UNSUPPORTED, "CG needs square matrices");
            DSM_CHECK(opts[k].mode == DSM_CG_F64, DSM_E_UNSUPPORTED, "batched solves are FP64 only");
            DSM_CHECK(opts[k].tol >= 0, DSM_E_INVALID, "negative tolerance");
            DSM_CHECK((b[k] && x[k]) || mats[k]->nrows == 0, DSM_E_INVALID, "null vector");
            if (!ctx) ctx = mats[k]->ctx;
            DSM_CHECK(mats[k]->ctx == ctx, DSM_E_INVALID, "all matrices must share one context");
        }
        DSM_HIP(hipSetDevice(ctx->device));
        hipStream_t s = (hipStream_t)stream;
        BatchJob job;
        std::vector<int> small, large;
        for (int k = 0; k < count; k++) {
            if (batch_eligible(mats[k], BATCH_SMALL_ROWS)) {
                small.push_back(k);
                job.mats.push_back(mats[k]);
                job.b.push_back(b[k]);
                job.x.push_back(x[k]);
                job.opts.push_back(opts[k]);
            } else {
                large.push_back(k);
            }
        }
        // large systems on a side stream, overlapping the batch
        hipStream_t side = nullptr;
        Workspace arena, cgws, spws;
        std::vector<dsm_cg_result> sres(small.size());
        auto cleanup = [&] {
            if (side) {
                (void)hipStreamSynchronize(side);
                (void)hipStreamDestroy(side);
            }
            (void)hipStreamSynchronize(s);
            ws_release(ctx, arena);
            ws_release(ctx, cgws);
            ws_release(ctx, spws);
        };
        try {
            if (!large.empty()) DSM_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
            if (!small.empty()) {
                // enqueue the batch first, then drive the large solves while it runs
                std::exception_ptr err;
                std::thread th([&] {
                    try {
                        DSM_HIP(hipSetDevice(ctx->device));
                        run_batch(ctx, job, sres.data(), arena, s);
                    } catch (...) {
                        err = std::current_exception();
                    }
                });
                try {
                    for (int k : large) cg_solve_ws(mats[k], b[k], x[k], opts[k], &results[k], side, cgws, spws, false);
                } catch (...) {
                    th.join();
                    throw;
                }
                th.join();
                if (err) std::rethrow_exception(err);
            } else {
                for (int k : large) cg_solve_ws(mats[k], b[k], x[k], opts[k], &results[k], side, cgws, spws, false);
            }
        } catch (...) {
            cleanup();
            throw;
        }
        cleanup();
        for (size_t i = 0; i < small.size(); i++) results[small[i]] = sres[i];
    });
}
