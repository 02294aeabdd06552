// C ABI: context, matrix lifecycle, conversion, inspection, export, SpMV.
#include <algorithm>
#include <cstdio>

#include "core.hpp"

namespace dsm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_cstr() { return g_last_error.c_str(); }
void clear_error() { g_last_error.clear(); }
void fail(dsm_status s, const std::string &msg) { throw Error{s, msg}; }

void *dev_alloc(dsm_ctx ctx, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (ctx->budget) {
        size_t cur = ctx->in_use.load();
        do {
            if (cur + bytes > ctx->budget)
                fail(DSM_E_NOMEM, "HBM budget exceeded: " + std::to_string(cur + bytes) + " > " +
                                      std::to_string(ctx->budget) + " bytes");
        } while (!ctx->in_use.compare_exchange_weak(cur, cur + bytes));
    } else {
        ctx->in_use += bytes;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ctx->in_use -= bytes;
        fail(DSM_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + ") failed: " + hipGetErrorString(e));
    }
    return p;
}

void dev_free(dsm_ctx ctx, void *p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    ctx->in_use -= bytes == 0 ? 16 : bytes;
}

static void drop_graph(Workspace &w) {
    if (w.graph) (void)hipGraphExecDestroy((hipGraphExec_t)w.graph);
    w.graph = nullptr;
    w.graph_key.clear();
}

void *ws_get(dsm_ctx ctx, Workspace &w, size_t bytes, hipStream_t s) {
    if (w.bytes >= bytes && w.p) return w.p;
    DSM_CHECK(!w.fixed, DSM_E_NOMEM, "workspace of fixed size too small");
    drop_graph(w);
    if (w.p) {
        DSM_HIP(hipStreamSynchronize(s));
        if (w.stream) DSM_HIP(hipStreamSynchronize(w.stream));
        dev_free(ctx, w.p, w.bytes);
        if (w.live) *w.live -= w.bytes;
        w.p = nullptr;
        w.bytes = 0;
    }
    const size_t b = w.grow_pow2 ? ws_round(bytes) : bytes;
    if (w.live) *w.live += b;
    try {
        w.p = dev_alloc(ctx, b);
    } catch (...) {
        if (w.live) *w.live -= b;
        throw;
    }
    w.bytes = b;
    return w.p;
}

void ws_release_host(Workspace &w) {
    drop_graph(w);
    if (w.stream) (void)hipStreamDestroy(w.stream);
    w.stream = nullptr;
    for (auto &e : w.events) {
        if (e) (void)hipEventDestroy((hipEvent_t)e);
        e = nullptr;
    }
    if (w.host) (void)hipHostFree(w.host);
    w.host = nullptr;
}

void ws_release(dsm_ctx ctx, Workspace &w) {
    ws_release_host(w);
    if (w.p) {
        dev_free(ctx, w.p, w.bytes);
        if (w.live) *w.live -= w.bytes;
    }
    w.p = nullptr;
    w.bytes = 0;
}

static void set_device(dsm_ctx ctx) { DSM_HIP(hipSetDevice(ctx->device)); }

static void check_matrix(dsm_matrix m) {
    DSM_CHECK(m != nullptr && m->ctx != nullptr, DSM_E_INVALID, "null matrix handle");
}

}  // namespace dsm

using namespace dsm;

DSM_API const char *dsm_status_string(dsm_status s) {
    switch (s) {
    case DSM_OK: return "ok";
    case DSM_E_INVALID: return "invalid argument";
    case DSM_E_NOMEM: return "out of device memory or HBM budget";
    case DSM_E_INFEASIBLE: return "format infeasible (padding ratio)";
    case DSM_E_UNSUPPORTED: return "unsupported";
    case DSM_E_NOT_CONVERGED: return "not converged";
    case DSM_E_BREAKDOWN: return "breakdown";
    case DSM_E_PENDING: return "pending";
    case DSM_E_DEVICE: return "device error";
    }
    return "unknown status";
}

DSM_API const char *dsm_last_error(void) { return last_error_cstr(); }

DSM_API int32_t dsm_version(void) { return 10000; }

DSM_API dsm_status dsm_ctx_create(int device, size_t hbm_budget_bytes, dsm_ctx *out) {
    return guard([&] {
        DSM_CHECK(out != nullptr, DSM_E_INVALID, "out is null");
        int n = 0;
        DSM_HIP(hipGetDeviceCount(&n));
        DSM_CHECK(device >= 0 && device < n, DSM_E_INVALID, "no such device");
        DSM_HIP(hipSetDevice(device));
        hipDeviceProp_t prop;
        DSM_HIP(hipGetDeviceProperties(&prop, device));
        DSM_CHECK(std::string(prop.gcnArchName).rfind("gfx950", 0) == 0, DSM_E_UNSUPPORTED,
                  std::string("library built for gfx950, device is ") + prop.gcnArchName);
        noalloc_scratch_init(device);
        auto *c = new dsm_ctx_s();
        c->device = device;
        c->budget = hbm_budget_bytes;
        *out = c;
    });
}

DSM_API dsm_status dsm_ctx_destroy(dsm_ctx ctx) {
    return guard([&] {
        if (!ctx) return;
        DSM_CHECK(ctx->live_matrices.load() == 0, DSM_E_INVALID, "context still has live matrices");
        delete ctx;
    });
}

DSM_API dsm_status dsm_ctx_bytes_in_use(dsm_ctx ctx, size_t *out) {
    return guard([&] {
        DSM_CHECK(ctx && out, DSM_E_INVALID, "null argument");
        *out = ctx->in_use.load();
    });
}

static void check_dims(int64_t nrows, int64_t ncols, int64_t nnz) {
    DSM_CHECK(nrows >= 0 && ncols >= 0 && nnz >= 0, DSM_E_INVALID, "negative size");
    DSM_CHECK(nrows < INT32_MAX && ncols < INT32_MAX && nnz < INT32_MAX, DSM_E_INVALID,
              "sizes must fit int32 indices");
}

static dsm_matrix new_matrix(dsm_ctx ctx, int64_t nrows, int64_t ncols, int64_t nnz) {
    auto *m = new dsm_matrix_s();
    m->ctx = ctx;
    m->nrows = nrows;
    m->ncols = ncols;
    m->nnz = nnz;
    ctx->live_matrices++;
    return m;
}

static void free_matrix(dsm_matrix m) {
    (void)hipDeviceSynchronize();
    m->P.release(m->ctx);
    ws_release(m->ctx, m->ws);
    ws_release(m->ctx, m->cgws);
    m->ctx->live_matrices--;
    delete m;
}

DSM_API dsm_status dsm_create_csr(dsm_ctx ctx, int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *row_ptr,
                                  const int32_t *col, const double *val, int on_device, void *stream,
                                  dsm_matrix *out) {
    dsm_matrix m = nullptr;
    dsm_status st = guard([&] {
        DSM_CHECK(ctx && out, DSM_E_INVALID, "null argument");
        check_dims(nrows, ncols, nnz);
        DSM_CHECK(row_ptr && (nnz == 0 || (col && val)), DSM_E_INVALID, "null array");
        set_device(ctx);
        hipStream_t s = (hipStream_t)stream;
        m = new_matrix(ctx, nrows, ncols, nnz);
        Payload &P = m->P;
        P.fmt = DSM_CSR;
        P.vdt = DSM_F64;
        P.csr_nnz = nnz;
        P.rp = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)(nrows + 1));
        P.col = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)nnz);
        P.val = P.alloc(ctx, sizeof(double) * (size_t)nnz);
        hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        DSM_HIP(hipMemcpyAsync(P.rp, row_ptr, sizeof(i32) * (size_t)(nrows + 1), k, s));
        if (nnz) {
            DSM_HIP(hipMemcpyAsync(P.col, col, sizeof(i32) * (size_t)nnz, k, s));
            DSM_HIP(hipMemcpyAsync(P.val, val, sizeof(double) * (size_t)nnz, k, s));
        }
        validate_csr(ctx, nrows, ncols, nnz, P.rp, P.col, s);
        build_row_blocks(ctx, P, nrows, s);
        DSM_HIP(hipStreamSynchronize(s));
        m->last_stream = s;
        *out = m;
    });
    if (st != DSM_OK && m) free_matrix(m);
    return st;
}

DSM_API dsm_status dsm_create_coo(dsm_ctx ctx, int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *row,
                                  const int32_t *col, const double *val, int sorted, int on_device, void *stream,
                                  dsm_matrix *out) {
    dsm_matrix m = nullptr;
    dsm_status st = guard([&] {
        DSM_CHECK(ctx && out, DSM_E_INVALID, "null argument");
        check_dims(nrows, ncols, nnz);
        DSM_CHECK(nnz == 0 || (row && col && val), DSM_E_INVALID, "null array");
        set_device(ctx);
        hipStream_t s = (hipStream_t)stream;
        m = new_matrix(ctx, nrows, ncols, nnz);
        const i32 *drow = row, *dcol = col;
        const double *dval = val;
        Payload staging;
        if (!on_device) {
            staging.crow = (i32 *)staging.alloc(ctx, sizeof(i32) * (size_t)nnz);
            staging.ccol = (i32 *)staging.alloc(ctx, sizeof(i32) * (size_t)nnz);
            staging.cval = staging.alloc(ctx, sizeof(double) * (size_t)nnz);
            if (nnz) {
                DSM_HIP(hipMemcpyAsync(staging.crow, row, sizeof(i32) * (size_t)nnz, hipMemcpyHostToDevice, s));
                DSM_HIP(hipMemcpyAsync(staging.ccol, col, sizeof(i32) * (size_t)nnz, hipMemcpyHostToDevice, s));
                DSM_HIP(hipMemcpyAsync(staging.cval, val, sizeof(double) * (size_t)nnz, hipMemcpyHostToDevice, s));
            }
            drow = staging.crow;
            dcol = staging.ccol;
            dval = (const double *)staging.cval;
        }
        try {
            m->P = coo_to_csr_payload(m, drow, dcol, dval, nnz, sorted != 0, s);
        } catch (...) {
            (void)hipStreamSynchronize(s);
            staging.release(ctx);
            throw;
        }
        DSM_HIP(hipStreamSynchronize(s));
        staging.release(ctx);
        m->last_stream = s;
        *out = m;
    });
    if (st != DSM_OK && m) free_matrix(m);
    return st;
}

DSM_API dsm_status dsm_matrix_destroy(dsm_matrix m) {
    return guard([&] {
        if (!m) return;
        set_device(m->ctx);
        free_matrix(m);
    });
}

DSM_API void dsm_convert_opts_default(dsm_convert_opts *o) {
    if (!o) return;
    o->value_dtype = DSM_F64;
    o->hdc_theta = 0.5;
    o->max_pad_ratio = 16.0;
    o->hyb_width = -1;
}

namespace dsm {
// Shared by dsm_convert and the selector: build `fmt` from the current
// payload without touching it.
Payload build_format(dsm_matrix m, int fmt, const dsm_convert_opts &o, hipStream_t s) {
    const Payload &cur = m->P;
    if (cur.fmt == DSM_CSR) return from_csr(m, cur, fmt, o.value_dtype, o, s);
    if (fmt == DSM_CSR) {
        Payload c = to_csr(m, cur, s);
        if (c.vdt == o.value_dtype) return c;
        Payload d;
        try {
            d = cast_csr(m, c, o.value_dtype, s);
        } catch (...) {
            c.release(m->ctx);
            throw;
        }
        c.release(m->ctx);
        return d;
    }
    Payload c = to_csr(m, cur, s);
    Payload out;
    try {
        out = from_csr(m, c, fmt, o.value_dtype, o, s);
    } catch (...) {
        c.release(m->ctx);
        throw;
    }
    c.release(m->ctx);
    return out;
}
}  // namespace dsm

DSM_API dsm_status dsm_convert(dsm_matrix m, dsm_format fmt, const dsm_convert_opts *opts, void *stream) {
    return guard([&] {
        check_matrix(m);
        DSM_CHECK((int)fmt >= 0 && (int)fmt < DSM_NUM_FORMATS, DSM_E_INVALID, "unknown format");
        set_device(m->ctx);
        dsm_convert_opts o;
        dsm_convert_opts_default(&o);
        o.value_dtype = (dsm_dtype)m->P.vdt;
        if (opts) o = *opts;
        DSM_CHECK(o.value_dtype >= DSM_F64 && o.value_dtype <= DSM_BF16, DSM_E_INVALID, "unknown value dtype");
        hipStream_t s = (hipStream_t)stream;
        if ((int)fmt == m->P.fmt && o.value_dtype == m->P.vdt &&
            !(fmt == DSM_HDC && o.hdc_theta > 0 && o.hdc_theta != m->P.theta) && !(fmt == DSM_HYB && o.hyb_width >= 0))
            return;  // already active
        Payload np = build_format(m, (int)fmt, o, s);
        DSM_HIP(hipStreamSynchronize(s));
        m->P.release(m->ctx);
        m->P = np;
        if (fmt == DSM_CSR) m->nnz = np.csr_nnz;
        if (m->P.fmt != DSM_CSR || m->variant >= CSR_VARIANTS) m->variant = 0;
        m->last_stream = s;
    });
}

DSM_API dsm_status dsm_get_info(dsm_matrix m, dsm_info *out) {
    return guard([&] {
        check_matrix(m);
        DSM_CHECK(out, DSM_E_INVALID, "out is null");
        const Payload &P = m->P;
        dsm_info i{};
        i.format = P.fmt;
        i.value_dtype = P.vdt;
        i.nrows = m->nrows;
        i.ncols = m->ncols;
        i.nnz = m->nnz;
        i.ndiag = (P.fmt == DSM_DIA || P.fmt == DSM_HDC) ? P.ndiag : 0;
        i.ell_width = (P.fmt == DSM_ELL || P.fmt == DSM_HYB) ? P.K : 0;
        i.coo_nnz = (P.fmt == DSM_COO || P.fmt == DSM_HYB) ? P.coo_nnz : 0;
        i.csr_nnz = (P.fmt == DSM_CSR || P.fmt == DSM_HDC) ? P.csr_nnz : 0;
        i.bytes = (int64_t)P.bytes;
        i.pitch = P.pitch;
        i.hdc_theta = P.fmt == DSM_HDC ? P.theta : 0.0;
        *out = i;
    });
}

static void copy_strided(void *dst, const void *src, size_t elem, int64_t rows, int64_t pitch, int64_t nslices,
                         hipStream_t s) {
    if (rows == 0 || nslices == 0) return;
    DSM_HIP(hipMemcpy2DAsync(dst, elem * (size_t)rows, src, elem * (size_t)pitch, elem * (size_t)rows,
                             (size_t)nslices, hipMemcpyDeviceToHost, s));
}

DSM_API dsm_status dsm_export(dsm_matrix m, const dsm_export_bufs *b, void *stream) {
    return guard([&] {
        check_matrix(m);
        DSM_CHECK(b, DSM_E_INVALID, "bufs is null");
        set_device(m->ctx);
        hipStream_t s = (hipStream_t)stream;
        const Payload &P = m->P;
        const size_t v = dtype_size(P.vdt);
        const int64_t n = m->nrows;
        auto d2h = [&](void *dst, const void *src, size_t bytes) {
            if (bytes == 0) return;
            DSM_CHECK(dst != nullptr, DSM_E_INVALID, "export buffer missing for the active format");
            DSM_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
        };
        auto need = [&](const void *p) { DSM_CHECK(p != nullptr, DSM_E_INVALID, "export buffer missing"); };
        switch (P.fmt) {
        case DSM_CSR:
        case DSM_HDC:
            need(b->row_ptr);
            d2h(b->row_ptr, P.rp, sizeof(i32) * (size_t)(n + 1));
            d2h(b->col, P.col, sizeof(i32) * (size_t)P.csr_nnz);
            d2h(b->val, P.val, v * (size_t)P.csr_nnz);
            break;
        default:
            break;
        }
        if (P.fmt == DSM_COO || P.fmt == DSM_HYB) {
            d2h(b->row, P.crow, sizeof(i32) * (size_t)P.coo_nnz);
            d2h(b->col, P.ccol, sizeof(i32) * (size_t)P.coo_nnz);
            d2h(b->val, P.cval, v * (size_t)P.coo_nnz);
        }
        if (P.fmt == DSM_DIA || P.fmt == DSM_HDC) {
            d2h(b->offsets, P.offs, sizeof(i32) * (size_t)P.ndiag);
            if (P.ndiag && n) need(b->dia_val);
            copy_strided(b->dia_val, P.dval, v, n, P.pitch, P.ndiag, s);
        }
        if (P.fmt == DSM_ELL || P.fmt == DSM_HYB) {
            if (P.K && n) {
                need(b->ell_col);
                need(b->ell_val);
            }
            copy_strided(b->ell_col, P.ecol, sizeof(i32), n, P.pitch, P.K, s);
            copy_strided(b->ell_val, P.evl, v, n, P.pitch, P.K, s);
        }
        DSM_HIP(hipStreamSynchronize(s));
    });
}

DSM_API dsm_status dsm_row_stats(dsm_matrix m, int64_t *out, void *stream) {
    return guard([&] {
        check_matrix(m);
        DSM_CHECK(out, DSM_E_INVALID, "out is null");
        set_device(m->ctx);
        row_stats(m, out, (hipStream_t)stream);
    });
}

DSM_API dsm_status dsm_values_exact(dsm_matrix m, dsm_dtype to, int32_t *exact, void *stream) {
    return guard([&] {
        check_matrix(m);
        DSM_CHECK(exact, DSM_E_INVALID, "exact is null");
        DSM_CHECK(to == DSM_F64 || to == DSM_F32 || to == DSM_BF16, DSM_E_INVALID, "unknown value dtype");
        set_device(m->ctx);
        *exact = values_exact(m, to, (hipStream_t)stream) ? 1 : 0;
    });
}

DSM_API dsm_status dsm_spmv(dsm_matrix m, const void *x, void *y, dsm_dtype vec_dtype, void *stream) {
    return guard([&] {
        check_matrix(m);
        DSM_CHECK((x || m->ncols == 0) && (y || m->nrows == 0), DSM_E_INVALID, "null vector");
        DSM_CHECK(x != y || m->nrows == 0, DSM_E_INVALID, "x and y must not alias");
        hipStream_t s = (hipStream_t)stream;
        spmv(m, m->P, x, y, vec_dtype, m->variant, s);
        m->last_stream = s;
    });
}

DSM_API dsm_status dsm_spmv_noalloc(dsm_matrix m, const void *x, void *y, dsm_dtype vec_dtype, void *stream) {
    return guard([&] {
        check_matrix(m);
        DSM_CHECK((x || m->ncols == 0) && (y || m->nrows == 0), DSM_E_INVALID, "null vector");
        DSM_CHECK(x != y || m->nrows == 0, DSM_E_INVALID, "x and y must not alias");
        hipStream_t s = (hipStream_t)stream;
        spmv_noalloc(m, x, y, vec_dtype, s);
        m->last_stream = s;
    });
}

DSM_API dsm_status dsm_spmv_accumulate(dsm_matrix m, const void *x, void *y, dsm_dtype vec_dtype, void *stream) {
    return guard([&] {
        check_matrix(m);
        DSM_CHECK((x || m->ncols == 0) && (y || m->nrows == 0), DSM_E_INVALID, "null vector");
        DSM_CHECK(x != y || m->nrows == 0, DSM_E_INVALID, "x and y must not alias");
        hipStream_t s = (hipStream_t)stream;
        spmv(m, m->P, x, y, vec_dtype, m->variant, s, nullptr, nullptr, true);
        m->last_stream = s;
    });
}

DSM_API dsm_status dsm_set_variant(dsm_matrix m, int32_t variant) {
    return guard([&] {
        check_matrix(m);
        const int f = m->P.fmt;
        int maxv = f == DSM_CSR ? CSR_VARIANTS
                   : (f == DSM_COO ? 1 : ((f == DSM_DIA || f == DSM_HDC) ? DIA_VARIANT_COUNT : SWEEP_VARIANT_COUNT));
        DSM_CHECK(variant >= 0 && variant < maxv, DSM_E_INVALID, "no such kernel variant for this format");
        m->variant = variant;
    });
}

DSM_API dsm_status dsm_get_variant(dsm_matrix m, int32_t *variant) {
    return guard([&] {
        check_matrix(m);
        DSM_CHECK(variant, DSM_E_INVALID, "out is null");
        *variant = m->variant;
    });
}
