// Diagonal extraction and update for every format (the paper lists both
// among the matrix operations, Section III-D; HPCG's TestCG edits the
// diagonal of the system matrix, Section IV-B).
//
// d[i] = A(i, i) for i < min(nrows, ncols); 0 where the structure has no
// diagonal entry.  An update writes A(i, i) = d[i] (rounded to the value
// dtype) into every diagonal entry the structure holds; a non-zero d[i] for
// an entry the structure lacks makes the call fail before anything changes.
#include <algorithm>

#include "core.hpp"

namespace dsm {

constexpr int DB = 256;

template <class V>
__device__ __forceinline__ double to_f64(V v) {
    return (double)v;
}
template <>
__device__ __forceinline__ double to_f64<bf16>(bf16 v) {
    return (double)bf16_to_float(v);
}
template <class V>
__device__ __forceinline__ V from_f64(double d);
template <>
__device__ __forceinline__ double from_f64<double>(double d) {
    return d;
}
template <>
__device__ __forceinline__ float from_f64<float>(double d) {
    return (float)d;
}
template <>
__device__ __forceinline__ bf16 from_f64<bf16>(double d) {
    return float_to_bf16((float)d);
}

// Index of the diagonal entry of row i in a sorted CSR row, or -1.
__device__ __forceinline__ i64 csr_find(const i32 *rp, const i32 *col, i64 i) {
    i64 lo = rp[i], hi = (i64)rp[i + 1] - 1;
    while (lo <= hi) {
        const i64 mid = (lo + hi) >> 1;
        const i32 c = col[mid];
        if (c == i) return mid;
        if (c < i) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// Index k of offset 0 in a DIA offset array, or -1 (offsets are few).
__device__ __forceinline__ i64 dia_main(const i32 *offs, i64 nd) {
    for (i64 k = 0; k < nd; k++)
        if (offs[k] == 0) return k;
    return -1;
}

// mode 0: extract into d; mode 1: count entries missing where d != 0;
// mode 2: write d into the entries present.
template <class V>
__global__ void k_diag_csr(i64 nd, const i32 *rp, const i32 *col, V *val, double *d, int mode, int *missing,
                           bool partial) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    const i64 e = csr_find(rp, col, i);
    if (mode == 0) {
        if (e >= 0) d[i] = to_f64(val[e]);
        else if (!partial) d[i] = 0.0;
    } else if (mode == 1) {
        if (e < 0 && d[i] != 0.0) atomicAdd(missing, 1);
    } else if (e >= 0) {
        val[e] = from_f64<V>(d[i]);
    }
}

template <class V>
__global__ void k_diag_coo(i64 nnz, const i32 *row, const i32 *col, V *val, double *d, int mode, int *present) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz || row[k] != col[k]) return;
    const i32 i = row[k];
    if (mode == 0) d[i] = to_f64(val[k]);
    else if (mode == 1) present[i] = 1;
    else val[k] = from_f64<V>(d[i]);
}

template <class V>
__global__ void k_diag_dia(i64 nd, i64 ndiag, const i32 *offs, V *dval, i64 pitch, double *d, int mode,
                           int *missing) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    const i64 k = dia_main(offs, ndiag);
    if (mode == 0) d[i] = k >= 0 ? to_f64(dval[k * pitch + i]) : 0.0;
    else if (mode == 1) {
        if (k < 0 && d[i] != 0.0) atomicAdd(missing, 1);
    } else if (k >= 0) {
        dval[k * pitch + i] = from_f64<V>(d[i]);
    }
}

// ELL rows (+ optionally the HYB COO part is handled separately)
template <class V>
__global__ void k_diag_ell(i64 nd, i64 K, i64 pitch, const i32 *ecol, V *evl, double *d, int mode, int *present) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    i64 e = -1;
    for (i64 k = 0; k < K; k++)
        if (ecol[k * pitch + i] == i) e = k * pitch + i;
    if (mode == 0) d[i] = e >= 0 ? to_f64(evl[e]) : 0.0;
    else if (mode == 1) {
        if (e >= 0) present[i] = 1;
    } else if (e >= 0) {
        evl[e] = from_f64<V>(d[i]);
    }
}

// HDC: the diagonal lives in the DIA part when offset 0 is a true diagonal,
// otherwise in the CSR part.
__global__ void k_diag_presence_hdc(i64 nd, i64 ndiag, const i32 *offs, const i32 *rp, const i32 *col,
                                    int *present) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nd) present[i] = (dia_main(offs, ndiag) >= 0 || csr_find(rp, col, i) >= 0) ? 1 : 0;
}

__global__ void k_count_missing(i64 nd, const int *present, const double *d, int *missing) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nd && !present[i] && d[i] != 0.0) atomicAdd(missing, 1);
}

template <class V>
static void diag_typed(dsm_matrix m, double *d, int mode, hipStream_t s) {
    Payload &P = m->P;
    const i64 nd = std::min(m->nrows, m->ncols);
    if (nd == 0) return;
    const dim3 g(grid_for(nd, DB)), b(DB);
    dsm_ctx ctx = m->ctx;
    // work buffer: [0] missing counter, [1..nd] presence flags
    int *w = (int *)dev_alloc(ctx, sizeof(int) * (size_t)(nd + 1));
    int *missing = w, *present = w + 1;
    auto cleanup = [&] { dev_free(ctx, w, sizeof(int) * (size_t)(nd + 1)); };
    try {
        auto run = [&](int md) {
            switch (P.fmt) {
            case DSM_CSR:
                hipLaunchKernelGGL(k_diag_csr<V>, g, b, 0, s, nd, P.rp, P.col, (V *)P.val, d, md, missing, false);
                break;
            case DSM_COO:
                hipLaunchKernelGGL(k_diag_coo<V>, dim3(grid_for(P.coo_nnz, DB)), b, 0, s, P.coo_nnz, P.crow, P.ccol,
                                   (V *)P.cval, d, md, present);
                break;
            case DSM_DIA:
                hipLaunchKernelGGL(k_diag_dia<V>, g, b, 0, s, nd, P.ndiag, P.offs, (V *)P.dval, P.pitch, d, md,
                                   missing);
                break;
            case DSM_HDC:
                // DIA part first (0 where offset 0 is not a true diagonal);
                // the CSR part then fills or writes the rows whose entry it holds
                hipLaunchKernelGGL(k_diag_dia<V>, g, b, 0, s, nd, P.ndiag, P.offs, (V *)P.dval, P.pitch, d, md,
                                   missing);
                hipLaunchKernelGGL(k_diag_csr<V>, g, b, 0, s, nd, P.rp, P.col, (V *)P.val, d, md, missing, true);
                break;
            case DSM_ELL:
            case DSM_HYB:
                hipLaunchKernelGGL(k_diag_ell<V>, g, b, 0, s, nd, P.K, P.pitch, P.ecol, (V *)P.evl, d, md, present);
                if (P.fmt == DSM_HYB && P.coo_nnz > 0)
                    hipLaunchKernelGGL(k_diag_coo<V>, dim3(grid_for(P.coo_nnz, DB)), b, 0, s, P.coo_nnz, P.crow,
                                       P.ccol, (V *)P.cval, d, md, present);
                break;
            }
            DSM_HIP(hipGetLastError());
        };
        if (mode == 0) {
            if (P.fmt == DSM_COO) DSM_HIP(hipMemsetAsync(d, 0, sizeof(double) * (size_t)nd, s));
            run(0);
            DSM_HIP(hipStreamSynchronize(s));
            cleanup();
            return;
        }
        // update: check first, then write
        DSM_HIP(hipMemsetAsync(w, 0, sizeof(int) * (size_t)(nd + 1), s));
        int bad = 0;
        if (P.fmt == DSM_HDC) {
            // present = main diagonal in the DIA part, or entry in the CSR part
            hipLaunchKernelGGL(k_diag_presence_hdc, g, b, 0, s, nd, P.ndiag, P.offs, P.rp, P.col, present);
            hipLaunchKernelGGL(k_count_missing, g, b, 0, s, nd, present, d, missing);
        } else if (P.fmt == DSM_COO || P.fmt == DSM_ELL || P.fmt == DSM_HYB) {
            run(1);
            hipLaunchKernelGGL(k_count_missing, g, b, 0, s, nd, present, d, missing);
        } else {
            run(1);
        }
        DSM_HIP(hipGetLastError());
        DSM_HIP(hipMemcpyAsync(&bad, missing, sizeof(int), hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
        DSM_CHECK(bad == 0, DSM_E_INVALID,
                  std::to_string(bad) + " diagonal entries are absent from the structure but asked to be non-zero");
        run(2);
        DSM_HIP(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipStreamSynchronize(s);
        cleanup();
        throw;
    }
    cleanup();
}

void diagonal_op(dsm_matrix m, double *d, int mode, hipStream_t s) {
    switch (m->P.vdt) {
    case DSM_F64: diag_typed<double>(m, d, mode, s); break;
    case DSM_F32: diag_typed<float>(m, d, mode, s); break;
    default: diag_typed<bf16>(m, d, mode, s); break;
    }
}

}  // namespace dsm

using namespace dsm;

DSM_API dsm_status dsm_extract_diagonal(dsm_matrix m, double *d, void *stream) {
    return guard([&] {
        DSM_CHECK(m && m->ctx, DSM_E_INVALID, "null matrix handle");
        DSM_CHECK(d || std::min(m->nrows, m->ncols) == 0, DSM_E_INVALID, "null vector");
        DSM_HIP(hipSetDevice(m->ctx->device));
        diagonal_op(m, d, 0, (hipStream_t)stream);
    });
}

DSM_API dsm_status dsm_update_diagonal(dsm_matrix m, const double *d, void *stream) {
    return guard([&] {
        DSM_CHECK(m && m->ctx, DSM_E_INVALID, "null matrix handle");
        DSM_CHECK(d || std::min(m->nrows, m->ncols) == 0, DSM_E_INVALID, "null vector");
        DSM_HIP(hipSetDevice(m->ctx->device));
        diagonal_op(m, const_cast<double *>(d), 1, (hipStream_t)stream);
    });
}
