// On-device format conversions (the "convert" operation: an element-wise
// copy between storage formats in the same memory space).
//
// Canonical CSR is the hub: every format is built from CSR and turned back
// into CSR with prefix scans, so each conversion is a handful of coalesced
// sweeps plus one scan and needs no sort.  Values are moved as raw bit
// patterns (64/32/16-bit words); the only arithmetic on values is the
// explicit narrowing cast (FP64 -> FP32 -> BF16, round to nearest even).
// Results are canonical encodings, identical bit for bit whatever the launch
// shape:
//   COO  sorted by (row, col)
//   DIA  offsets = ascending distinct (col - row); slot (k, i) holds
//        A(i, i + off_k) or +0; diagonal-major with a padded pitch
//   ELL  K = longest row; slot (k, i) = k-th entry of row i, empty slots
//        col -1 / value +0
//   HYB  ELL of width K_h (largest k reached by >= ceil(nrows/3) rows) plus
//        the remaining entries as sorted COO
//   HDC  DIA over diagonals with count >= theta * length, CSR for the rest
#include <algorithm>
#include <vector>

#include "clusters.hpp"
#include "core.hpp"

namespace dsm {

constexpr int CB = 256;        // threads per workgroup
constexpr int EB_ROWS = 256;   // rows per workgroup when walking entries
constexpr int CB_U = 8;        // entries a row-per-thread kernel loads per batch
constexpr int RB_T = 1024;     // adaptive CSR: nnz bucket per row block
constexpr int RB_RCAP = 256;   // adaptive CSR: max rows per block

static i64 pitch_for(i64 nrows) { return ((nrows + 63) / 64) * 64; }

// Raw storage word for a value dtype.
template <int DT> struct Word;
template <> struct Word<DSM_F64> { using T = u64; };
template <> struct Word<DSM_F32> { using T = u32; };
template <> struct Word<DSM_BF16> { using T = uint16_t; };

// +0 and -0 have all bits but the sign clear.
template <class W>
__device__ __forceinline__ bool word_is_zero(W w) {
    return (W)(w << 1) == 0;
}

// Calls f(row, entry) for every entry of rows [blockIdx.x*EB_ROWS, +EB_ROWS).
template <class F>
__device__ __forceinline__ void for_each_entry(i64 nrows, const i32 *rp, F f) {
    __shared__ i32 srp[EB_ROWS + 1];
    const i64 r0 = (i64)blockIdx.x * EB_ROWS;
    const int nr = (int)min((i64)EB_ROWS, nrows - r0);
    for (int t = threadIdx.x; t <= nr; t += blockDim.x) srp[t] = rp[r0 + t];
    __syncthreads();
    const i64 e0 = srp[0], e1 = srp[nr];
    for (i64 e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        int lo = 0, hi = nr;  // invariant: srp[lo] <= e < srp[hi]
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if ((i64)srp[mid] <= e) lo = mid;
            else hi = mid;
        }
        f(r0 + lo, e);
    }
}

static unsigned entry_grid(i64 nrows) { return grid_for(nrows, EB_ROWS); }

// Privatised counting for histograms whose keys repeat heavily inside a
// workgroup (the diagonals of a banded matrix, the row lengths of a regular
// one): one global atomic per entry on a handful of bins serialises at the
// memory side (about 15 ms for the 29.8M entries of HPCG 104^3).  Counts go
// to an open-addressing table in LDS instead and reach the global bins once
// per workgroup and key; a key that finds no free slot within HT_PROBES goes
// straight to its global bin.  Keys are non-negative int32 (-1 = empty).
constexpr int HT_LOG = 11, HT = 1 << HT_LOG, HT_PROBES = 8;

__device__ __forceinline__ void ht_init(i32 *hk, i32 *hv) {
    for (int t = threadIdx.x; t < HT; t += blockDim.x) {
        hk[t] = -1;
        hv[t] = 0;
    }
    __syncthreads();
}

__device__ __forceinline__ void ht_add(i32 *hk, i32 *hv, i32 key, i32 *global) {
    unsigned h = ((unsigned)key * 2654435761u) >> (32 - HT_LOG);
    for (int probe = 0; probe < HT_PROBES; probe++, h = (h + 1) & (HT - 1)) {
        i32 k = __atomic_load_n(&hk[h], __ATOMIC_RELAXED);
        if (k == -1) {
            k = atomicCAS(&hk[h], -1, key);
            if (k == -1) k = key;
        }
        if (k == key) {
            atomicAdd(&hv[h], 1);
            return;
        }
    }
    atomicAdd(&global[key], 1);
}

// after a barrier that follows every ht_add of the workgroup
__device__ __forceinline__ void ht_flush(const i32 *hk, const i32 *hv, i32 *global) {
    for (int t = threadIdx.x; t < HT; t += blockDim.x)
        if (hk[t] >= 0 && hv[t] > 0) atomicAdd(&global[hk[t]], hv[t]);
}

// ---------------------------------------------------------------- validation
// err: bit 0 row_ptr[0] != 0, bit 1 row_ptr[n] != nnz, bit 2 decreasing or
// out-of-range pointers, bit 3 column out of range, bit 4 columns not
// strictly ascending (duplicates included).
__global__ void k_validate_csr(i64 nrows, i64 ncols, i64 nnz, const i32 *rp, const i32 *col, int *err) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (rp[0] != 0) atomicOr(err, 1);
        if ((i64)rp[nrows] != nnz) atomicOr(err, 2);
    }
    if (i >= nrows) return;
    i64 a = rp[i], b = rp[i + 1];
    if (a < 0 || b < a || b > nnz) {
        atomicOr(err, 4);
        return;
    }
    // CB_U columns loaded together (indices clamped into the row, so every
    // load is unconditional), then checked in order
    i32 prev = -1;
    int bad = 0;
    for (i64 k0 = a; k0 < b; k0 += CB_U) {
        i32 c[CB_U];
#pragma unroll
        for (int u = 0; u < CB_U; u++) c[u] = col[min(k0 + u, b - 1)];
#pragma unroll
        for (int u = 0; u < CB_U; u++)
            if (k0 + u < b) {
                if (c[u] < 0 || (i64)c[u] >= ncols) bad |= 8;
                if (c[u] <= prev) bad |= 16;
                prev = c[u];
            }
    }
    if (bad) atomicOr(err, bad);
}

static int read_flag(int *d, hipStream_t s) {
    int h = 0;
    DSM_HIP(hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, s));
    DSM_HIP(hipStreamSynchronize(s));
    return h;
}

// RAII scratch allocation (freed on scope exit, after a stream sync by caller).
// hipFree waits for the device, so no work still reading the buffer can
// outlive it.
struct Tmp {
    dsm_ctx ctx;
    void *p = nullptr;
    size_t n = 0;
    Tmp(dsm_ctx c, size_t bytes) : ctx(c), n(bytes ? bytes : 16) { p = dev_alloc(ctx, n); }
    ~Tmp() {
        if (p) dev_free(ctx, p, n);
    }
    template <class T> T *as() { return (T *)p; }
};

void validate_csr(dsm_ctx ctx, i64 nrows, i64 ncols, i64 nnz, const i32 *rp, const i32 *col, hipStream_t s) {
    Tmp err(ctx, sizeof(int));
    DSM_HIP(hipMemsetAsync(err.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_validate_csr, dim3(grid_for(nrows, CB)), dim3(CB), 0, s, nrows, ncols, nnz, rp, col,
                       err.as<int>());
    DSM_HIP(hipGetLastError());
    int f = read_flag(err.as<int>(), s);
    if (f) {
        std::string why;
        if (f & 1) why += " row_ptr[0] != 0;";
        if (f & 2) why += " row_ptr[nrows] != nnz;";
        if (f & 4) why += " row pointers decrease or leave [0, nnz];";
        if (f & 8) why += " column index out of range;";
        if (f & 16) why += " columns not strictly ascending within a row (unsorted or duplicate);";
        fail(DSM_E_INVALID, "invalid CSR:" + why);
    }
}

// ---------------------------------------------------------------- row blocks
// Row i opens a block when its first entry falls in another RB_T-bucket than
// row i-1's, when row i or row i-1 is longer than RB_T (long rows stand
// alone), or at every multiple of RB_RCAP.  Every block therefore holds fewer
// than 2*RB_T entries and at most RB_RCAP rows, or is one long row.
__global__ void k_rowblock_flags(i64 nrows, const i32 *rp, i32 *flag) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    int f = 1;
    if (i > 0) {
        i32 a = rp[i - 1], b = rp[i], c = rp[i + 1];
        f = (b / RB_T != a / RB_T) || (b - a > RB_T) || (c - b > RB_T) || (i % RB_RCAP == 0);
    }
    flag[i] = f;
}

__global__ void k_rowblock_scatter(i64 nrows, const i32 *flag, const i32 *pos, i32 *blocks, i64 nblocks) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrows && flag[i]) blocks[pos[i]] = (i32)i;
    if (i == 0) blocks[nblocks] = (i32)nrows;
}

void build_row_blocks(dsm_ctx ctx, Payload &P, i64 nrows, hipStream_t s) {
    if (nrows == 0) {
        P.nrblocks = 0;
        P.rblocks = (i32 *)P.alloc(ctx, sizeof(i32));
        DSM_HIP(hipMemsetAsync(P.rblocks, 0, sizeof(i32), s));
        return;
    }
    Tmp flag(ctx, sizeof(i32) * (size_t)nrows), pos(ctx, sizeof(i32) * (size_t)(nrows + 1));
    hipLaunchKernelGGL(k_rowblock_flags, dim3(grid_for(nrows, CB)), dim3(CB), 0, s, nrows, P.rp, flag.as<i32>());
    DSM_HIP(hipGetLastError());
    i64 nb = exclusive_scan_i32(ctx, flag.as<i32>(), pos.as<i32>(), nrows, s, true);
    P.nrblocks = nb;
    P.rblocks = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)(nb + 1));
    hipLaunchKernelGGL(k_rowblock_scatter, dim3(grid_for(nrows, CB)), dim3(CB), 0, s, nrows, flag.as<i32>(),
                       pos.as<i32>(), P.rblocks, nb);
    DSM_HIP(hipGetLastError());
    DSM_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- small kernels
__global__ void k_row_len(i64 nrows, const i32 *rp, i32 *len) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrows) len[i] = rp[i + 1] - rp[i];
}

template <class Wi, class Wo, int DTI, int DTO>
__global__ void k_cast(i64 n, const Wi *in, Wo *out) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Wi w = in[i];
    double d;
    float f;
    if constexpr (DTI == DSM_F64) {
        memcpy(&d, &w, 8);
    } else if constexpr (DTI == DSM_F32) {
        memcpy(&f, &w, 4);
        d = (double)f;
    } else {
        bf16 h;
        h.bits = w;
        d = (double)bf16_to_float(h);
    }
    Wo o;
    if constexpr (DTO == DSM_F64) {
        memcpy(&o, &d, 8);
    } else if constexpr (DTO == DSM_F32) {
        f = (float)d;  // round to nearest even (exact when widening)
        memcpy(&o, &f, 4);
    } else {
        // narrowing goes through FP32; from FP32 or BF16 sources it is exact
        f = (float)d;
        o = float_to_bf16(f).bits;
    }
    out[i] = o;
}

// Flags a value whose cast to DTO (the cast k_cast applies), widened back,
// differs from it bit for bit (NaN payloads and the sign of zero included).
template <class Wi, int DTI, int DTO>
__global__ void k_values_exact(i64 n, const Wi *in, int *bad) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Wi w = in[i];
    double d;
    if constexpr (DTI == DSM_F64) {
        memcpy(&d, &w, 8);
    } else {
        float f;
        memcpy(&f, &w, 4);
        d = (double)f;
    }
    const float f = (float)d;
    const double back = DTO == DSM_F32 ? (double)f : (double)bf16_to_float(float_to_bf16(f));
    u64 a, b;
    memcpy(&a, &d, 8);
    memcpy(&b, &back, 8);
    if (a != b) *bad = 1;
}

// Dispatch helpers over the value storage width.
#define DSM_BY_DTYPE(dt, ...)                                                            \
    switch (dt) {                                                                        \
    case DSM_F64: { using W = u64; __VA_ARGS__; break; }                                 \
    case DSM_F32: { using W = u32; __VA_ARGS__; break; }                                 \
    default: { using W = uint16_t; __VA_ARGS__; break; }                                 \
    }

static void cast_values(int dti, const void *in, int dto, void *out, i64 n, hipStream_t s) {
    if (n == 0) return;
    if (dti == dto) {
        DSM_HIP(hipMemcpyAsync(out, in, (size_t)n * dtype_size(dti), hipMemcpyDeviceToDevice, s));
        return;
    }
    dim3 g(grid_for(n, CB)), b(CB);
#define CASTK(WI, WO, A, B) hipLaunchKernelGGL((k_cast<WI, WO, A, B>), g, b, 0, s, n, (const WI *)in, (WO *)out)
    if (dti == DSM_F64 && dto == DSM_F32) CASTK(u64, u32, DSM_F64, DSM_F32);
    else if (dti == DSM_F64 && dto == DSM_BF16) CASTK(u64, uint16_t, DSM_F64, DSM_BF16);
    else if (dti == DSM_F32 && dto == DSM_F64) CASTK(u32, u64, DSM_F32, DSM_F64);
    else if (dti == DSM_F32 && dto == DSM_BF16) CASTK(u32, uint16_t, DSM_F32, DSM_BF16);
    else if (dti == DSM_BF16 && dto == DSM_F64) CASTK(uint16_t, u64, DSM_BF16, DSM_F64);
    else CASTK(uint16_t, u32, DSM_BF16, DSM_F32);
#undef CASTK
    DSM_HIP(hipGetLastError());
}

Payload cast_csr(dsm_matrix m, const Payload &src, int vdt, hipStream_t s) {
    Payload P;
    P.fmt = DSM_CSR;
    P.vdt = vdt;
    P.csr_nnz = src.csr_nnz;
    try {
        P.rp = (i32 *)P.alloc(m->ctx, sizeof(i32) * (size_t)(m->nrows + 1));
        P.col = (i32 *)P.alloc(m->ctx, sizeof(i32) * (size_t)src.csr_nnz);
        P.val = P.alloc(m->ctx, dtype_size(vdt) * (size_t)src.csr_nnz);
        DSM_HIP(hipMemcpyAsync(P.rp, src.rp, sizeof(i32) * (size_t)(m->nrows + 1), hipMemcpyDeviceToDevice, s));
        DSM_HIP(hipMemcpyAsync(P.col, src.col, sizeof(i32) * (size_t)src.csr_nnz, hipMemcpyDeviceToDevice, s));
        cast_values(src.vdt, src.val, vdt, P.val, src.csr_nnz, s);
        build_row_blocks(m->ctx, P, m->nrows, s);
    } catch (...) {
        P.release(m->ctx);
        throw;
    }
    return P;
}

// ---------------------------------------------------------------- CSR <-> COO
__global__ void __launch_bounds__(CB) k_csr_expand_rows(i64 nrows, const i32 *rp, i32 *row) {
    for_each_entry(nrows, rp, [&](i64 r, i64 e) { row[e] = (i32)r; });
}

// Sorted COO rows -> row pointers; flags unsorted/duplicate/out-of-range.
__global__ void k_coo_rowptr(i64 nnz, i64 nrows, i64 ncols, const i32 *row, const i32 *col, i32 *rp, int *err) {
    i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nnz) return;
    i64 prev = k == 0 ? -1 : (i64)row[k - 1];
    i64 cur = k == nnz ? nrows : (i64)row[k];
    if (k < nnz) {
        if (cur < 0 || cur >= nrows || col[k] < 0 || (i64)col[k] >= ncols) {
            if (err) atomicOr(err, 8);
            return;
        }
        if (k > 0 && (cur < prev || (cur == prev && col[k] <= col[k - 1]))) {
            if (err) atomicOr(err, 16);
            return;
        }
    }
    if (prev < -1 || prev >= nrows) return;  // reported by the previous entry
    for (i64 r = prev + 1; r <= cur; r++) rp[r] = (i32)k;
}

// ---------------------------------------------------------------- DIA
__global__ void __launch_bounds__(CB) k_diag_mark(i64 nrows, const i32 *rp, const i32 *col, i32 *flag) {
    for_each_entry(nrows, rp, [&](i64 r, i64 e) { flag[(i64)col[e] - r + nrows - 1] = 1; });
}

// Entries per diagonal (index col - row + nrows - 1).  `table`: the span of
// indices fits int32 keys, so the counts are privatised in LDS.
__global__ void __launch_bounds__(CB) k_diag_count(i64 nrows, const i32 *rp, const i32 *col, i32 *cnt, int table) {
    __shared__ i32 hk[HT], hv[HT];
    if (!table) {
        for_each_entry(nrows, rp, [&](i64 r, i64 e) { atomicAdd(&cnt[(i64)col[e] - r + nrows - 1], 1); });
        return;
    }
    ht_init(hk, hv);
    for_each_entry(nrows, rp, [&](i64 r, i64 e) { ht_add(hk, hv, (i32)((i64)col[e] - r + nrows - 1), cnt); });
    __syncthreads();
    ht_flush(hk, hv, cnt);
}

static void diag_count(i64 n, i64 span, const i32 *rp, const i32 *col, i32 *cnt, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_diag_count, dim3(entry_grid(n)), dim3(CB), 0, s, n, rp, col, cnt,
                           span <= (i64)INT32_MAX ? 1 : 0);
}

__global__ void k_offsets_compact(i64 span, i64 nrows, const i32 *flag, const i32 *slot, i32 *offs) {
    i64 d = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (d < span && flag[d]) offs[slot[d]] = (i32)(d - (nrows - 1));
}

// Diagonal d (index d + nrows - 1) is "true" for HDC when its count reaches
// theta times the number of in-range positions on it (decided in FP64).
__global__ void k_hdc_true(i64 span, i64 nrows, i64 ncols, double theta, const i32 *cnt, i32 *flag) {
    i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= span) return;
    i64 d = s - (nrows - 1);
    i64 lo = d < 0 ? -d : 0;
    i64 hi = min(nrows, ncols - d);
    i64 L = hi > lo ? hi - lo : 0;
    i32 c = cnt[s];
    flag[s] = (c > 0 && (double)c >= theta * (double)L) ? 1 : 0;
}

// Entries on a marked diagonal go to DIA slot (slot[d], row); with
// `rest_pos` != null the others are appended to the CSR remainder of their
// row in ascending column order (rest_pos = that row's write cursor start).
template <class W>
__global__ void __launch_bounds__(CB) k_dia_scatter(i64 nrows, const i32 *rp, const i32 *col, const W *val,
                                                     const i32 *flag, const i32 *slot, i64 pitch, W *dval) {
    for_each_entry(nrows, rp, [&](i64 r, i64 e) {
        i64 d = (i64)col[e] - r + nrows - 1;
        if (!flag || flag[d]) dval[(i64)slot[d] * pitch + r] = val[e];
    });
}

// Per row: entries not on a true diagonal (HDC remainder).  Column loads of
// CB_U entries, then their flag loads, are issued together (entries past the
// row read the sentinel column, then the sentinel as their flag: nonzero, so
// they count nothing).
__global__ void __launch_bounds__(CB) k_rest_count(i64 nrows, const i32 *rp, const i32 *col, const i32 *flag,
                                                   i32 *cnt) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    const i64 a = rp[i], b = rp[i + 1];
    i32 n_rest = 0;
    for (i64 e0 = a; e0 < b; e0 += CB_U) {
        i32 c[CB_U], f[CB_U];
#pragma unroll
        for (int u = 0; u < CB_U; u++) c[u] = *(e0 + u < b ? col + e0 + u : sentinel_ptr<i32>());
#pragma unroll
        for (int u = 0; u < CB_U; u++) f[u] = *(c[u] >= 0 ? flag + ((i64)c[u] - i + nrows - 1) : sentinel_ptr<i32>());
#pragma unroll
        for (int u = 0; u < CB_U; u++) n_rest += f[u] ? 0 : 1;
    }
    cnt[i] = n_rest;
}

template <class W>
__global__ void k_rest_fill(i64 nrows, const i32 *rp, const i32 *col, const W *val, const i32 *flag,
                            const i32 *orp, i32 *ocol, W *oval) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    i64 o = orp[i];
    for (i64 e = rp[i]; e < rp[i + 1]; e++) {
        if (flag[(i64)col[e] - i + nrows - 1]) continue;
        ocol[o] = col[e];
        oval[o] = val[e];
        o++;
    }
}

// DIA -> CSR: count, then fill in ascending offset order, dropping +-0.
template <class W>
__global__ void k_dia_rowcount(i64 nrows, i64 ncols, i64 ndiag, const i32 *offs, const W *dval, i64 pitch,
                               const i32 *extra_rp, i32 *cnt) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    i32 c = 0;
    for (i64 k = 0; k < ndiag; k++) {
        i64 j = i + offs[k];
        if (j >= 0 && j < ncols && !word_is_zero(dval[k * pitch + i])) c++;
    }
    if (extra_rp) c += extra_rp[i + 1] - extra_rp[i];
    cnt[i] = c;
}

// Merges a row's DIA slots with (optional) CSR entries by ascending column.
template <class W>
__global__ void k_dia_merge_fill(i64 nrows, i64 ncols, i64 ndiag, const i32 *offs, const W *dval, i64 pitch,
                                 const i32 *xrp, const i32 *xcol, const W *xval, const i32 *orp, i32 *ocol,
                                 W *oval) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    i64 o = orp[i];
    i64 k = 0;
    i64 e = xrp ? xrp[i] : 0, e1 = xrp ? xrp[i + 1] : 0;
    for (;;) {
        while (k < ndiag) {
            i64 j = i + offs[k];
            if (j >= 0 && j < ncols && !word_is_zero(dval[k * pitch + i])) break;
            k++;
        }
        bool hd = k < ndiag, hc = e < e1;
        if (!hd && !hc) break;
        i64 jd = hd ? i + offs[k] : INT64_MAX;
        i64 jc = hc ? (i64)xcol[e] : INT64_MAX;
        if (jd < jc) {
            ocol[o] = (i32)jd;
            oval[o] = dval[k * pitch + i];
            k++;
        } else {
            ocol[o] = (i32)jc;
            oval[o] = xval[e];
            e++;
        }
        o++;
    }
}

// ---------------------------------------------------------------- ELL / HYB
// Every slot of rows [0, pitch): the k-th entry of the row for k < len, the
// -1 column sentinel and a zero value after the row's end and in the pitch
// padding rows (so no memset is needed first).  The loads of CB_U slots are
// issued together; slots past the row read the sentinel and zero words, whose
// bits are exactly the padding encoding.
template <class W>
__global__ void __launch_bounds__(CB) k_ell_fill(i64 nrows, i64 pitch, const i32 *rp, const i32 *col, const W *val,
                                                 i64 K, i32 *ecol, W *eval) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pitch) return;
    const i64 a = i < nrows ? rp[i] : 0, len = i < nrows ? rp[i + 1] - a : 0;
    for (i64 k0 = 0; k0 < K; k0 += CB_U) {
        i32 c[CB_U];
        W v[CB_U];
#pragma unroll
        for (int u = 0; u < CB_U; u++) {
            const i64 k = k0 + u;
            c[u] = *(k < len ? col + a + k : sentinel_ptr<i32>());
            v[u] = *(k < len ? val + a + k : zero_ptr<W>());
        }
#pragma unroll
        for (int u = 0; u < CB_U; u++)
            if (k0 + u < K) {
                ecol[(k0 + u) * pitch + i] = c[u];
                eval[(k0 + u) * pitch + i] = v[u];
            }
    }
}

// Row-length histogram (bins privatised in LDS per workgroup).
__global__ void __launch_bounds__(CB) k_len_hist(i64 nrows, const i32 *rp, i32 *hist) {
    __shared__ i32 hk[HT], hv[HT];
    ht_init(hk, hv);
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < nrows; i += (i64)gridDim.x * blockDim.x)
        ht_add(hk, hv, rp[i + 1] - rp[i], hist);
    __syncthreads();
    ht_flush(hk, hv, hist);
}

constexpr unsigned STATS_GRID = 1024;  // workgroups of the grid-stride statistics kernels

static void len_hist(i64 n, const i32 *rp, i32 *hist, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_len_hist, dim3(std::min<unsigned>(grid_for(n, CB), STATS_GRID)), dim3(CB), 0, s, n, rp,
                           hist);
}

// K_h = largest k with #{rows : len >= k} >= need (single thread; maxlen is
// the longest row).
__global__ void k_hyb_width(const i32 *hist, i64 maxlen, i64 need, i32 *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    i64 ge = 0;
    i64 k = maxlen;
    for (; k > 0; k--) {
        ge += hist[k];
        if (ge >= need) break;
    }
    *out = (i32)k;
}

__global__ void k_overflow_count(i64 nrows, const i32 *rp, i64 K, i32 *cnt) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    i64 len = rp[i + 1] - rp[i];
    cnt[i] = (i32)(len > K ? len - K : 0);
}

template <class W>
__global__ void k_overflow_fill(i64 nrows, const i32 *rp, const i32 *col, const W *val, i64 K, const i32 *orp,
                                i32 *crow, i32 *ccol, W *cval) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    i64 o = orp[i];
    for (i64 e = rp[i] + K; e < rp[i + 1]; e++, o++) {
        crow[o] = (i32)i;
        ccol[o] = col[e];
        cval[o] = val[e];
    }
}

// ELL (+ optional COO part with row pointers crp) -> CSR counts and fill.
__global__ void k_ell_rowcount(i64 nrows, i64 K, i64 pitch, const i32 *ecol, const i32 *crp, i32 *cnt) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    i32 c = 0;
    for (i64 k = 0; k < K; k++) c += ecol[k * pitch + i] >= 0 ? 1 : 0;
    if (crp) c += crp[i + 1] - crp[i];
    cnt[i] = c;
}

template <class W>
__global__ void k_ell_to_csr_fill(i64 nrows, i64 K, i64 pitch, const i32 *ecol, const W *eval, const i32 *crp,
                                  const i32 *ccol, const W *cval, const i32 *orp, i32 *ocol, W *oval) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    i64 o = orp[i];
    for (i64 k = 0; k < K; k++) {
        i32 c = ecol[k * pitch + i];
        if (c < 0) continue;
        ocol[o] = c;
        oval[o] = eval[k * pitch + i];
        o++;
    }
    if (crp)
        for (i64 e = crp[i]; e < crp[i + 1]; e++, o++) {
            ocol[o] = ccol[e];
            oval[o] = cval[e];
        }
}

// ---------------------------------------------------------------- stats
__global__ void __launch_bounds__(CB) k_row_stats(i64 nrows, const i32 *rp, unsigned long long *acc) {
    // acc: [0] max, [1] min, [2] sum, [3] sumsq, [4] empty, [5..37] histogram
    // of floor(log2(len)) + 1 (0 for empty rows); reduced per workgroup in
    // LDS, then one global atomic per field and workgroup
    __shared__ unsigned long long sh[5];
    __shared__ unsigned hb[33];
    if (threadIdx.x < 5) sh[threadIdx.x] = threadIdx.x == 1 ? ~0ull : 0ull;
    if (threadIdx.x < 33) hb[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long mx = 0, mn = ~0ull, sum = 0, sq = 0, empty = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < nrows; i += (i64)gridDim.x * blockDim.x) {
        const unsigned long long len = (unsigned long long)(rp[i + 1] - rp[i]);
        mx = max(mx, len);
        mn = min(mn, len);
        sum += len;
        sq += len * len;
        empty += len == 0 ? 1 : 0;
        int b = len == 0 ? 0 : 64 - __clzll(len);  // floor(log2(len)) + 1
        if (b > 32) b = 32;
        atomicAdd(&hb[b], 1u);
    }
    atomicMax(&sh[0], mx);
    atomicMin(&sh[1], mn);
    atomicAdd(&sh[2], sum);
    atomicAdd(&sh[3], sq);
    atomicAdd(&sh[4], empty);
    __syncthreads();
    const int t = threadIdx.x;
    if (t == 0) atomicMax(&acc[0], sh[0]);
    else if (t == 1) atomicMin(&acc[1], sh[1]);
    else if (t < 5) {
        if (sh[t]) atomicAdd(&acc[t], sh[t]);
    } else if (t < 38) {
        if (hb[t - 5]) atomicAdd(&acc[t], (unsigned long long)hb[t - 5]);
    }
}

__global__ void k_stats_init(unsigned long long *acc) {
    int t = threadIdx.x;
    if (t < 38) acc[t] = t == 1 ? ~0ull : 0ull;
}

// ================================================================ host side
static void sync(hipStream_t s) { DSM_HIP(hipStreamSynchronize(s)); }

static void check_pad(double slots, double nnz, double ratio, const char *what) {
    if (ratio <= 0) ratio = 16.0;
    if (slots > ratio * std::max(nnz, 1.0))
        fail(DSM_E_INFEASIBLE, std::string(what) + ": " + std::to_string((long long)slots) +
                                   " stored slots exceed max_pad_ratio * nnz");
}

// row lengths of a CSR part -> longest row
static i64 max_row_len(dsm_ctx ctx, i64 nrows, const i32 *rp, hipStream_t s) {
    if (nrows == 0) return 0;
    Tmp len(ctx, sizeof(i32) * (size_t)nrows);
    hipLaunchKernelGGL(k_row_len, dim3(grid_for(nrows, CB)), dim3(CB), 0, s, nrows, rp, len.as<i32>());
    DSM_HIP(hipGetLastError());
    return reduce_max_i32(ctx, len.as<i32>(), nrows, s);
}

template <class W>
static void dia_from_csr(dsm_matrix m, const Payload &C, Payload &P, const i32 *flag_true, bool hdc,
                         const dsm_convert_opts &o, hipStream_t s) {
    dsm_ctx ctx = m->ctx;
    const i64 n = m->nrows, nc = m->ncols, span = n + nc - 1;
    Tmp flag(ctx, sizeof(i32) * (size_t)span), slot(ctx, sizeof(i32) * (size_t)(span + 1));
    const i32 *use_flag = flag_true;
    if (!flag_true) {
        DSM_HIP(hipMemsetAsync(flag.p, 0, sizeof(i32) * (size_t)span, s));
        if (n > 0)
            hipLaunchKernelGGL(k_diag_mark, dim3(entry_grid(n)), dim3(CB), 0, s, n, C.rp, C.col, flag.as<i32>());
        DSM_HIP(hipGetLastError());
        use_flag = flag.as<i32>();
    }
    i64 nd = exclusive_scan_i32(ctx, use_flag, slot.as<i32>(), span, s, true);
    P.pitch = pitch_for(n);
    if (!hdc) check_pad((double)nd * (double)n, (double)C.csr_nnz, o.max_pad_ratio, "DIA");
    P.ndiag = nd;
    // offsets padded with zeros to a multiple of 16 entries: the sweep reads
    // them in batches of up to 16 without a bound check
    const i64 offs_len = (std::max<i64>(nd, 1) + 15) / 16 * 16;
    P.offs = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)offs_len);
    DSM_HIP(hipMemsetAsync(P.offs, 0, sizeof(i32) * (size_t)offs_len, s));
    P.dval = P.alloc(ctx, sizeof(W) * (size_t)std::max<i64>(nd * P.pitch, 1));
    DSM_HIP(hipMemsetAsync(P.dval, 0, sizeof(W) * (size_t)(nd * P.pitch), s));
    hipLaunchKernelGGL(k_offsets_compact, dim3(grid_for(span, CB)), dim3(CB), 0, s, span, n, use_flag,
                       slot.as<i32>(), P.offs);
    // diagonal clusters for the LDS-staged sweep (host pass over the offsets)
    if (nd > 0) {
        std::vector<i32> ho((size_t)nd);
        DSM_HIP(hipMemcpyAsync(ho.data(), P.offs, sizeof(i32) * (size_t)nd, hipMemcpyDeviceToHost, s));
        sync(s);
        const std::vector<i32> hc = diagonal_clusters(ho, DIA_CLUSTER_K, DIA_CLUSTER_SPAN);
        P.nclu = (i64)hc.size() / CLU_REC;
        P.clu = (i32 *)P.alloc(ctx, sizeof(i32) * hc.size());
        DSM_HIP(hipMemcpyAsync(P.clu, hc.data(), sizeof(i32) * hc.size(), hipMemcpyHostToDevice, s));
        sync(s);  // hc is a host temporary
    }
    if (n > 0)
        hipLaunchKernelGGL((k_dia_scatter<W>), dim3(entry_grid(n)), dim3(CB), 0, s, n, C.rp, C.col,
                           (const W *)C.val, hdc ? use_flag : (const i32 *)nullptr, slot.as<i32>(), P.pitch,
                           (W *)P.dval);
    DSM_HIP(hipGetLastError());
    sync(s);
}

template <class W>
static Payload from_csr_typed(dsm_matrix m, const Payload &C, int fmt, const dsm_convert_opts &o, hipStream_t s) {
    dsm_ctx ctx = m->ctx;
    const i64 n = m->nrows, nc = m->ncols, nnz = C.csr_nnz;
    Payload P;
    P.fmt = fmt;
    P.vdt = C.vdt;
    try {
        switch (fmt) {
        case DSM_COO: {
            P.coo_nnz = nnz;
            P.crow = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)nnz);
            P.ccol = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)nnz);
            P.cval = P.alloc(ctx, sizeof(W) * (size_t)nnz);
            if (n > 0)
                hipLaunchKernelGGL(k_csr_expand_rows, dim3(entry_grid(n)), dim3(CB), 0, s, n, C.rp, P.crow);
            DSM_HIP(hipGetLastError());
            DSM_HIP(hipMemcpyAsync(P.ccol, C.col, sizeof(i32) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
            DSM_HIP(hipMemcpyAsync(P.cval, C.val, sizeof(W) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
            sync(s);
            break;
        }
        case DSM_DIA:
            dia_from_csr<W>(m, C, P, nullptr, false, o, s);
            break;
        case DSM_ELL:
        case DSM_HYB: {
            i64 K;
            if (fmt == DSM_ELL) {
                K = max_row_len(ctx, n, C.rp, s);
                check_pad((double)K * (double)n, (double)nnz, o.max_pad_ratio, "ELL");
            } else if (o.hyb_width >= 0) {
                K = o.hyb_width;
            } else {
                i64 mx = max_row_len(ctx, n, C.rp, s);
                Tmp hist(ctx, sizeof(i32) * (size_t)(mx + 2));
                DSM_HIP(hipMemsetAsync(hist.p, 0, sizeof(i32) * (size_t)(mx + 2), s));
                len_hist(n, C.rp, hist.as<i32>(), s);
                i32 *kout = hist.as<i32>() + mx + 1;
                hipLaunchKernelGGL(k_hyb_width, dim3(1), dim3(64), 0, s, hist.as<i32>(), mx, (n + 2) / 3, kout);
                DSM_HIP(hipGetLastError());
                i32 kh = 0;
                DSM_HIP(hipMemcpyAsync(&kh, kout, sizeof(i32), hipMemcpyDeviceToHost, s));
                sync(s);
                K = n > 0 ? kh : 0;
            }
            P.K = K;
            P.pitch = pitch_for(n);
            P.ecol = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)(K * P.pitch));
            P.evl = P.alloc(ctx, sizeof(W) * (size_t)(K * P.pitch));
            // every slot, the pitch padding rows included (sentinel columns,
            // so any sweep stays valid)
            if (P.pitch > 0 && K > 0)
                hipLaunchKernelGGL((k_ell_fill<W>), dim3(grid_for(P.pitch, CB)), dim3(CB), 0, s, n, P.pitch, C.rp,
                                   C.col, (const W *)C.val, K, P.ecol, (W *)P.evl);
            DSM_HIP(hipGetLastError());
            if (fmt == DSM_HYB) {
                Tmp cnt(ctx, sizeof(i32) * (size_t)std::max<i64>(n, 1)), orp(ctx, sizeof(i32) * (size_t)(n + 1));
                if (n > 0)
                    hipLaunchKernelGGL(k_overflow_count, dim3(grid_for(n, CB)), dim3(CB), 0, s, n, C.rp, K,
                                       cnt.as<i32>());
                i64 nco = exclusive_scan_i32(ctx, cnt.as<i32>(), orp.as<i32>(), n, s, true);
                P.coo_nnz = nco;
                P.crow = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)nco);
                P.ccol = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)nco);
                P.cval = P.alloc(ctx, sizeof(W) * (size_t)nco);
                if (n > 0 && nco > 0)
                    hipLaunchKernelGGL((k_overflow_fill<W>), dim3(grid_for(n, CB)), dim3(CB), 0, s, n, C.rp,
                                       C.col, (const W *)C.val, K, orp.as<i32>(), P.crow, P.ccol, (W *)P.cval);
                DSM_HIP(hipGetLastError());
            }
            sync(s);
            break;
        }
        case DSM_HDC: {
            const i64 span = n + nc - 1;
            double theta = o.hdc_theta > 0 ? o.hdc_theta : 0.5;
            P.theta = theta;
            Tmp cnt(ctx, sizeof(i32) * (size_t)std::max<i64>(span, 1)),
                flag(ctx, sizeof(i32) * (size_t)std::max<i64>(span, 1));
            DSM_HIP(hipMemsetAsync(cnt.p, 0, sizeof(i32) * (size_t)span, s));
            diag_count(n, span, C.rp, C.col, cnt.as<i32>(), s);
            if (span > 0)
                hipLaunchKernelGGL(k_hdc_true, dim3(grid_for(span, CB)), dim3(CB), 0, s, span, n, nc, theta,
                                   cnt.as<i32>(), flag.as<i32>());
            DSM_HIP(hipGetLastError());
            dia_from_csr<W>(m, C, P, flag.as<i32>(), true, o, s);
            // CSR remainder
            Tmp rc(ctx, sizeof(i32) * (size_t)std::max<i64>(n, 1));
            P.rp = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)(n + 1));
            if (n > 0)
                hipLaunchKernelGGL(k_rest_count, dim3(grid_for(n, CB)), dim3(CB), 0, s, n, C.rp, C.col,
                                   flag.as<i32>(), rc.as<i32>());
            i64 nr = exclusive_scan_i32(ctx, rc.as<i32>(), P.rp, n, s, true);
            P.csr_nnz = nr;
            P.col = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)nr);
            P.val = P.alloc(ctx, sizeof(W) * (size_t)nr);
            if (n > 0 && nr > 0)
                hipLaunchKernelGGL((k_rest_fill<W>), dim3(grid_for(n, CB)), dim3(CB), 0, s, n, C.rp, C.col,
                                   (const W *)C.val, flag.as<i32>(), P.rp, P.col, (W *)P.val);
            DSM_HIP(hipGetLastError());
            build_row_blocks(ctx, P, n, s);
            sync(s);
            break;
        }
        default:
            fail(DSM_E_INVALID, "unknown format");
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        P.release(ctx);
        throw;
    }
    return P;
}

Payload from_csr(dsm_matrix m, const Payload &csr, int fmt, int vdt, const dsm_convert_opts &o, hipStream_t s) {
    DSM_CHECK(csr.fmt == DSM_CSR, DSM_E_INVALID, "from_csr needs a CSR payload");
    if (fmt == DSM_CSR) return cast_csr(m, csr, vdt, s);
    Payload casted;
    const Payload *src = &csr;
    if (vdt != csr.vdt) {
        casted = cast_csr(m, csr, vdt, s);
        src = &casted;
    }
    Payload out;
    try {
        DSM_BY_DTYPE(vdt, out = from_csr_typed<W>(m, *src, fmt, o, s));
    } catch (...) {
        if (src == &casted) casted.release(m->ctx);
        throw;
    }
    if (src == &casted) casted.release(m->ctx);
    return out;
}

template <class W>
static Payload to_csr_typed(dsm_matrix m, const Payload &S, hipStream_t s) {
    dsm_ctx ctx = m->ctx;
    const i64 n = m->nrows, nc = m->ncols;
    Payload P;
    P.fmt = DSM_CSR;
    P.vdt = S.vdt;
    try {
        P.rp = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)(n + 1));
        Tmp cnt(ctx, sizeof(i32) * (size_t)std::max<i64>(n, 1));
        i64 nnz = 0;
        switch (S.fmt) {
        case DSM_COO: {
            hipLaunchKernelGGL(k_coo_rowptr, dim3(grid_for(S.coo_nnz + 1, CB)), dim3(CB), 0, s, S.coo_nnz, n, nc,
                               S.crow, S.ccol, P.rp, (int *)nullptr);
            DSM_HIP(hipGetLastError());
            nnz = S.coo_nnz;
            P.col = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)nnz);
            P.val = P.alloc(ctx, sizeof(W) * (size_t)nnz);
            DSM_HIP(hipMemcpyAsync(P.col, S.ccol, sizeof(i32) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
            DSM_HIP(hipMemcpyAsync(P.val, S.cval, sizeof(W) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
            break;
        }
        case DSM_DIA:
        case DSM_HDC: {
            const i32 *xrp = S.fmt == DSM_HDC ? S.rp : nullptr;
            if (n > 0)
                hipLaunchKernelGGL((k_dia_rowcount<W>), dim3(grid_for(n, CB)), dim3(CB), 0, s, n, nc, S.ndiag,
                                   S.offs, (const W *)S.dval, S.pitch, xrp, cnt.as<i32>());
            DSM_HIP(hipGetLastError());
            nnz = exclusive_scan_i32(ctx, cnt.as<i32>(), P.rp, n, s, true);
            P.col = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)nnz);
            P.val = P.alloc(ctx, sizeof(W) * (size_t)nnz);
            if (n > 0)
                hipLaunchKernelGGL((k_dia_merge_fill<W>), dim3(grid_for(n, CB)), dim3(CB), 0, s, n, nc, S.ndiag,
                                   S.offs, (const W *)S.dval, S.pitch, xrp, S.col, (const W *)S.val, P.rp, P.col,
                                   (W *)P.val);
            DSM_HIP(hipGetLastError());
            break;
        }
        case DSM_ELL:
        case DSM_HYB: {
            Tmp crp(ctx, sizeof(i32) * (size_t)(n + 1));
            const i32 *cr = nullptr;
            if (S.fmt == DSM_HYB) {
                hipLaunchKernelGGL(k_coo_rowptr, dim3(grid_for(S.coo_nnz + 1, CB)), dim3(CB), 0, s, S.coo_nnz, n,
                                   nc, S.crow, S.ccol, crp.as<i32>(), (int *)nullptr);
                cr = crp.as<i32>();
            }
            if (n > 0)
                hipLaunchKernelGGL(k_ell_rowcount, dim3(grid_for(n, CB)), dim3(CB), 0, s, n, S.K, S.pitch, S.ecol,
                                   cr, cnt.as<i32>());
            DSM_HIP(hipGetLastError());
            nnz = exclusive_scan_i32(ctx, cnt.as<i32>(), P.rp, n, s, true);
            P.col = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)nnz);
            P.val = P.alloc(ctx, sizeof(W) * (size_t)nnz);
            if (n > 0)
                hipLaunchKernelGGL((k_ell_to_csr_fill<W>), dim3(grid_for(n, CB)), dim3(CB), 0, s, n, S.K, S.pitch,
                                   S.ecol, (const W *)S.evl, cr, S.ccol, (const W *)S.cval, P.rp, P.col,
                                   (W *)P.val);
            DSM_HIP(hipGetLastError());
            sync(s);
            break;
        }
        default:
            fail(DSM_E_INVALID, "to_csr: unknown source format");
        }
        P.csr_nnz = nnz;
        build_row_blocks(ctx, P, n, s);
        sync(s);
    } catch (...) {
        (void)hipStreamSynchronize(s);
        P.release(ctx);
        throw;
    }
    return P;
}

Payload to_csr(dsm_matrix m, const Payload &src, hipStream_t s) {
    if (src.fmt == DSM_CSR) return cast_csr(m, src, src.vdt, s);
    Payload out;
    DSM_BY_DTYPE(src.vdt, out = to_csr_typed<W>(m, src, s));
    return out;
}

// ---------------------------------------------------------------- structure features
// Entries whose column lies within `w` of the row (x gathers that stay in a
// cache-sized window around the diagonal).
__global__ void __launch_bounds__(CB) k_near_count(i64 nrows, const i32 *rp, const i32 *col, i64 w,
                                                   unsigned long long *out) {
    __shared__ unsigned long long lds[CB / WAVE];
    unsigned long long c = 0;
    for_each_entry(nrows, rp, [&](i64 r, i64 e) {
        const i64 d = (i64)col[e] - r;
        c += (d <= w && d >= -w) ? 1ull : 0ull;
    });
    c = block_sum(c, lds);
    if (threadIdx.x == 0) atomicAdd(out, c);
}

// Entries on diagonals whose flag is set (HDC's DIA part).
__global__ void k_masked_count(i64 span, const i32 *cnt, const i32 *flag, unsigned long long *out) {
    const i64 d = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (d < span && flag[d]) atomicAdd(out, (unsigned long long)cnt[d]);
}

StructFeatures structure_features(dsm_matrix m, const Payload &C, double theta, i64 window, hipStream_t s) {
    DSM_CHECK(C.fmt == DSM_CSR, DSM_E_INVALID, "structure_features needs a CSR payload");
    dsm_ctx ctx = m->ctx;
    const i64 n = m->nrows, nc = m->ncols, span = n + nc - 1;
    StructFeatures F{};
    F.nnz = C.csr_nnz;
    if (n == 0) return F;
    F.max_len = max_row_len(ctx, n, C.rp, s);
    // HYB width from the row-length histogram
    {
        Tmp hist(ctx, sizeof(i32) * (size_t)(F.max_len + 2));
        DSM_HIP(hipMemsetAsync(hist.p, 0, sizeof(i32) * (size_t)(F.max_len + 2), s));
        len_hist(n, C.rp, hist.as<i32>(), s);
        i32 *kout = hist.as<i32>() + F.max_len + 1;
        hipLaunchKernelGGL(k_hyb_width, dim3(1), dim3(64), 0, s, hist.as<i32>(), F.max_len, (n + 2) / 3, kout);
        Tmp cnt(ctx, sizeof(i32) * (size_t)n), orp(ctx, sizeof(i32) * (size_t)(n + 1));
        i32 kh = 0;
        DSM_HIP(hipMemcpyAsync(&kh, kout, sizeof(i32), hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
        F.hyb_width = kh;
        hipLaunchKernelGGL(k_overflow_count, dim3(grid_for(n, CB)), dim3(CB), 0, s, n, C.rp, (i64)kh, cnt.as<i32>());
        DSM_HIP(hipGetLastError());
        F.hyb_coo = exclusive_scan_i32(ctx, cnt.as<i32>(), orp.as<i32>(), n, s, true);
    }
    // diagonals: all of them (DIA) and the well-filled ones (HDC)
    {
        Tmp cnt(ctx, sizeof(i32) * (size_t)span), flag(ctx, sizeof(i32) * (size_t)span),
            acc(ctx, 2 * sizeof(unsigned long long));
        DSM_HIP(hipMemsetAsync(cnt.p, 0, sizeof(i32) * (size_t)span, s));
        DSM_HIP(hipMemsetAsync(acc.p, 0, 2 * sizeof(unsigned long long), s));
        diag_count(n, span, C.rp, C.col, cnt.as<i32>(), s);
        hipLaunchKernelGGL(k_hdc_true, dim3(grid_for(span, CB)), dim3(CB), 0, s, span, n, nc, theta, cnt.as<i32>(),
                           flag.as<i32>());
        hipLaunchKernelGGL(k_masked_count, dim3(grid_for(span, CB)), dim3(CB), 0, s, span, cnt.as<i32>(),
                           flag.as<i32>(), acc.as<unsigned long long>());
        hipLaunchKernelGGL(k_near_count, dim3(entry_grid(n)), dim3(CB), 0, s, n, C.rp, C.col, window,
                           acc.as<unsigned long long>() + 1);
        DSM_HIP(hipGetLastError());
        Tmp slot(ctx, sizeof(i32) * (size_t)(span + 1));
        F.hdc_ndiag = exclusive_scan_i32(ctx, flag.as<i32>(), slot.as<i32>(), span, s, true);
        // every diagonal with at least one entry: mark then count
        DSM_HIP(hipMemsetAsync(flag.p, 0, sizeof(i32) * (size_t)span, s));
        hipLaunchKernelGGL(k_diag_mark, dim3(entry_grid(n)), dim3(CB), 0, s, n, C.rp, C.col, flag.as<i32>());
        F.ndiag = exclusive_scan_i32(ctx, flag.as<i32>(), slot.as<i32>(), span, s, true);
        unsigned long long h[2];
        DSM_HIP(hipMemcpyAsync(h, acc.p, sizeof(h), hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
        F.hdc_dia_nnz = (i64)h[0];
        F.near = (i64)h[1];
    }
    return F;
}

// ---------------------------------------------------------------- COO ingest
// Unsorted triplets are ordered by a stable counting sort on rows followed by
// a per-row insertion sort on columns; the result is the canonical (unique)
// order, so the intermediate order of equal rows does not matter.
__global__ void k_row_hist(i64 nnz, i64 nrows, const i32 *row, i32 *cnt, int *err) {
    i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    i32 r = row[k];
    if (r < 0 || (i64)r >= nrows) {
        atomicOr(err, 8);
        return;
    }
    atomicAdd(&cnt[r], 1);
}

__global__ void k_row_bucket(i64 nnz, const i32 *row, const i32 *col, const double *val, i32 *cursor, i32 *ocol,
                             double *oval) {
    i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    i32 p = atomicAdd(&cursor[row[k]], 1);
    ocol[p] = col[k];
    oval[p] = val[k];
}

__global__ void k_row_sort(i64 nrows, i64 ncols, const i32 *rp, i32 *col, double *val, int *err) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    i64 a = rp[i], b = rp[i + 1];
    for (i64 x = a + 1; x < b; x++) {
        i32 c = col[x];
        double v = val[x];
        i64 y = x - 1;
        while (y >= a && col[y] > c) {
            col[y + 1] = col[y];
            val[y + 1] = val[y];
            y--;
        }
        col[y + 1] = c;
        val[y + 1] = v;
    }
    for (i64 x = a; x < b; x++) {
        if (col[x] < 0 || (i64)col[x] >= ncols) atomicOr(err, 8);
        if (x > a && col[x] == col[x - 1]) atomicOr(err, 16);
    }
}

Payload coo_to_csr_payload(dsm_matrix m, const i32 *row, const i32 *col, const double *val, i64 nnz, bool sorted,
                           hipStream_t s) {
    dsm_ctx ctx = m->ctx;
    const i64 n = m->nrows, nc = m->ncols;
    Payload P;
    P.fmt = DSM_CSR;
    P.vdt = DSM_F64;
    P.csr_nnz = nnz;
    try {
        P.rp = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)(n + 1));
        P.col = (i32 *)P.alloc(ctx, sizeof(i32) * (size_t)nnz);
        P.val = P.alloc(ctx, sizeof(double) * (size_t)nnz);
        Tmp err(ctx, sizeof(int));
        DSM_HIP(hipMemsetAsync(err.p, 0, sizeof(int), s));
        if (sorted) {
            hipLaunchKernelGGL(k_coo_rowptr, dim3(grid_for(nnz + 1, CB)), dim3(CB), 0, s, nnz, n, nc, row, col, P.rp,
                               err.as<int>());
            DSM_HIP(hipGetLastError());
            DSM_HIP(hipMemcpyAsync(P.col, col, sizeof(i32) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
            DSM_HIP(hipMemcpyAsync(P.val, val, sizeof(double) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
        } else {
            Tmp cnt(ctx, sizeof(i32) * (size_t)std::max<i64>(n, 1)), cur(ctx, sizeof(i32) * (size_t)(n + 1));
            DSM_HIP(hipMemsetAsync(cnt.p, 0, sizeof(i32) * (size_t)std::max<i64>(n, 1), s));
            if (nnz > 0)
                hipLaunchKernelGGL(k_row_hist, dim3(grid_for(nnz, CB)), dim3(CB), 0, s, nnz, n, row, cnt.as<i32>(),
                                   err.as<int>());
            DSM_HIP(hipGetLastError());
            if (read_flag(err.as<int>(), s)) fail(DSM_E_INVALID, "invalid COO: row index out of range");
            exclusive_scan_i32(ctx, cnt.as<i32>(), P.rp, n, s, false);
            DSM_HIP(hipMemcpyAsync(cur.p, P.rp, sizeof(i32) * (size_t)(n + 1), hipMemcpyDeviceToDevice, s));
            if (nnz > 0)
                hipLaunchKernelGGL(k_row_bucket, dim3(grid_for(nnz, CB)), dim3(CB), 0, s, nnz, row, col, val,
                                   cur.as<i32>(), P.col, (double *)P.val);
            if (n > 0)
                hipLaunchKernelGGL(k_row_sort, dim3(grid_for(n, CB)), dim3(CB), 0, s, n, nc, P.rp, P.col,
                                   (double *)P.val, err.as<int>());
            DSM_HIP(hipGetLastError());
        }
        int f = read_flag(err.as<int>(), s);
        if (f & 8) fail(DSM_E_INVALID, "invalid COO: index out of range");
        if (f & 16) fail(DSM_E_INVALID, "invalid COO: unsorted or duplicate (row, col) entries");
        build_row_blocks(ctx, P, n, s);
    } catch (...) {
        (void)hipStreamSynchronize(s);
        P.release(ctx);
        throw;
    }
    return P;
}

// ---------------------------------------------------------------- stats
bool values_exact(dsm_matrix m, int to, hipStream_t s) {
    const Payload &P = m->P;
    // widening (or keeping) the value type is exact; narrowing order F64, F32, BF16
    if (to <= P.vdt) return true;
    Tmp flag(m->ctx, sizeof(int));
    DSM_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
    auto check = [&](const void *v, i64 n) {
        if (!v || n <= 0) return;
        dim3 g(grid_for(n, CB)), b(CB);
        if (P.vdt == DSM_F64 && to == DSM_F32)
            hipLaunchKernelGGL((k_values_exact<u64, DSM_F64, DSM_F32>), g, b, 0, s, n, (const u64 *)v, flag.as<int>());
        else if (P.vdt == DSM_F64)
            hipLaunchKernelGGL((k_values_exact<u64, DSM_F64, DSM_BF16>), g, b, 0, s, n, (const u64 *)v, flag.as<int>());
        else
            hipLaunchKernelGGL((k_values_exact<u32, DSM_F32, DSM_BF16>), g, b, 0, s, n, (const u32 *)v, flag.as<int>());
        DSM_HIP(hipGetLastError());
    };
    // every stored value of the active format (padding slots hold +0, exact)
    switch (P.fmt) {
    case DSM_CSR: check(P.val, P.csr_nnz); break;
    case DSM_COO: check(P.cval, P.coo_nnz); break;
    case DSM_DIA: check(P.dval, P.ndiag * P.pitch); break;
    case DSM_ELL: check(P.evl, P.K * P.pitch); break;
    case DSM_HYB: check(P.evl, P.K * P.pitch); check(P.cval, P.coo_nnz); break;
    case DSM_HDC: check(P.dval, P.ndiag * P.pitch); check(P.val, P.csr_nnz); break;
    }
    int h = 0;
    DSM_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    DSM_HIP(hipStreamSynchronize(s));
    return h == 0;
}

void row_stats(dsm_matrix m, i64 *out, hipStream_t s) {
    dsm_ctx ctx = m->ctx;
    const i64 n = m->nrows;
    Payload tmp;
    const i32 *rp = nullptr;
    if (m->P.fmt == DSM_CSR) {
        rp = m->P.rp;
    } else {
        tmp = to_csr(m, m->P, s);
        rp = tmp.rp;
    }
    try {
        Tmp acc(ctx, sizeof(unsigned long long) * 38);
        hipLaunchKernelGGL(k_stats_init, dim3(1), dim3(64), 0, s, acc.as<unsigned long long>());
        if (n > 0)
            hipLaunchKernelGGL(k_row_stats, dim3(std::min<unsigned>(grid_for(n, CB), STATS_GRID)), dim3(CB), 0, s, n, rp,
                               acc.as<unsigned long long>());
        DSM_HIP(hipGetLastError());
        unsigned long long h[38];
        DSM_HIP(hipMemcpyAsync(h, acc.p, sizeof(h), hipMemcpyDeviceToHost, s));
        sync(s);
        if (n == 0) h[1] = 0;
        for (int i = 0; i < 38; i++) out[i] = (i64)h[i];
    } catch (...) {
        tmp.release(ctx);
        throw;
    }
    tmp.release(ctx);
}

}  // namespace dsm
