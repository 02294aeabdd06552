// SpMV y = A x for every storage format ("multiply" of the dynamic matrix).
//
// All kernels are bandwidth kernels: no matrix-core work, coalesced sweeps
// over the stored arrays, vector entries gathered through the caches.
// Products are accumulated in the vector type X (FP64 or FP32); stored
// FP32/BF16 values are widened exactly before the multiply.  No kernel uses
// floating-point atomics, so every result is reproducible bit for bit.
//
//   CSR  adaptive row blocks: a workgroup streams one block's entries
//        (fewer than 2*1024, coalesced) into LDS as products, then reduces
//        each row with a power-of-two group of lanes; a row longer than 1024
//        entries gets a workgroup of its own.  Vector variants assign W lanes
//        to each row.
//   DIA  one thread per row sweeps the diagonals in batches; the
//        diagonal-major layout makes every value load and every x load
//        contiguous across a wave.  Variants 16-31 instead stage x in LDS
//        once per cluster of nearby diagonals (k_dia_lds).
//   ELL  one thread per row sweeps the K slots (column-major, coalesced) in
//        batches: all column and value loads, then the x gathers.
//
// Operands that must vanish (past a row, past the last diagonal, a column
// outside the matrix) are read from fixed zero / -1 words rather than
// selected after the load, so every load is unconditional and a lane keeps
// a batch of loads in flight.
//   COO  each wave owns a tile of 64*E consecutive entries (E per lane); rows
//        are combined with a segmented scan across lanes; rows cut by a tile
//        boundary are finished by a second pass that adds the per-tile
//        partials in tile order.
//   HYB  ELL part writes y, then the COO part adds its rows.
//   HDC  DIA part writes y, then the CSR part adds its rows.
#include <hip/hip_ext.h>

#include "clusters.hpp"
#include "core.hpp"

namespace dsm {

constexpr int SB = 256;       // threads per workgroup
constexpr int RB_T = 1024;    // must match the row-block builder
constexpr int CU = 4;         // CSR: entries a lane loads before gathering x
constexpr int COO_E = 4;      // entries per lane in the COO kernel
constexpr int COO_TE = WAVE * COO_E;
constexpr int DIA_LOADS = 8;  // value loads a DIA lane issues per batch (16 measured no faster)

thread_local LaunchTiming *t_launch_timing = nullptr;

// Every SpMV kernel launch goes through DSM_LAUNCH: a plain launch, or, while
// kernel-only timing is on for this thread, one whose events are recorded by
// the dispatch itself (the first launch of the SpMV starts the interval, each
// launch moves its end).
#define DSM_LAUNCH(K, G, B, SH, S, ...)                                                     \
    do {                                                                                   \
        LaunchTiming *lt_ = t_launch_timing;                                               \
        if (lt_) {                                                                         \
            hipEvent_t a_ = lt_->started ? nullptr : lt_->start;                           \
            lt_->started = true;                                                           \
            hipExtLaunchKernelGGL(K, G, B, SH, S, a_, lt_->stop, 0, __VA_ARGS__);          \
        } else {                                                                           \
            hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                               \
        }                                                                                  \
    } while (0)

// Raw words of each size a value load can take, for the nontemporal builtin
// (which takes integer, float and vector types only).
template <int B>
struct raw_word;
template <>
struct raw_word<2> {
    using t = unsigned short;
};
template <>
struct raw_word<4> {
    using t = unsigned int;
};
template <>
struct raw_word<8> {
    using t = unsigned long long;
};
template <>
struct raw_word<16> {
    typedef unsigned int t __attribute__((ext_vector_type(4)));
};

// Load of a stored matrix value.  NT marks it nontemporal: each value is
// read once per SpMV, and the hint lets a sweep that starts with cold caches
// stream its values at a higher rate (a plain read of HPCG 104^3's 252 MB of
// DIA values and y went from 0.69 to 0.76 of the HBM peak).  It also keeps
// them from being retained for the next SpMV, so back-to-back SpMVs whose
// matrix mostly fits the 256 MB Infinity Cache are slower with it: the
// timed selection decides.
template <bool NT, class T>
__device__ __forceinline__ T load_val(const T *p) {
    if constexpr (NT) {
        using W = typename raw_word<sizeof(T)>::t;
        const W w = __builtin_nontemporal_load((const W *)p);
        return __builtin_bit_cast(T, w);
    } else {
        return *p;
    }
}

template <class X>
__device__ __forceinline__ void store_y(X *y, i64 i, X v, bool acc) {
    y[i] = acc ? y[i] + v : v;
}

// ---------------------------------------------------------------- CSR
// DOT (square matrices inside CG): the workgroup also writes its partial of
// x . y over the rows it owns, in FP64, to part[blockIdx.x] (workgroup 0
// counts the launch), as the DIA/ELL sweeps do; every thread of a
// workgroup reaches its reduction.
template <class V, class X, bool ACC, bool XCD, bool NT = false, bool DOT = false>
__global__ void __launch_bounds__(SB) k_csr_adaptive(const i32 *__restrict__ blocks, const i32 *__restrict__ rp,
                                                     const i32 *__restrict__ col, const V *__restrict__ val,
                                                     const X *__restrict__ x, X *__restrict__ y,
                                                     const int *__restrict__ stop, double *__restrict__ part = nullptr,
                                                     long long *count = nullptr) {
    __shared__ int s_stop;
    if (threadIdx.x == 0) s_stop = stop ? *stop : 0;
    __syncthreads();
    if (s_stop) return;
    __shared__ X prod[2 * RB_T];
    __shared__ X red[SB / WAVE];
    const u32 b = XCD ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const int tid = threadIdx.x;
    const i64 r0 = blocks[b], r1 = blocks[b + 1];
    const i64 e0 = rp[r0], e1 = rp[r1];
    if (r1 - r0 == 1 && e1 - e0 > RB_T) {  // one long row: whole workgroup
        // CU entries per lane per pass: all index/value loads are issued
        // before the dependent x gathers, so a lane keeps CU round trips in
        // flight instead of one.
        X s = 0;
        for (i64 base = e0 + tid; base < e1; base += (i64)CU * SB) {
            i32 c[CU];
            V v[CU];
            X xv[CU];
#pragma unroll
            for (int u = 0; u < CU; u++) {
                const i64 e = base + (i64)u * SB;
                c[u] = load_val<NT>(e < e1 ? col + e : sentinel_ptr<i32>());
                v[u] = load_val<NT>(e < e1 ? val + e : zero_ptr<V>());
            }
#pragma unroll
            for (int u = 0; u < CU; u++) xv[u] = *(c[u] >= 0 ? x + c[u] : zero_ptr<X>());
#pragma unroll
            for (int u = 0; u < CU; u++) s += widen<X>(v[u]) * xv[u];
        }
        s = block_sum(s, red);
        if (tid == 0) {
            store_y(y, r0, s, ACC);
            if constexpr (DOT) {
                part[blockIdx.x] = (double)x[r0] * (double)s;
                if (count && blockIdx.x == 0) *count += 1;
            }
        }
        return;
    }
    {
        // fewer than 2*RB_T entries: at most 2*RB_T/SB per lane, loaded
        // together, then gathered together (here the bounds stay branches:
        // whole waves past the block's entries then skip their loads, which
        // measured faster than loading the zero word)
        constexpr int PU = 2 * RB_T / SB;
        const int ne = (int)(e1 - e0);
        i32 c[PU];
        V v[PU];
#pragma unroll
        for (int u = 0; u < PU; u++) {
            const int k = tid + u * SB;
            if (k < ne) {
                c[u] = load_val<NT>(col + e0 + k);
                v[u] = load_val<NT>(val + e0 + k);
            }
        }
#pragma unroll
        for (int u = 0; u < PU; u++) {
            const int k = tid + u * SB;
            if (k < ne) prod[k] = widen<X>(v[u]) * x[c[u]];
        }
    }
    __syncthreads();
    const int nr = (int)(r1 - r0);
    const int avg = (int)((e1 - e0 + nr - 1) / nr);
    int L = 1;
    while (L < WAVE && 2 * L * nr <= SB && L < avg) L <<= 1;
    const int rl = tid / L, lane = tid % L;
    X s = 0;
    if (rl < nr) {
        const int a = (int)(rp[r0 + rl] - e0), c = (int)(rp[r0 + rl + 1] - e0);
        // four independent sums, so a lane has four LDS reads in flight
        // instead of one dependent read per product (Zipf 1M: 205 -> 186 us;
        // rows of hundreds of entries inside a row block gave a long chain;
        // eight sums measured no faster)
        X s4[4] = {0, 0, 0, 0};
        int k = a + lane;
        for (; k + 3 * L < c; k += 4 * L) {
#pragma unroll
            for (int u = 0; u < 4; u++) s4[u] += prod[k + u * L];
        }
        for (; k < c; k += L) s4[0] += prod[k];
        s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    for (int off = L >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
    if (rl < nr && lane == 0) store_y(y, r0 + rl, s, ACC);
    if constexpr (DOT) {
        __shared__ double dred[SB / WAVE];
        double d = rl < nr && lane == 0 ? (double)x[r0 + rl] * (double)s : 0.0;
        d = block_sum(d, dred);
        if (tid == 0) {
            part[blockIdx.x] = d;
            if (count && blockIdx.x == 0) *count += 1;
        }
    }
}

template <class V, class X, int W, bool ACC, bool NT = false, bool DOT = false>
__global__ void __launch_bounds__(SB) k_csr_vector(i64 nrows, const i32 *__restrict__ rp, const i32 *__restrict__ col,
                                                   const V *__restrict__ val, const X *__restrict__ x,
                                                   X *__restrict__ y, const int *__restrict__ stop,
                                                   double *__restrict__ part = nullptr, long long *count = nullptr) {
    if (stop && *stop) return;
    // launch order, not the XCD-aware order: with it the HPCG 104^3 launch
    // fetched 382 instead of 456 MB (no x lines fetched into several L2s)
    // but ran 3% slower, this kernel being bound by gather latency
    const i64 row = ((i64)blockIdx.x * SB + threadIdx.x) / W;
    const int lane = threadIdx.x % W;
    X s = 0;
    if (row < nrows) {
        const i64 a = rp[row], c = rp[row + 1];
        for (i64 base = a + lane; base < c; base += (i64)CU * W) {
            i32 cc[CU];
            V v[CU];
            X xv[CU];
#pragma unroll
            for (int u = 0; u < CU; u++) {
                const i64 e = base + (i64)u * W;
                cc[u] = load_val<NT>(e < c ? col + e : sentinel_ptr<i32>());
                v[u] = load_val<NT>(e < c ? val + e : zero_ptr<V>());
            }
#pragma unroll
            for (int u = 0; u < CU; u++) xv[u] = *(cc[u] >= 0 ? x + cc[u] : zero_ptr<X>());
#pragma unroll
            for (int u = 0; u < CU; u++) s += widen<X>(v[u]) * xv[u];
        }
    }
    s = group_sum<W>(s);
    if (row < nrows && lane == 0) store_y(y, row, s, ACC);
    if constexpr (DOT) {
        __shared__ double dred[SB / WAVE];
        double d = row < nrows && lane == 0 ? (double)x[row] * (double)s : 0.0;
        d = block_sum(d, dred);
        if (threadIdx.x == 0) {
            part[blockIdx.x] = d;
            if (count && blockIdx.x == 0) *count += 1;
        }
    }
}

// ---------------------------------------------------------------- DIA / ELL
// Variant bits shared by the DIA and ELL sweeps: bit 0 turns the XCD-aware
// tile order off, bits 1-2 give log2 of the row groups per thread (1, 2, 4;
// each group has its own accumulators, so more loads are in flight), bit 3
// makes a group two adjacent rows whose stored values (and ELL column
// indices) are fetched with one load of twice the width.
template <class V>
struct alignas(2 * sizeof(V)) pair2 {
    V a, b;
};

// Square sweeps inside CG: the workgroup's partial of x . y (p . q with
// x = p, y = q = A p) over its own rows, accumulated in FP64 and stored in
// part[blockIdx.x]; workgroup 0 also counts the launch.  Every thread
// reaches the barrier: the early exit on `stop` is uniform (the flag is
// written only by other launches).
template <class X, int R, int RW>
__device__ __forceinline__ void dot_epilogue(const X (&s)[R][RW], const X *__restrict__ x, i64 i0, i64 nrows,
                                             double *__restrict__ part, long long *count) {
    __shared__ double lds[SB / WAVE];
    double acc = 0;
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int w = 0; w < RW; w++) {
            const i64 i = i0 + (i64)r * SB * RW + w;
            if (i < nrows) acc += (double)x[i] * (double)s[r][w];
        }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc;
        if (count && blockIdx.x == 0) *count += 1;
    }
}

// Diagonals (ELL: slots) per batch of the DIA and ELL sweeps: every load of
// a batch (values and x, for all row groups) is issued before its products
// are summed, so a lane has 2 * KU * R * RW loads in flight.
template <int R, int RW>
constexpr int dia_batch() {
    return (R * RW) >= DIA_LOADS ? 1 : DIA_LOADS / (R * RW);
}

template <class V, class X, bool ACC, bool XCD, int R, bool P2, bool DOT = false, bool NT = false>
__global__ void __launch_bounds__(SB) k_dia(i64 nrows, i64 ncols, i64 ndiag, const i32 *__restrict__ offs,
                                            const V *__restrict__ dval, i64 pitch, const X *__restrict__ x,
                                            X *__restrict__ y, const int *__restrict__ stop,
                                            double *__restrict__ part = nullptr, long long *count = nullptr) {
    if (stop && *stop) return;
    constexpr int RW = P2 ? 2 : 1;
    constexpr int KU = dia_batch<R, RW>();
    const u32 b = XCD ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const i64 i0 = (i64)b * SB * R * RW + (i64)threadIdx.x * RW;
    X s[R][RW];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int w = 0; w < RW; w++) s[r][w] = 0;
    // A slot whose column lies outside the matrix is padding (+0), and its x
    // operand is the zero word, so its product is +0 exactly as if it were
    // skipped; slots past the last diagonal and rows past the end read the
    // zero word for both operands (rows past the end are never stored).
    // Zero slots inside the column range drop their x operand after the load
    // (a select on registers that are both loaded anyway).
    //
    // Rows this wave covers (all groups): [wlo, whi], as scalars.  A batch
    // whose diagonals all exist and whose columns stay inside the matrix for
    // every one of these rows (offsets ascend, so the first and last offset
    // of the batch decide) takes the interior path: plain loads, no bounds
    // tests or operand selects per element.  Only tiles near the first and
    // last rows of a banded matrix take the general path.  FP32/BF16 values
    // only: there the per-element index work limits the sweep (BF16 at HPCG
    // 128^3: 27.3 -> 22.7 us); FP64 sweeps measured 2-5% slower with it.
    constexpr bool INTERIOR = sizeof(V) < sizeof(double);
    const i64 wlo = (i64)b * SB * R * RW + (i64)__builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~(WAVE - 1))) * RW;
    const i64 whi = wlo + (i64)(R - 1) * SB * RW + (i64)WAVE * RW - 1;
    for (i64 k0 = 0; k0 < ndiag; k0 += KU) {
        V v[KU][R][RW];
        X xv[KU][R][RW];
        if (INTERIOR && k0 + KU <= ndiag && whi < nrows && wlo + offs[k0] >= 0 && whi + offs[k0 + KU - 1] < ncols) {
#pragma unroll
            for (int u = 0; u < KU; u++) {
                const i64 off = offs[k0 + u];
                const V *dk = dval + (k0 + u) * pitch;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const i64 i = i0 + (i64)r * SB * RW;
                    if constexpr (P2) {
                        const pair2<V> pv = load_val<NT>((const pair2<V> *)(dk + i));
                        v[u][r][0] = pv.a;
                        v[u][r][1] = pv.b;
                        xv[u][r][0] = x[i + off];
                        xv[u][r][1] = x[i + off + 1];
                    } else {
                        v[u][r][0] = load_val<NT>(dk + i);
                        xv[u][r][0] = x[i + off];
                    }
                }
            }
        } else {
#pragma unroll
        for (int u = 0; u < KU; u++) {
            // offs is zero-padded to a multiple of 16 entries (KU divides 16)
            const bool kin = k0 + u < ndiag;
            const i64 k = k0 + u;
            const i64 off = offs[k];
            const V *dk = dval + (kin ? k : 0) * pitch;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const i64 i = i0 + (i64)r * SB * RW;
                const i64 j = i + off;
                if constexpr (P2) {
                    // i is even and the pitch a multiple of 64, so the pair is
                    // aligned; slot i + 1 < pitch always exists (padding is 0)
                    const pair2<V> pv = load_val<NT>(kin && i < nrows ? (const pair2<V> *)(dk + i) : zero_ptr<pair2<V>>());
                    v[u][r][0] = pv.a;
                    v[u][r][1] = pv.b;
                    const bool ok0 = kin && i < nrows && j >= 0 && j < ncols;
                    const bool ok1 = kin && i + 1 < nrows && j + 1 >= 0 && j + 1 < ncols;
                    xv[u][r][0] = *(ok0 ? x + j : zero_ptr<X>());
                    xv[u][r][1] = *(ok1 ? x + j + 1 : zero_ptr<X>());
                } else {
                    const bool ok = kin && i < nrows && j >= 0 && j < ncols;
                    v[u][r][0] = load_val<NT>(kin && i < nrows ? dk + i : zero_ptr<V>());
                    xv[u][r][0] = *(ok ? x + j : zero_ptr<X>());
                }
            }
        }
        }
        // pin every x operand as loaded: the select below then stays a
        // register select instead of a branch around the load
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int w = 0; w < RW; w++) asm volatile("" : "+v"(xv[u][r][w]));
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int w = 0; w < RW; w++) {
                    // a zero slot (padding or a stored zero, which DIA cannot
                    // tell apart) is no entry: its x operand does not count,
                    // so a non-finite x entry reaches only the rows that
                    // store a nonzero in its column
                    const X wv = widen<X>(v[u][r][w]);
                    s[r][w] += wv * (wv != (X)0 ? xv[u][r][w] : (X)0);
                }
    }
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int w = 0; w < RW; w++) {
            const i64 i = i0 + (i64)r * SB * RW + w;
            if (i < nrows) store_y(y, i, s[r][w], ACC);
        }
    if constexpr (DOT) dot_epilogue<X, R, RW>(s, x, i0, nrows, part, count);
}

// One cluster of the LDS-staged sweep (the records clusters.hpp builds).
struct alignas(64) CluRec {
    i32 kb, ke, lo, hi;
    i32 d[CLU_MAXK];  // offsets of diagonals kb.. relative to lo, 0 past ke
};
static_assert(sizeof(CluRec) == CLU_REC * sizeof(i32), "cluster record layout");
static_assert(DIA_CLUSTER_K <= CLU_MAXK, "a cluster record holds CLU_MAXK relative offsets");

// DIA sweep with x staged in LDS (variant bit 4).  A workgroup owns
// T = SB*R*RW consecutive rows (thread t: rows r0 + t*RW + q*SB*RW (+1 with
// paired rows, whose values come in one double-width load)).  For each cluster of
// nearby diagonals (offsets lo..hi, at most DIA_CLUSTER_SPAN apart) it
// loads the x window [r0 + lo, r0 + hi + T) once, coalesced, into LDS, and
// every diagonal of the cluster reads its operands there instead of
// gathering them from L2: the 27 diagonals of a 27-point stencil need 3
// window loads instead of 27 gathers.  Columns outside the matrix read +0
// (their slots are padding, +0); zero slots drop their operand as in k_dia.
// Measured faster than k_dia beyond the Infinity Cache (HPCG 128^3 and
// 144^3), slower at 104^3, where k_dia's gathers hit the caches.
template <class V, class X, bool ACC, bool XCD, int R, bool P2, bool DOT = false, bool NT = false>
__global__ void __launch_bounds__(SB) k_dia_lds(i64 nrows, i64 ncols, i64 nclu, const i32 *__restrict__ clu,
                                                const i32 *__restrict__ offs, const V *__restrict__ dval, i64 pitch,
                                                const X *__restrict__ x, X *__restrict__ y,
                                                const int *__restrict__ stop, double *__restrict__ part = nullptr,
                                                long long *count = nullptr) {
    if (stop && *stop) return;
    constexpr int RW = P2 ? 2 : 1;
    constexpr int T = SB * R * RW;
    constexpr int WMAX = T + DIA_CLUSTER_SPAN;
    constexpr int WP = (WMAX + SB - 1) / SB;
    // A cluster holds up to KC = 9 diagonals (the nine of one z-plane of a
    // 27-point stencil), so one cluster's value loads keep 9 (18 with row
    // pairs) loads per thread in flight, and a 27-point sweep has three
    // windows and six barriers.  Clusters of at most 3 diagonals (64 apart)
    // needed the loads of three clusters issued together to reach the same
    // depth and nine windows and eighteen barriers: 46.8 against 45.0-45.4
    // us for the cold sweep of HPCG 104^3 (variant 56) on one box.
    constexpr int KC = DIA_CLUSTER_K;
    __shared__ X xs[WMAX];
    const u32 b = XCD ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const i64 r0 = (i64)b * T;
    const int t0 = threadIdx.x * RW;  // first row of this thread's group 0, within the tile
    X s[R][RW];
#pragma unroll
    for (int q = 0; q < R; q++)
#pragma unroll
        for (int w = 0; w < RW; w++) s[q][w] = 0;
    // one cluster's operands in registers: its x window and its values
    struct Stage {
        X win[WP];
        V v[KC][R][RW];
        int d[KC];
        int W;
    };
    auto load = [&](i64 c, Stage &st) {
        // the cluster's record in one scalar load (no dependent offset loads)
        const CluRec r = ((const CluRec *)clu)[c];
        const i64 kb = r.kb, ke = r.ke, lo = r.lo, hi = r.hi;
        const i64 base = r0 + lo;
        const int W = T + (int)(hi - lo);
        st.W = W;
        // FP32/BF16 values: a cluster with all KC diagonals, rows all inside
        // the matrix and a window inside x takes plain loads (the index work
        // per element limits those sweeps, as in k_dia)
        if (sizeof(V) < sizeof(double) && ke - kb == KC && r0 + T <= nrows && base >= 0 && base + W <= ncols) {
#pragma unroll
            for (int p = 0; p < WP; p++) {
                const int t = threadIdx.x + p * SB;
                st.win[p] = x[base + min(t, W - 1)];
            }
#pragma unroll
            for (int u = 0; u < KC; u++) {
                st.d[u] = r.d[u];
                const V *dk = dval + (kb + u) * pitch;
#pragma unroll
                for (int q = 0; q < R; q++) {
                    const i64 i = r0 + t0 + (i64)q * SB * RW;
                    if constexpr (P2) {
                        const pair2<V> pv = load_val<NT>((const pair2<V> *)(dk + i));
                        st.v[u][q][0] = pv.a;
                        st.v[u][q][1] = pv.b;
                    } else {
                        st.v[u][q][0] = load_val<NT>(dk + i);
                    }
                }
            }
        } else {
#pragma unroll
            for (int p = 0; p < WP; p++) {
                const int t = threadIdx.x + p * SB;
                const i64 j = base + t;
                st.win[p] = *(t < W && j >= 0 && j < ncols ? x + j : zero_ptr<X>());
            }
#pragma unroll
            for (int u = 0; u < KC; u++) {
                const bool kin = kb + u < ke;
                st.d[u] = r.d[u];  // 0 past the cluster's last diagonal
#pragma unroll
                for (int q = 0; q < R; q++) {
                    const i64 i = r0 + t0 + (i64)q * SB * RW;
                    const V *dk = dval + (kb + u) * pitch;
                    if constexpr (P2) {
                        // i is even and the pitch a multiple of 64: the pair is
                        // aligned and slot i + 1 < pitch exists (padding is 0)
                        const pair2<V> pv =
                            load_val<NT>(kin && i < nrows ? (const pair2<V> *)(dk + i) : zero_ptr<pair2<V>>());
                        st.v[u][q][0] = pv.a;
                        st.v[u][q][1] = pv.b;
                    } else {
                        st.v[u][q][0] = load_val<NT>(kin && i < nrows ? dk + i : zero_ptr<V>());
                    }
                }
            }
        }
    };
    auto consume = [&](const Stage &st) {
        __syncthreads();  // the previous cluster's reads of xs are done
#pragma unroll
        for (int p = 0; p < WP; p++) {
            const int t = threadIdx.x + p * SB;
            if (t < st.W) xs[t] = st.win[p];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < KC; u++)
#pragma unroll
            for (int q = 0; q < R; q++)
#pragma unroll
                for (int w = 0; w < RW; w++) {
                    X xv = xs[t0 + q * SB * RW + w + st.d[u]];
                    asm volatile("" : "+v"(xv));
                    const X wv = widen<X>(st.v[u][q][w]);
                    s[q][w] += wv * (wv != (X)0 ? xv : (X)0);
                }
    };
    for (i64 c = 0; c < nclu; c++) {
        Stage st;
        load(c, st);
        consume(st);
    }
#pragma unroll
    for (int q = 0; q < R; q++)
#pragma unroll
        for (int w = 0; w < RW; w++) {
            const i64 i = r0 + t0 + (i64)q * SB * RW + w;
            if (i < nrows) store_y(y, i, s[q][w], ACC);
        }
    if constexpr (DOT) dot_epilogue<X, R, RW>(s, x, r0 + t0, nrows, part, count);
}

template <class V, class X, bool ACC, bool XCD, int R, bool P2, bool DOT = false>
__global__ void __launch_bounds__(SB) k_ell(i64 nrows, i64 K, i64 pitch, const i32 *__restrict__ ecol,
                                            const V *__restrict__ evl, const X *__restrict__ x, X *__restrict__ y,
                                            const int *__restrict__ stop, double *__restrict__ part = nullptr,
                                            long long *count = nullptr) {
    if (stop && *stop) return;
    constexpr int RW = P2 ? 2 : 1;
    constexpr int KU = dia_batch<R, RW>();
    const u32 b = XCD ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const i64 i0 = (i64)b * SB * R * RW + (i64)threadIdx.x * RW;
    X s[R][RW];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int w = 0; w < RW; w++) s[r][w] = 0;
    // Batches of KU slots: all column and value loads of a batch, then all
    // x gathers, then the products.  Padding slots (column -1, value +0)
    // take their x operand from the zero word, so their product is +0
    // exactly as if skipped; slots past K and rows past the end read the
    // sentinel column and the zero value (rows past the end are never
    // stored).  A pair load at the last (even) row also reads the padding
    // row after it, which exists below the pitch.
    for (i64 k0 = 0; k0 < K; k0 += KU) {
        i32 c[KU][R][RW];
        V v[KU][R][RW];
        X xv[KU][R][RW];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int r = 0; r < R; r++) {
                const i64 i = i0 + (i64)r * SB * RW;
                const bool live = k0 + u < K && i < nrows;
                const i64 slot = (k0 + u) * pitch + i;
                if constexpr (P2) {
                    const pair2<i32> cc = *(live ? (const pair2<i32> *)(ecol + slot) : sentinel_ptr<pair2<i32>>());
                    const pair2<V> vv = *(live ? (const pair2<V> *)(evl + slot) : zero_ptr<pair2<V>>());
                    c[u][r][0] = cc.a;
                    c[u][r][1] = cc.b;
                    v[u][r][0] = vv.a;
                    v[u][r][1] = vv.b;
                } else {
                    c[u][r][0] = *(live ? ecol + slot : sentinel_ptr<i32>());
                    v[u][r][0] = *(live ? evl + slot : zero_ptr<V>());
                }
            }
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int w = 0; w < RW; w++) {
                    const i32 cc = c[u][r][w];
                    xv[u][r][w] = *(cc >= 0 ? x + cc : zero_ptr<X>());
                }
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int w = 0; w < RW; w++) s[r][w] += widen<X>(v[u][r][w]) * xv[u][r][w];
    }
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int w = 0; w < RW; w++) {
            const i64 i = i0 + (i64)r * SB * RW + w;
            if (i < nrows) store_y(y, i, s[r][w], ACC);
        }
    if constexpr (DOT) dot_epilogue<X, R, RW>(s, x, i0, nrows, part, count);
}

// ---------------------------------------------------------------- COO
// Tile = one wave's 64*E consecutive entries.  Per tile the kernel records
// head = sum of the tile's entries of its first row, tail = sum of the
// entries of its last row.  A row is written here when it both starts and
// ends inside the tile; a row that starts in this tile and runs on is
// written by k_coo_fixup; a row that started in an earlier tile only
// contributes its head.  Empty rows are zeroed by the lane that holds the
// entry following the gap (non-accumulating mode).
template <class V, class X, int E, bool ACC>
__global__ void __launch_bounds__(SB) k_coo_tiles(i64 nnz, i64 nrows, const i32 *__restrict__ row,
                                                  const i32 *__restrict__ col, const V *__restrict__ val,
                                                  const X *__restrict__ x, X *__restrict__ y,
                                                  X *__restrict__ head_val, X *__restrict__ tail_val,
                                                  const int *__restrict__ stop) {
    if (stop && *stop) return;
    constexpr i32 SENT = INT32_MAX;
    constexpr i64 TE = (i64)WAVE * E;
    const int lane = threadIdx.x % WAVE;
    const i64 tile = (i64)xcd_tile(blockIdx.x, gridDim.x) * (SB / WAVE) + threadIdx.x / WAVE;
    const i64 t0 = tile * TE;
    if (t0 >= nnz) return;  // uniform per wave
    const i64 t1 = min(t0 + TE, nnz);
    const i64 base = t0 + (i64)lane * E;
    const int cnt = (int)max((i64)0, min((i64)E, t1 - base));

    // entries past the end read the sentinel word as row and column (the
    // row becomes SENT) and the zero word as value and x operand
    i32 r[E], c[E];
    V v[E];
    X p[E];
#pragma unroll
    for (int k = 0; k < E; k++) {
        const bool in = k < cnt;
        r[k] = *(in ? row + base + k : sentinel_ptr<i32>());
        c[k] = *(in ? col + base + k : sentinel_ptr<i32>());
        v[k] = *(in ? val + base + k : zero_ptr<V>());
    }
#pragma unroll
    for (int k = 0; k < E; k++) r[k] = r[k] < 0 ? SENT : r[k];
#pragma unroll
    for (int k = 0; k < E; k++) p[k] = widen<X>(v[k]) * *(c[k] >= 0 ? x + c[k] : zero_ptr<X>());
    const i32 fr = cnt > 0 ? r[0] : SENT;
    const i32 lr = cnt > 0 ? r[cnt - 1] : SENT;

    // tile-level facts (uniform in the wave)
    const i32 first_row = row[t0];
    const bool head_before = t0 > 0 && row[t0 - 1] == first_row;
    const i32 next_tile_row = t1 < nnz ? row[t1] : SENT;

    // empty rows before this lane's first entry / after the last entry
    if (!ACC && cnt > 0) {
        const i64 prev = base > 0 ? (i64)row[base - 1] : -1;
        for (i64 g = prev + 1; g < fr; g++) y[g] = 0;
        if (base + cnt == nnz)
            for (i64 g = (i64)lr + 1; g < nrows; g++) y[g] = 0;
    }

    // lane-local pass: interior rows are complete here
    X fsum = 0, cur = 0;
    bool first_done = false;
    i32 cr = fr;
#pragma unroll
    for (int k = 0; k < E; k++) {
        if (k >= cnt) break;
        if (r[k] != cr) {
            if (!first_done) {
                fsum = cur;
                first_done = true;
            } else {
                store_y(y, cr, cur, ACC);
            }
            if (!ACC)
                for (i64 g = (i64)cr + 1; g < r[k]; g++) y[g] = 0;
            cr = r[k];
            cur = 0;
        }
        cur += p[k];
    }
    const X lsum = cur;
    if (!first_done) fsum = cur;

    // segmented inclusive scan of the last-row sums across lanes
    i32 lr_prev = __shfl_up(lr, 1, WAVE);
    const int head_flag = (lane == 0 || !(fr == lr && lr_prev == fr)) ? 1 : 0;
    X T = lsum;
    int h = head_flag;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        X tv = __shfl_up(T, off, WAVE);
        int th = __shfl_up(h, off, WAVE);
        if (lane >= off && !h) {
            T += tv;
            h = th;
        }
    }
    const X T_prev = __shfl_up(T, 1, WAVE);
    i32 fr_next = __shfl_down(fr, 1, WAVE);
    if (lane == WAVE - 1) fr_next = next_tile_row;
    if (cnt == 0) return;

    // first row of the lane when it ends inside the lane
    if (fr != lr) {
        const X w = fsum + ((lane > 0 && lr_prev == fr) ? T_prev : (X)0);
        if (fr == first_row && head_before) head_val[tile] = w;
        else store_y(y, fr, w, ACC);
    }
    // last row of the lane
    const bool ends_here = fr_next != lr;
    const bool lr_started_before = lr == first_row && head_before;
    if (ends_here) {
        if (lr_started_before) head_val[tile] = T;
        else store_y(y, lr, T, ACC);
    }
    if (base + cnt == t1) {
        // the wave's last real lane records the tile tail; a tile holding a
        // single row that runs on from earlier tiles also records it as head
        tail_val[tile] = T;
        if (!ends_here && lr_started_before) head_val[tile] = T;
    }
}

// Rows that cross tile boundaries: the tile where such a row starts adds its
// tail to the heads of the following tiles, in tile order.
template <class X, int E, bool ACC>
__global__ void k_coo_fixup(i64 nnz, i64 ntiles, const i32 *__restrict__ row, const X *__restrict__ head_val,
                            const X *__restrict__ tail_val, X *__restrict__ y, const int *__restrict__ stop) {
    if (stop && *stop) return;
    constexpr i64 TE = (i64)WAVE * E;
    const i64 u = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= ntiles) return;
    const i64 t0 = u * TE, t1 = min(t0 + TE, nnz);
    const i32 last = row[t1 - 1];
    const bool starts_here = row[t0] != last || t0 == 0 || row[t0 - 1] != last;
    const bool continues = t1 < nnz && row[t1] == last;
    if (!starts_here || !continues) return;
    X total = tail_val[u];
    for (i64 v = u + 1; v < ntiles; v++) {
        total += head_val[v];
        const i64 v1 = min((v + 1) * TE, nnz);
        if (!(v1 < nnz && row[v1] == last)) break;
    }
    store_y(y, last, total, ACC);
}

template <class X>
__global__ void k_fill(i64 n, X *y, X v, const int *stop) {
    if (stop && *stop) return;
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}

// ================================================================ host dispatch
template <class V, class X>
static void coo_launch(dsm_matrix m, i64 nnz, const i32 *row, const i32 *col, const V *val, const X *x, X *y,
                       bool acc, hipStream_t s, Workspace *scratch, const int *stop) {
    const i64 n = m->nrows;
    if (nnz == 0) {
        if (!acc && n > 0) DSM_LAUNCH(k_fill<X>, dim3(grid_for(n, SB)), dim3(SB), 0, s, n, y, (X)0, stop);
        return;
    }
    const i64 ntiles = (nnz + COO_TE - 1) / COO_TE;
    X *part = (X *)ws_get(m->ctx, scratch ? *scratch : m->ws, sizeof(X) * (size_t)(2 * ntiles), s);
    X *head = part, *tail = part + ntiles;
    const unsigned g = grid_for(ntiles, SB / WAVE);
    if (acc) {
        DSM_LAUNCH((k_coo_tiles<V, X, COO_E, true>), dim3(g), dim3(SB), 0, s, nnz, n, row, col, val, x, y,
                           head, tail, stop);
        DSM_LAUNCH((k_coo_fixup<X, COO_E, true>), dim3(grid_for(ntiles, SB)), dim3(SB), 0, s, nnz, ntiles,
                           row, head, tail, y, stop);
    } else {
        DSM_LAUNCH((k_coo_tiles<V, X, COO_E, false>), dim3(g), dim3(SB), 0, s, nnz, n, row, col, val, x, y,
                           head, tail, stop);
        DSM_LAUNCH((k_coo_fixup<X, COO_E, false>), dim3(grid_for(ntiles, SB)), dim3(SB), 0, s, nnz, ntiles,
                           row, head, tail, y, stop);
    }
}

// CSR launches; returns the number of workgroups (= partials with DOT).
template <class V, class X, bool ACC, bool NT, bool DOT = false>
static unsigned csr_launch_nt(dsm_matrix m, const Payload &P, const X *x, X *y, int variant, hipStream_t s,
                              const int *stop, double *part = nullptr, long long *count = nullptr) {
    const i64 n = m->nrows;
    if (n == 0) return 0;
    const V *val = (const V *)P.val;
    if (variant == 0 || variant >= 7) {
        if (P.nrblocks == 0) return 0;
        if (variant == 0)
            DSM_LAUNCH((k_csr_adaptive<V, X, ACC, true, NT, DOT>), dim3((unsigned)P.nrblocks), dim3(SB), 0, s,
                       P.rblocks, P.rp, P.col, val, x, y, stop, part, count);
        else
            DSM_LAUNCH((k_csr_adaptive<V, X, ACC, false, NT, DOT>), dim3((unsigned)P.nrblocks), dim3(SB), 0, s,
                       P.rblocks, P.rp, P.col, val, x, y, stop, part, count);
        return (unsigned)P.nrblocks;
    }
    const int W = 1 << variant;  // 2 .. 64
    const unsigned g = grid_for(n * W, SB);
#define VEC(WW)                                                                                                \
    DSM_LAUNCH((k_csr_vector<V, X, WW, ACC, NT, DOT>), dim3(g), dim3(SB), 0, s, n, P.rp, P.col, val, x, y, stop, \
               part, count)
    switch (W) {
    case 2: VEC(2); break;
    case 4: VEC(4); break;
    case 8: VEC(8); break;
    case 16: VEC(16); break;
    case 32: VEC(32); break;
    default: VEC(64); break;
    }
#undef VEC
    return g;
}

// Workgroups (= partials) a CSR launch of this variant runs.
static i64 csr_groups(dsm_matrix m, const Payload &P, int variant) {
    const int v = variant & ~CSR_VARIANT_NT;
    if (v == 0 || v >= 7) return P.nrblocks;
    return grid_for(m->nrows * (1 << v), SB);
}

// CSR variants: 0 adaptive row blocks (XCD-aware order), 1-6 vector
// kernels with 2^v lanes per row, 7 adaptive in launch order; plus 8 (bit 3):
// column indices and values loaded nontemporally, so the single-use matrix
// stream does not displace the x lines that later gathers hit in the L2.
template <class V, class X, bool ACC, bool DOT = false>
static unsigned csr_launch(dsm_matrix m, const Payload &P, const X *x, X *y, int variant, hipStream_t s,
                           const int *stop, double *part = nullptr, long long *count = nullptr) {
    if (variant & CSR_VARIANT_NT)
        return csr_launch_nt<V, X, ACC, true, DOT>(m, P, x, y, variant & ~CSR_VARIANT_NT, s, stop, part, count);
    return csr_launch_nt<V, X, ACC, false, DOT>(m, P, x, y, variant, s, stop, part, count);
}

// Launch geometry of a sweep variant (workgroups = partials of the dot form).
static unsigned sweep_groups(i64 n, int variant) {
    const int lr = (variant >> 1) & 3, R = lr == 0 ? 1 : (lr == 1 ? 2 : 4);
    return grid_for(n, SB * R * (((variant >> 3) & 1) ? 2 : 1));
}

template <class V, class X, bool ACC, bool XCD, int R, bool P2, bool DOT, bool NT>
static void sweep_lds_launch(dsm_matrix m, const Payload &P, const X *x, X *y, hipStream_t s, const int *stop,
                             double *part, long long *count) {
    const i64 n = m->nrows;
    DSM_LAUNCH((k_dia_lds<V, X, ACC, XCD, R, P2, DOT, NT>), dim3(grid_for(n, SB * R * (P2 ? 2 : 1))), dim3(SB),
               0, s, n, m->ncols, P.nclu, P.clu, P.offs, (const V *)P.dval, P.pitch, x, y, stop, part, count);
}

template <class V, class X, bool ACC, bool XCD, bool P2, bool DOT, bool NT>
static void sweep_lds_r(dsm_matrix m, const Payload &P, const X *x, X *y, int lr, hipStream_t s, const int *stop,
                        double *part, long long *count) {
    if (lr == 0) sweep_lds_launch<V, X, ACC, XCD, 1, P2, DOT, NT>(m, P, x, y, s, stop, part, count);
    else if (lr == 1) sweep_lds_launch<V, X, ACC, XCD, 2, P2, DOT, NT>(m, P, x, y, s, stop, part, count);
    else sweep_lds_launch<V, X, ACC, XCD, 4, P2, DOT, NT>(m, P, x, y, s, stop, part, count);
}

// NT (nontemporal value loads) exists for the DIA sweep only.
template <class V, class X, bool ACC, bool XCD, int R, bool P2, bool DOT, bool NT>
static void sweep_launch(dsm_matrix m, const Payload &P, const X *x, X *y, hipStream_t s, const int *stop,
                         double *part, long long *count) {
    const i64 n = m->nrows;
    const unsigned g = grid_for(n, SB * R * (P2 ? 2 : 1));
    if (NT || P.fmt == DSM_DIA || P.fmt == DSM_HDC) {
        DSM_LAUNCH((k_dia<V, X, ACC, XCD, R, P2, DOT, NT>), dim3(g), dim3(SB), 0, s, n, m->ncols, P.ndiag, P.offs,
                   (const V *)P.dval, P.pitch, x, y, stop, part, count);
    } else if constexpr (!NT) {
        DSM_LAUNCH((k_ell<V, X, ACC, XCD, R, P2, DOT>), dim3(g), dim3(SB), 0, s, n, P.K, P.pitch, P.ecol,
                   (const V *)P.evl, x, y, stop, part, count);
    }
}

template <class V, class X, bool ACC, bool XCD, bool P2, bool DOT, bool NT>
static void sweep_r(dsm_matrix m, const Payload &P, const X *x, X *y, int lr, hipStream_t s, const int *stop,
                    double *part, long long *count) {
    if (lr == 0) sweep_launch<V, X, ACC, XCD, 1, P2, DOT, NT>(m, P, x, y, s, stop, part, count);
    else if (lr == 1) sweep_launch<V, X, ACC, XCD, 2, P2, DOT, NT>(m, P, x, y, s, stop, part, count);
    else sweep_launch<V, X, ACC, XCD, 4, P2, DOT, NT>(m, P, x, y, s, stop, part, count);
}

template <class V, class X, bool ACC, bool DOT, bool NT>
static void sweep_nt(dsm_matrix m, const Payload &P, const X *x, X *y, int variant, hipStream_t s, const int *stop,
                     double *part, long long *count) {
    const bool xcd = !(variant & 1), p2 = (variant >> 3) & 1;
    const int lr = (variant >> 1) & 3;
    if (((variant >> 4) & 1) && (P.fmt == DSM_DIA || P.fmt == DSM_HDC)) {
        if (xcd && p2) sweep_lds_r<V, X, ACC, true, true, DOT, NT>(m, P, x, y, lr, s, stop, part, count);
        else if (xcd) sweep_lds_r<V, X, ACC, true, false, DOT, NT>(m, P, x, y, lr, s, stop, part, count);
        else if (p2) sweep_lds_r<V, X, ACC, false, true, DOT, NT>(m, P, x, y, lr, s, stop, part, count);
        else sweep_lds_r<V, X, ACC, false, false, DOT, NT>(m, P, x, y, lr, s, stop, part, count);
        return;
    }
    if (xcd && p2) sweep_r<V, X, ACC, true, true, DOT, NT>(m, P, x, y, lr, s, stop, part, count);
    else if (xcd) sweep_r<V, X, ACC, true, false, DOT, NT>(m, P, x, y, lr, s, stop, part, count);
    else if (p2) sweep_r<V, X, ACC, false, true, DOT, NT>(m, P, x, y, lr, s, stop, part, count);
    else sweep_r<V, X, ACC, false, false, DOT, NT>(m, P, x, y, lr, s, stop, part, count);
}

// Bit 5 (nontemporal value loads) applies to DIA/HDC; the dot form inside CG
// runs the same sweep with plain loads (identical results: the hint changes
// only what the caches keep).
template <class V, class X, bool ACC, bool DOT = false>
static void sweep(dsm_matrix m, const Payload &P, const X *x, X *y, int variant, hipStream_t s, const int *stop,
                  double *part = nullptr, long long *count = nullptr) {
    if constexpr (!DOT) {
        if ((variant & DIA_VARIANT_NT) && (P.fmt == DSM_DIA || P.fmt == DSM_HDC)) {
            sweep_nt<V, X, ACC, false, true>(m, P, x, y, variant, s, stop, part, count);
            return;
        }
    }
    sweep_nt<V, X, ACC, DOT, false>(m, P, x, y, variant, s, stop, part, count);
}

template <class V, class X, bool ACC>
static void spmv_typed(dsm_matrix m, const Payload &P, const X *x, X *y, int variant, hipStream_t s,
                       Workspace *scratch, const int *stop) {
    const i64 n = m->nrows;
    switch (P.fmt) {
    case DSM_CSR:
        csr_launch<V, X, ACC>(m, P, x, y, variant, s, stop);
        break;
    case DSM_COO:
        coo_launch<V, X>(m, P.coo_nnz, P.crow, P.ccol, (const V *)P.cval, x, y, ACC, s, scratch, stop);
        break;
    case DSM_DIA:
    case DSM_HDC:
        if (n > 0) sweep<V, X, ACC>(m, P, x, y, variant, s, stop);
        if (P.fmt == DSM_HDC && P.csr_nnz > 0) csr_launch<V, X, true>(m, P, x, y, 0, s, stop);
        break;
    case DSM_ELL:
    case DSM_HYB:
        if (n > 0) sweep<V, X, ACC>(m, P, x, y, variant, s, stop);
        if (P.fmt == DSM_HYB && P.coo_nnz > 0)
            coo_launch<V, X>(m, P.coo_nnz, P.crow, P.ccol, (const V *)P.cval, x, y, true, s, scratch, stop);
        break;
    default:
        fail(DSM_E_INVALID, "spmv: unknown format");
    }
    DSM_HIP(hipGetLastError());
}

void spmv(dsm_matrix m, const Payload &P, const void *x, void *y, int vdt, int variant, hipStream_t s,
          Workspace *scratch, const int *stop, bool acc) {
    DSM_CHECK(vdt == DSM_F64 || vdt == DSM_F32, DSM_E_UNSUPPORTED, "spmv: vectors must be F64 or F32");
    if (vdt == DSM_F64) {
        const double *xx = (const double *)x;
        double *yy = (double *)y;
        switch (P.vdt) {
        case DSM_F64: acc ? spmv_typed<double, double, true>(m, P, xx, yy, variant, s, scratch, stop) : spmv_typed<double, double, false>(m, P, xx, yy, variant, s, scratch, stop); break;
        case DSM_F32: acc ? spmv_typed<float, double, true>(m, P, xx, yy, variant, s, scratch, stop) : spmv_typed<float, double, false>(m, P, xx, yy, variant, s, scratch, stop); break;
        default: acc ? spmv_typed<bf16, double, true>(m, P, xx, yy, variant, s, scratch, stop) : spmv_typed<bf16, double, false>(m, P, xx, yy, variant, s, scratch, stop); break;
        }
    } else {
        const float *xx = (const float *)x;
        float *yy = (float *)y;
        switch (P.vdt) {
        case DSM_F64: acc ? spmv_typed<double, float, true>(m, P, xx, yy, variant, s, scratch, stop) : spmv_typed<double, float, false>(m, P, xx, yy, variant, s, scratch, stop); break;
        case DSM_F32: acc ? spmv_typed<float, float, true>(m, P, xx, yy, variant, s, scratch, stop) : spmv_typed<float, float, false>(m, P, xx, yy, variant, s, scratch, stop); break;
        default: acc ? spmv_typed<bf16, float, true>(m, P, xx, yy, variant, s, scratch, stop) : spmv_typed<bf16, float, false>(m, P, xx, yy, variant, s, scratch, stop); break;
        }
    }
}

template <class X>
static int spmv_dot_typed(dsm_matrix m, const Payload &P, const X *x, X *y, int variant, hipStream_t s,
                          double *part, long long *count, const int *stop) {
    if (P.fmt == DSM_CSR) {
        switch (P.vdt) {
        case DSM_F64: return (int)csr_launch<double, X, false, true>(m, P, x, y, variant, s, stop, part, count);
        case DSM_F32: return (int)csr_launch<float, X, false, true>(m, P, x, y, variant, s, stop, part, count);
        default: return (int)csr_launch<bf16, X, false, true>(m, P, x, y, variant, s, stop, part, count);
        }
    }
    switch (P.vdt) {
    case DSM_F64: sweep<double, X, false, true>(m, P, x, y, variant, s, stop, part, count); break;
    case DSM_F32: sweep<float, X, false, true>(m, P, x, y, variant, s, stop, part, count); break;
    default: sweep<bf16, X, false, true>(m, P, x, y, variant, s, stop, part, count); break;
    }
    DSM_HIP(hipGetLastError());
    return (int)sweep_groups(m->nrows, variant);
}

int spmv_dot(dsm_matrix m, const Payload &P, const void *x, void *y, int vdt, int variant, hipStream_t s,
             double *part, long long *count, const int *stop) {
    // HDC whose CSR part is empty and HYB whose COO part is empty are one
    // DIA or ELL sweep, which writes y alone and can carry the epilogue
    const bool one_sweep = P.fmt == DSM_DIA || P.fmt == DSM_ELL || (P.fmt == DSM_HDC && P.csr_nnz == 0) ||
                           (P.fmt == DSM_HYB && P.coo_nnz == 0);
    // CSR: when its workgroups fit the solvers' partial buffers (the
    // adaptive kernel runs a workgroup per row block: about nnz/1024 of them)
    const bool csr = P.fmt == DSM_CSR && csr_groups(m, P, variant) <= dot_partials_cap(m->nrows) &&
                     csr_groups(m, P, variant) > 0;
    if (!(one_sweep || csr) || m->nrows != m->ncols || m->nrows == 0) return 0;
    if (vdt == DSM_F64)
        return spmv_dot_typed<double>(m, P, (const double *)x, (double *)y, variant, s, part, count, stop);
    return spmv_dot_typed<float>(m, P, (const float *)x, (float *)y, variant, s, part, count, stop);
}

// ---------------------------------------------------------------- kernel-only timing
double spmv_kernel_us(dsm_matrix m, const void *x, void *y, int vdt, hipStream_t s) {
    LaunchTiming lt;
    DSM_HIP(hipEventCreate(&lt.start));
    if (hipEventCreate(&lt.stop) != hipSuccess) {
        (void)hipEventDestroy(lt.start);
        fail(DSM_E_DEVICE, "hipEventCreate failed");
    }
    struct Reset {
        LaunchTiming &lt;
        ~Reset() {
            t_launch_timing = nullptr;
            (void)hipEventDestroy(lt.start);
            (void)hipEventDestroy(lt.stop);
        }
    } reset{lt};
    t_launch_timing = &lt;
    spmv(m, m->P, x, y, vdt, m->variant, s);
    t_launch_timing = nullptr;
    if (!lt.started) return 0.0;  // nothing to launch (no rows)
    DSM_HIP(hipEventSynchronize(lt.stop));
    float ms = 0;
    DSM_HIP(hipEventElapsedTime(&ms, lt.start, lt.stop));
    return ms * 1000.0;
}

// ---------------------------------------------------------------- allocation-free entry
// The COO pass's per-tile partials for callers that cannot allocate: a
// static device array, one copy per device, of NOALLOC_SCRATCH_BYTES.  Host
// code never uses the array's name as an address: the address of each
// device's copy is taken with hipGetSymbolAddress once, with that device
// current, and kept in g_noalloc_ptr.  Nothing in it needs clearing: every
// tile writes its two partials before the fix-up pass reads them.
static __device__ __align__(256) unsigned char g_noalloc_scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

void noalloc_scratch_init(int device) {
    DSM_CHECK(device >= 0 && device < NOALLOC_MAX_DEVICES, DSM_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return;
    void *p = nullptr;
    DSM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(g_noalloc_scratch)));
    DSM_CHECK(p != nullptr, DSM_E_DEVICE, "no device address for the static scratch buffer");
    g_noalloc_ptr[device] = p;
}

void spmv_noalloc(dsm_matrix m, const void *x, void *y, int vdt, hipStream_t s) {
    const int dev = m->ctx->device;
    void *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        p = g_noalloc_ptr[dev];
    }
    DSM_CHECK(p != nullptr, DSM_E_INVALID, "static scratch not set up for this device");
    DSM_CHECK(vdt == DSM_F64 || vdt == DSM_F32, DSM_E_UNSUPPORTED, "spmv: vectors must be F64 or F32");
    const size_t need = spmv_scratch_bytes(m, m->P, vdt);
    DSM_CHECK(need <= NOALLOC_SCRATCH_BYTES, DSM_E_NOMEM,
              "allocation-free SpMV: the COO part needs " + std::to_string(need) +
                  " bytes of scratch, more than the static buffer's " + std::to_string(NOALLOC_SCRATCH_BYTES));
    Workspace w;
    w.p = p;
    w.bytes = NOALLOC_SCRATCH_BYTES;
    w.fixed = true;
    spmv(m, m->P, x, y, vdt, m->variant, s, &w, nullptr, false);
}

size_t spmv_scratch_bytes(const dsm_matrix_s *m, const Payload &P, int vec_dtype) {
    (void)m;
    if (!(P.fmt == DSM_COO || P.fmt == DSM_HYB) || P.coo_nnz == 0) return 0;
    const i64 ntiles = (P.coo_nnz + COO_TE - 1) / COO_TE;
    return dtype_size(vec_dtype) * (size_t)(2 * ntiles);
}

double spmv_bytes(const dsm_matrix_s *m, const Payload &P, int vec_dtype) {
    const double v = (double)dtype_size(P.vdt), i = 4.0, X = (double)dtype_size(vec_dtype);
    const double N = (double)m->nrows, NC = (double)m->ncols;
    const double xy = NC * X + N * X;
    switch (P.fmt) {
    case DSM_COO: return (double)P.coo_nnz * (v + 2 * i) + xy;
    case DSM_CSR: return (double)P.csr_nnz * (v + i) + (N + 1) * i + xy;
    case DSM_DIA: return (double)P.ndiag * N * v + (double)P.ndiag * i + xy;
    case DSM_ELL: return (double)P.K * N * (v + i) + xy;
    case DSM_HYB: return (double)P.K * N * (v + i) + (double)P.coo_nnz * (v + 2 * i) + xy;
    case DSM_HDC:
        return (double)P.ndiag * N * v + (double)P.ndiag * i + (double)P.csr_nnz * (v + i) + (N + 1) * i + xy;
    }
    return 0;
}

}  // namespace dsm
