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
// state only every few iterations (a one-thread kernel copies it to pinned
// host memory at the end of each chunk, and the next chunk is usually
// queued already, so the device does not wait for the host).
//
// Mixed precision (iterative refinement): the outer loop keeps x, the
// residual b - A x, its norm and the update x += d in FP64 (the residual
// SpMV accumulates the stored FP32/BF16 values in FP64); the inner CG solves
// A d = r/||r|| with FP32 vectors and FP32-accumulated SpMV, while its dot
// products are accumulated in FP64.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "cg_common.hpp"

namespace dsm {

// cont: the first direction continues the one p holds, p = r + pc p (IR
// with continued directions); otherwise p = r.
template <class X>
__global__ void __launch_bounds__(CGB) k_cg_init(i64 n, const X *b, const X *q, X *r, X *p, double *part,
                                                 bool cont, X pc) {
    __shared__ double lds[CGB / WAVE];
    double acc = 0;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x) {
        X ri = b[i] - q[i];
        r[i] = ri;
        p[i] = cont ? ri + pc * p[i] : ri;
        acc += (double)ri * (double)ri;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(CGB) k_cg_init_state(const double *part, int npart, CgState *st, double tol,
                                                       long long maxit) {
    __shared__ double lds[CGB / WAVE];
    double rho = reduce_partials(part, lds, npart);
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
    if (wg_done(&st->done)) return;
    double acc = 0;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x)
        acc += (double)p[i] * (double)q[i];
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc;
        if (blockIdx.x == 0) st->iters += 1;
    }
}

constexpr int VU = 4;  // loads per vector per lane per pass in the vector updates

// L consecutive elements of X in one load: a 16-byte vector for L > 1, the
// element itself for L = 1.
template <class X, int L>
struct Lanes {
    typedef X T __attribute__((ext_vector_type(L)));
    static __device__ __forceinline__ X get(const T &v, int e) { return v[e]; }
};
template <class X>
struct Lanes<X, 1> {
    typedef X T;
    static __device__ __forceinline__ X get(const T &v, int) { return v; }
};

template <class X, int L, bool NT>
__device__ __forceinline__ typename Lanes<X, L>::T ld_lanes(const X *p) {
    using T = typename Lanes<X, L>::T;
    if constexpr (NT) return __builtin_nontemporal_load((const T *)p);
    else return *(const T *)p;
}
template <class X, int L, bool NT>
__device__ __forceinline__ void st_lanes(X *p, typename Lanes<X, L>::T v) {
    using T = typename Lanes<X, L>::T;
    if constexpr (NT) __builtin_nontemporal_store(v, (T *)p);
    else *(T *)p = v;
}

// Where the L-element loads of this workgroup's slice end: slices start at
// multiples of blockDim.x (a multiple of L), so only the end of the vector
// can leave fewer than L elements, handled one by one by the workgroup that
// owns them.
template <int L>
__device__ __forceinline__ i64 lanes_hi(i64 n, i64 hi) {
    return L == 1 ? hi : min(hi, n / L * L);
}

// The vector updates load their first VU vectors of L elements per lane
// before they reduce the partials their scalar depends on (the loads do not
// need it), so the latency of the reduction and of the first stream overlap;
// every load of a pass is issued before any of its stores.  They must stay
// within 128 VGPRs, so that two 512-thread workgroups share a CU and the
// 512-workgroup grid runs in one round on 256 CUs (the offsets are written
// out per load: a 64-bit stride variable took the 16-byte-load kernels to
// 136 VGPRs and one workgroup per CU, slower than one element per load).
// The host takes
// L = 2 for FP64 when all vectors are 16-byte aligned (about 2% per
// iteration at HPCG 104^3 over one element per load), else L = 1.
// The per-lane sums run over a lane's elements in a different order for
// different L; each L is deterministic.
//
// NT: x and q are streamed (x is not read again until the next update, q
// not before the next SpMV rewrites it), so they need not displace the
// matrix lines the next SpMV may still find in the Infinity Cache.
//
// x is updated here and not in the p update, although that would save one
// read of p: the p update's workgroup 0 sets the done flag, and a workgroup
// of the same launch that starts after that store exits at once.  Skipping
// the p update is harmless then (p is dead); skipping a share of the last
// x += alpha p is not (seen when concurrent solves delayed workgroups).
template <class X, bool NT, int L>
__global__ void __launch_bounds__(CGB) k_cg_update_xr(i64 n, X *x, X *r, const X *p, const X *q,
                                                       const double *part_pq, int npq, double *part_rr,
                                                       CgState *st) {
    using LT = Lanes<X, L>;
    using V = typename LT::T;
    __shared__ double lds[CGB / WAVE];
    const i64 lo = slice_lo(n), hi = slice_hi(n), hv = lanes_hi<L>(n, hi);
    i64 base = lo + (i64)L * threadIdx.x;
    V xv[VU], pv[VU], rv[VU], qv[VU];
    auto load = [&]() {
#pragma unroll
        for (int u = 0; u < VU; u++) {
            const i64 i = base + (i64)u * L * blockDim.x;
            if (i < hv) {
                xv[u] = ld_lanes<X, L, NT>(x + i);
                pv[u] = ld_lanes<X, L, false>(p + i);
                rv[u] = ld_lanes<X, L, false>(r + i);
                qv[u] = ld_lanes<X, L, NT>(q + i);
            }
        }
    };
    load();
    const long long k = st->iters;
    const double rho_even = st->rho[0], rho_odd = st->rho[1];
    double pq;
    if (wg_done_sum(&st->done, part_pq, npq, lds, &pq)) return;
    const double rho = ((k - 1) & 1) ? rho_odd : rho_even;
    if (!(pq > 0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->done = 3;
        }
        return;
    }
    const X a = (X)(rho / pq);
    double acc = 0;
    while (base < hv) {
#pragma unroll
        for (int u = 0; u < VU; u++) {
            const i64 i = base + (i64)u * L * blockDim.x;
            if (i < hv) {
                st_lanes<X, L, NT>(x + i, xv[u] + a * pv[u]);
                const V ri = rv[u] - a * qv[u];
                st_lanes<X, L, false>(r + i, ri);
#pragma unroll
                for (int e = 0; e < L; e++) acc += (double)LT::get(ri, e) * (double)LT::get(ri, e);
            }
        }
        base += (i64)VU * L * blockDim.x;
        load();
    }
    if (L > 1 && lo < hi && hv < hi) {
        const i64 i = hv + threadIdx.x;
        if (i < hi) {
            x[i] = x[i] + a * p[i];
            const X ri = r[i] - a * q[i];
            r[i] = ri;
            acc += (double)ri * (double)ri;
        }
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = acc;
        if (blockIdx.x == 0) st->pq = pq;
    }
}

template <class X, bool NT, int L>
__global__ void __launch_bounds__(CGB) k_cg_update_p(i64 n, const X *r, X *p, const double *part_rr, int nrr,
                                                      CgState *st) {
    using V = typename Lanes<X, L>::T;
    __shared__ double lds[CGB / WAVE];
    const i64 lo = slice_lo(n), hi = slice_hi(n), hv = lanes_hi<L>(n, hi);
    i64 base = lo + (i64)L * threadIdx.x;
    V rv[VU], pv[VU];
    auto load = [&]() {
#pragma unroll
        for (int u = 0; u < VU; u++) {
            const i64 i = base + (i64)u * L * blockDim.x;
            if (i < hv) {
                rv[u] = ld_lanes<X, L, NT>(r + i);
                pv[u] = ld_lanes<X, L, false>(p + i);
            }
        }
    };
    load();
    const long long k = st->iters;
    const double rho_even = st->rho[0], rho_odd = st->rho[1];
    const double tol = st->tol, nr0 = st->nr0;
    const long long maxit = st->maxit;
    double rho1;
    if (wg_done_sum(&st->done, part_rr, nrr, lds, &rho1)) return;
    const double rho = ((k - 1) & 1) ? rho_odd : rho_even;
    const double nr = sqrt(rho1);
    int done = 0;
    if (!isfinite(rho1)) done = 3;
    else if (nr <= tol * nr0) done = 1;
    else if (k >= maxit) done = 2;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->relres = nr0 > 0 ? nr / nr0 : 0.0;
        st->rho[k & 1] = rho1;
        if (done) st->done = done;
    }
    if (done) return;
    const X beta = (X)(rho1 / rho);
    while (base < hv) {
#pragma unroll
        for (int u = 0; u < VU; u++) {
            const i64 i = base + (i64)u * L * blockDim.x;
            if (i < hv) st_lanes<X, L, false>(p + i, rv[u] + beta * pv[u]);
        }
        base += (i64)VU * L * blockDim.x;
        load();
    }
    if (L > 1 && lo < hi && hv < hi) {
        const i64 i = hv + threadIdx.x;
        if (i < hi) p[i] = r[i] + beta * p[i];
    }
}

// ---------------------------------------------------------------- IR helpers
// r = b - q (FP64) and partial sums of r.r and b.b
__global__ void __launch_bounds__(CGB) k_residual(i64 n, const double *b, const double *q, double *r, double *part_rr,
                                                  double *part_bb) {
    __shared__ double lds[CGB / WAVE];
    double a = 0, c = 0;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x) {
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
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x) {
        r32[i] = (float)(r[i] * inv);
        d32[i] = 0.0f;
    }
}

// x += ||r|| * d32 (FP64)
__global__ void __launch_bounds__(CGB) k_apply_update(i64 n, double *x, const float *d32, const double *nrm) {
    const double s = nrm[0];
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x)
        x[i] = x[i] + s * (double)d32[i];
}


// ---------------------------------------------------------------- fused iteration (DIA / ELL)
// Two kernels per iteration instead of four.  Iteration k (parity ph = k & 1):
//   F1: rho_{k-1} = sum of the r.r partials of the previous update; stop if
//       converged / out of iterations; beta = rho_{k-1} / rho_{k-2} (0 at
//       k = 1); every workgroup then forms p_k = r + beta p_{k-1} on the fly
//       for each x entry it gathers and for its own rows (stored to the other
//       p buffer), computes q = A p_k and partials of p_k . q.
//   F2: alpha = rho_{k-1} / (p_k . q); x += alpha p_k; r -= alpha q; partials
//       of r.r.
// p_k is formed with one fused multiply-add, so the value gathered by any
// workgroup equals the stored one bit for bit.  rho_{k-1} goes to slot
// (k-1) & 1 (written by workgroup 0 of F1, read by F2), rho_{k-2} is read
// from slot k & 1; the completed-iteration count is written only by F2.
template <class X>
__device__ __forceinline__ X p_next(X r, X pold, X beta, bool first) {
    return first ? r : fma(beta, pold, r);
}

template <class V, class X, int R, bool XCD, bool ELL>
__global__ void __launch_bounds__(256) k_cgf_spmv(i64 n, i64 nd, const i32 *__restrict__ offs,
                                                  const i32 *__restrict__ ecol, const V *__restrict__ vals, i64 pitch,
                                                  const X *__restrict__ r, const X *__restrict__ pold,
                                                  X *__restrict__ pnew, X *__restrict__ q,
                                                  const double *__restrict__ part_rr, double *__restrict__ part_pq,
                                                  CgState *st, int ph) {
    __shared__ double lds[256 / WAVE];
    if (wg_done(&st->done)) return;
    const double rho1 = reduce_partials(part_rr, lds);
    const long long done_iters = st->iters;
    const bool first = done_iters == 0;
    if (!first) {
        int done = 0;
        const double nr = sqrt(rho1);
        if (!isfinite(rho1)) done = 3;
        else if (nr <= st->tol * st->nr0) done = 1;
        else if (done_iters >= st->maxit) done = 2;
        if (done) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->relres = st->nr0 > 0 ? nr / st->nr0 : 0.0;
                st->done = done;
            }
            return;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->rho[ph ^ 1] = rho1;
    const X beta = first ? (X)0 : (X)(rho1 / st->rho[ph]);
    const u32 b = XCD ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const i64 i0 = (i64)b * 256 * R + threadIdx.x;
    X s[R];
#pragma unroll
    for (int t = 0; t < R; t++) s[t] = 0;
    // Batches of KU diagonals (ELL: slots): every value, r and p load of a
    // batch is issued before its products; operands that must vanish come
    // from the zero word (ELL columns past K from the sentinel word), and a
    // DIA zero slot drops its operand after the loads, as in the SpMV sweep.
    constexpr int KU = R >= 8 ? 1 : 8 / R;
    for (i64 k0 = 0; k0 < nd; k0 += KU) {
        V v[KU][R];
        X rj[KU][R], pj[KU][R];
#pragma unroll
        for (int u = 0; u < KU; u++) {
            const i64 k = k0 + u;
            const bool kin = k < nd;
#pragma unroll
            for (int t = 0; t < R; t++) {
                const i64 i = i0 + (i64)t * 256;
                const bool live = kin && i < n;
                if constexpr (!ELL) {
                    // offs is zero-padded to a multiple of 16 entries
                    const i64 j = i + offs[k];
                    const bool ok = live && j >= 0 && j < n;
                    v[u][t] = *(live ? vals + k * pitch + i : zero_ptr<V>());
                    rj[u][t] = *(ok ? r + j : zero_ptr<X>());
                    pj[u][t] = *(ok ? pold + j : zero_ptr<X>());
                } else {
                    const i32 c = *(live ? ecol + k * pitch + i : sentinel_ptr<i32>());
                    v[u][t] = *(live ? vals + k * pitch + i : zero_ptr<V>());
                    rj[u][t] = *(c >= 0 ? r + c : zero_ptr<X>());
                    pj[u][t] = *(c >= 0 ? pold + c : zero_ptr<X>());
                }
            }
        }
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int t = 0; t < R; t++) {
                asm volatile("" : "+v"(rj[u][t]));
                asm volatile("" : "+v"(pj[u][t]));
            }
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int t = 0; t < R; t++) {
                const X wv = widen<X>(v[u][t]);
                const X pv = p_next<X>(rj[u][t], pj[u][t], beta, first);
                s[t] += wv * (ELL || wv != (X)0 ? pv : (X)0);
            }
    }
    double acc = 0;
#pragma unroll
    for (int t = 0; t < R; t++) {
        const i64 i = i0 + (i64)t * 256;
        if (i < n) {
            const X pi = p_next<X>(r[i], pold[i], beta, first);
            pnew[i] = pi;
            q[i] = s[t];
            acc += (double)pi * (double)s[t];
        }
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part_pq[blockIdx.x] = acc;
}

template <class X>
__global__ void __launch_bounds__(CGB) k_cgf_update(i64 n, X *x, X *r, const X *p, const X *q,
                                                     const double *part_pq, int npq, double *part_rr, CgState *st,
                                                     int ph) {
    __shared__ double lds[CGB / WAVE];
    if (wg_done(&st->done)) return;
    const double pq = reduce_partials(part_pq, lds, npq);
    const double rho = st->rho[ph ^ 1];
    if (!(pq > 0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->iters += 1;
            st->done = 3;
        }
        return;
    }
    const X a = (X)(rho / pq);
    double acc = 0;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x) {
        x[i] = x[i] + a * p[i];
        const X ri = r[i] - a * q[i];
        r[i] = ri;
        acc += (double)ri * (double)ri;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = acc;
        if (blockIdx.x == 0) {
            st->pq = pq;
            st->iters += 1;
        }
    }
}

// Whether the two-kernel iteration is used (square DIA/ELL payload, asked
// for with DSM_CG_FUSED=1).  It saves a launch and the p update's pass over
// r and p, but gathers two vectors per stored entry instead of one; on
// MI355X the three-kernel loop (SpMV with p.q, x/r update, p update) is
// faster at the HPCG sizes, so it is the default.
static bool fused_ok(const dsm_matrix_s *m) {
    const char *e = getenv("DSM_CG_FUSED");
    if (!(e && e[0] == '1')) return false;
    return m->nrows == m->ncols && (m->P.fmt == DSM_DIA || m->P.fmt == DSM_ELL);
}

// Partials F1 writes (one per workgroup).
static int fused_groups(const dsm_matrix_s *m) {
    const int lr = (m->variant >> 1) & 3;
    const int R = lr == 0 ? 1 : (lr == 1 ? 2 : 4);
    return (int)grid_for(m->nrows, 256 * R);
}

template <class V, class X, int R, bool XCD>
static void cgf_launch(dsm_matrix m, const X *r, const X *pold, X *pnew, X *q, double *part_rr, double *part_pq,
                       CgState *st, int ph, hipStream_t s) {
    const Payload &P = m->P;
    const i64 n = m->nrows;
    const unsigned g = grid_for(n, 256 * R);
    if (P.fmt == DSM_DIA)
        hipLaunchKernelGGL((k_cgf_spmv<V, X, R, XCD, false>), dim3(g), dim3(256), 0, s, n, P.ndiag, P.offs,
                           (const i32 *)nullptr, (const V *)P.dval, P.pitch, r, pold, pnew, q, part_rr, part_pq, st,
                           ph);
    else
        hipLaunchKernelGGL((k_cgf_spmv<V, X, R, XCD, true>), dim3(g), dim3(256), 0, s, n, P.K,
                           (const i32 *)nullptr, P.ecol, (const V *)P.evl, P.pitch, r, pold, pnew, q, part_rr,
                           part_pq, st, ph);
}

template <class V, class X, bool XCD>
static void cgf_r(dsm_matrix m, int lr, const X *r, const X *pold, X *pnew, X *q, double *prr, double *ppq,
                  CgState *st, int ph, hipStream_t s) {
    if (lr == 0) cgf_launch<V, X, 1, XCD>(m, r, pold, pnew, q, prr, ppq, st, ph, s);
    else if (lr == 1) cgf_launch<V, X, 2, XCD>(m, r, pold, pnew, q, prr, ppq, st, ph, s);
    else cgf_launch<V, X, 4, XCD>(m, r, pold, pnew, q, prr, ppq, st, ph, s);
}

template <class V, class X>
static void cgf_dispatch(dsm_matrix m, const X *r, const X *pold, X *pnew, X *q, double *prr, double *ppq,
                         CgState *st, int ph, hipStream_t s) {
    // the fused kernel takes the tile order and rows per thread from the
    // SpMV variant (bits 0-2); it has no paired-row form
    const int v = m->variant;
    const bool xcd = !(v & 1);
    const int lr = (v >> 1) & 3;
    if (xcd) cgf_r<V, X, true>(m, lr, r, pold, pnew, q, prr, ppq, st, ph, s);
    else cgf_r<V, X, false>(m, lr, r, pold, pnew, q, prr, ppq, st, ph, s);
}

// One fused iteration with parity ph; p buffers alternate: p[ph] is written.
template <class X>
static void enqueue_fused(dsm_matrix m, X *x, X *r, X *pbuf[2], X *q, double *part_pq, double *part_rr,
                          CgState *st, int ph, hipStream_t s) {
    const i64 n = m->nrows;
    X *pnew = pbuf[ph], *pold = pbuf[ph ^ 1];
    switch (m->P.vdt) {
    case DSM_F64: cgf_dispatch<double, X>(m, r, pold, pnew, q, part_rr, part_pq, st, ph, s); break;
    case DSM_F32: cgf_dispatch<float, X>(m, r, pold, pnew, q, part_rr, part_pq, st, ph, s); break;
    default: cgf_dispatch<bf16, X>(m, r, pold, pnew, q, part_rr, part_pq, st, ph, s); break;
    }
    hipLaunchKernelGGL((k_cgf_update<X>), dim3(CGG), dim3(CGB), 0, s, n, x, r, pnew, q, part_pq, fused_groups(m),
                       part_rr, st, ph);
}


// ---------------------------------------------------------------- Jacobi PCG
// M = diag(A).  Same loop shape as the plain solver with z = M^-1 r formed on
// the fly: rho = r.z drives alpha and beta, the stopping test uses ||r||.
__global__ void k_invert_diag(i64 n, double *d, int *zero) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = d[i];
    if (v == 0.0 || !isfinite(v)) atomicOr(zero, 1);
    d[i] = v != 0.0 ? 1.0 / v : 0.0;
}

__global__ void __launch_bounds__(CGB) k_pcg_init(i64 n, const double *b, const double *q, const double *dinv,
                                                  double *r, double *p, double *part_rz, double *part_rr) {
    __shared__ double lds[CGB / WAVE];
    double rz = 0, rr = 0;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x) {
        const double ri = b[i] - q[i];
        const double zi = ri * dinv[i];
        r[i] = ri;
        p[i] = zi;
        rz += ri * zi;
        rr += ri * ri;
    }
    rz = block_sum(rz, lds);
    rr = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        part_rz[blockIdx.x] = rz;
        part_rr[blockIdx.x] = rr;
    }
}

__global__ void __launch_bounds__(CGB) k_pcg_init_state(const double *part_rz, const double *part_rr, int count,
                                                        CgState *st, double tol, long long maxit) {
    __shared__ double lds[CGB / WAVE];
    const double rz = reduce_partials(part_rz, lds, count);
    const double rr = reduce_partials(part_rr, lds, count);
    if (threadIdx.x == 0) {
        st->rho[0] = rz;
        st->rho[1] = 0;
        st->nr0 = sqrt(rr);
        st->pq = 0;
        st->relres = rr > 0 ? 1.0 : 0.0;
        st->tol = tol;
        st->iters = 0;
        st->maxit = maxit;
        st->done = rr == 0 ? 1 : ((!isfinite(rr) || !isfinite(rz)) ? 3 : (maxit <= 0 ? 2 : 0));
    }
}

__global__ void __launch_bounds__(CGB) k_pcg_update_xr(i64 n, double *x, double *r, const double *p, const double *q,
                                                       const double *dinv, const double *part_pq, int npq,
                                                       double *part_rz, double *part_rr, CgState *st) {
    __shared__ double lds[CGB / WAVE];
    if (wg_done(&st->done)) return;
    const double pq = reduce_partials(part_pq, lds, npq);
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
    double rz = 0, rr = 0;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x) {
        x[i] = x[i] + alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        rz += ri * (ri * dinv[i]);
        rr += ri * ri;
    }
    rz = block_sum(rz, lds);
    rr = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        part_rz[blockIdx.x] = rz;
        part_rr[blockIdx.x] = rr;
        if (blockIdx.x == 0) st->pq = pq;
    }
}

__global__ void __launch_bounds__(CGB) k_pcg_update_p(i64 n, const double *r, double *p, const double *dinv,
                                                      const double *part_rz, const double *part_rr, int count,
                                                      CgState *st) {
    __shared__ double lds[CGB / WAVE];
    if (wg_done(&st->done)) return;
    const double rho1 = reduce_partials(part_rz, lds, count);
    const double nr = sqrt(reduce_partials(part_rr, lds, count));
    const long long k = st->iters;
    const double rho = st->rho[(k - 1) & 1];
    int done = 0;
    if (!isfinite(nr) || !isfinite(rho1)) done = 3;
    else if (nr <= st->tol * st->nr0) done = 1;
    else if (k >= st->maxit) done = 2;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->relres = st->nr0 > 0 ? nr / st->nr0 : 0.0;
        st->rho[k & 1] = rho1;
        if (done) st->done = done;
    }
    if (done) return;
    const double beta = rho1 / rho;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x)
        p[i] = r[i] * dinv[i] + beta * p[i];
}

// ================================================================ host side
struct CgBuffers {
    // FP64 part (p2: second p buffer of the fused iteration; dinv: inverse
    // diagonal of the Jacobi preconditioner; xw: the iterate of the
    // graph-replayed FP64 loop)
    double *r = nullptr, *p = nullptr, *q = nullptr, *p2 = nullptr, *dinv = nullptr, *part_c = nullptr;
    double *xw = nullptr;
    double *part_a = nullptr, *part_b = nullptr, *norms = nullptr;
    CgState *st = nullptr, *st2 = nullptr;
    // FP32 inner part (IR)
    float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr, *ri32 = nullptr, *p32b = nullptr;
};

// Partials per workgroup: the vector kernels use CGG, the fused SpMV one per
// 256-row tile.
static size_t partial_slots(i64 n) { return (size_t)dot_partials_cap(n); }
static_assert(CGG <= 512, "the vector kernels' partials must fit dot_partials_cap");

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace bytes a solve of this matrix needs (also used for admission).
size_t cg_workspace_bytes(i64 n, bool ir) {
    const size_t nn = (size_t)std::max<i64>(n, 1);
    size_t bytes = 6 * round256(nn * 8) + 3 * round256(partial_slots(n) * 8) + 8 * 256;
    if (ir) bytes += 6 * round256(nn * 4);
    return bytes;
}

static CgBuffers cg_buffers(dsm_matrix m, bool ir, Workspace &cgws, hipStream_t s) {
    const size_t n = (size_t)std::max<i64>(m->nrows, 1);
    char *base = (char *)ws_get(m->ctx, cgws, cg_workspace_bytes(m->nrows, ir), s);
    CgBuffers B;
    auto take = [&](size_t sz) {
        char *p = base;
        base += round256(sz);
        return (void *)p;
    };
    B.r = (double *)take(n * 8);
    B.p = (double *)take(n * 8);
    B.q = (double *)take(n * 8);
    B.p2 = (double *)take(n * 8);
    B.part_a = (double *)take(partial_slots(m->nrows) * 8);
    B.part_b = (double *)take(partial_slots(m->nrows) * 8);
    B.part_c = (double *)take(partial_slots(m->nrows) * 8);
    B.dinv = (double *)take(n * 8);
    B.xw = (double *)take(n * 8);
    B.norms = (double *)take(64);
    B.st = (CgState *)take(sizeof(CgState));
    B.st2 = (CgState *)take(sizeof(CgState));
    if (ir) {
        B.r32 = (float *)take(n * 4);
        B.p32 = (float *)take(n * 4);
        B.q32 = (float *)take(n * 4);
        B.d32 = (float *)take(n * 4);
        B.ri32 = (float *)take(n * 4);
        B.p32b = (float *)take(n * 4);
    }
    return B;
}

// Workgroups of the vector kernels (= their partials): one per CGB
// elements up to CGG.  A small system gets a small grid: the kernels stay
// short and every consumer reduces only that many partials (in the serving
// mix, full 512-workgroup grids on systems of 10^4-10^5 rows made the two
// vector kernels 40% of all kernel time).
static unsigned vec_grid(i64 n) { return (unsigned)std::max<i64>(1, std::min<i64>(CGG, (n + CGB - 1) / CGB)); }

// One CG iteration: SpMV with p.q, x/r update, p update (DIA/ELL sweeps and
// CSR launches of at most dot_partials_cap(n) workgroups write the p.q
// partials themselves; the rest take a separate dot kernel).  Every kernel checks the state's done flag first, so iterations
// enqueued past convergence cost only their launches.
template <class X>
static void enqueue_iteration(dsm_matrix m, X *x, X *r, X *p, X *q, double *part_a, double *part_b, CgState *st,
                              int vdt, hipStream_t s, Workspace &spws) {
    const i64 n = m->nrows;
    const unsigned G = vec_grid(n);
    int npq = spmv_dot(m, m->P, p, q, vdt, m->variant, s, part_a, &st->iters, &st->done);
    if (npq == 0) {
        spmv(m, m->P, p, q, vdt, m->variant, s, &spws, &st->done);
        hipLaunchKernelGGL((k_cg_dot_pq<X>), dim3(G), dim3(CGB), 0, s, n, p, q, part_a, st);
        npq = (int)G;
    }
    // FP64 vectors are streamed past the caches where they are not reused
    // soon (3-5% per iteration at HPCG 104^3); the FP32 inner loop of IR
    // keeps its vectors cached (its matrix is smaller, the vectors matter more)
    constexpr bool NT = std::is_same<X, double>::value;
    // FP64: two elements per 16-byte load where every vector allows it; the
    // FP32 loop keeps one element per load (two or four per load measured
    // about 1% slower there)
    constexpr int L = std::is_same<X, double>::value ? 2 : 1;
    if (L > 1 && ((uintptr_t)x | (uintptr_t)r | (uintptr_t)p | (uintptr_t)q) % 16 == 0) {
        hipLaunchKernelGGL((k_cg_update_xr<X, NT, L>), dim3(G), dim3(CGB), 0, s, n, x, r, p, q, part_a, npq, part_b,
                           st);
        hipLaunchKernelGGL((k_cg_update_p<X, NT, L>), dim3(G), dim3(CGB), 0, s, n, r, p, part_b, (int)G, st);
    } else {
        hipLaunchKernelGGL((k_cg_update_xr<X, NT, 1>), dim3(G), dim3(CGB), 0, s, n, x, r, p, q, part_a, npq, part_b,
                           st);
        hipLaunchKernelGGL((k_cg_update_p<X, NT, 1>), dim3(G), dim3(CGB), 0, s, n, r, p, part_b, (int)G, st);
    }
}

// Copies the state into slot (seq & 1) of a two-slot host buffer, where seq
// counts the copies since the last k_state_seq_reset, and stores seq in the
// copy's pad field.  The host buffer is coherent pinned memory, so the
// stores go to host memory directly.
__global__ void k_state_out(CgState *st, CgState *host) {
    if (threadIdx.x != 0) return;
    const int seq = st->pad;
    CgState v = *st;
    v.pad = seq;
    host[seq & 1] = v;
    __threadfence_system();
    st->pad = seq + 1;
}

__global__ void k_state_seq_reset(CgState *st) {
    if (threadIdx.x == 0) st->pad = 0;
}

void enqueue_state_out(CgState *st, CgState *host_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_state_out, dim3(1), dim3(WAVE), 0, s, st, host_dev);
}

void enqueue_state_seq_reset(CgState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_state_seq_reset, dim3(1), dim3(WAVE), 0, s, st);
}

bool cg_graphs_enabled() {
    const char *e = getenv("DSM_CG_GRAPH");
    return !(e && e[0] == '0');
}

// Runs CG on (b, x) with vectors of type X.  Uses buffers r, p, q, part_*.
// The loop is replayed in chunks of `check_every` iterations from a HIP
// graph captured once per (matrix payload, buffers, chunk) and kept in
// `cgws`; the host reads the device state back once per chunk.  Returns the
// final state.
template <class X>
static CgState run_cg(dsm_matrix m, const X *b, X *x, X *r, X *p, X *q, X *p2, double *part_a, double *part_b,
                      CgState *st, int vdt, double tol, long long maxit, int check_every, hipStream_t s,
                      Workspace &spws, Workspace &cgws, bool use_graph, double pcont = 0) {
    const i64 n = m->nrows;
    const bool fused = fused_ok(m);
    if (fused) check_every += check_every & 1;  // even chunks keep the p-buffer parity
    X *pbuf[2] = {p, p2};
    // fused: init leaves the r.r partials where the first F1 reads them
    double *init_part = fused ? part_b : part_a;
    // the fused loop's first sweep reduces CGG partials of the init
    const unsigned G = fused ? (unsigned)CGG : vec_grid(n);
    spmv(m, m->P, x, q, vdt, m->variant, s, &spws);
    // a continued direction needs the p of the previous solve in p (the
    // fused loop alternates two p buffers, so it always starts afresh)
    const bool cont = pcont != 0 && !fused;
    hipLaunchKernelGGL((k_cg_init<X>), dim3(G), dim3(CGB), 0, s, n, b, q, r, p, init_part, cont, (X)pcont);
    hipLaunchKernelGGL(k_cg_init_state, dim3(1), dim3(CGB), 0, s, init_part, (int)G, st, tol, maxit);
    DSM_HIP(hipGetLastError());
    // iteration j of a chunk (0-based) has parity (j + 1) & 1
    auto enqueue = [&](int j, hipStream_t ss) {
        if (fused) enqueue_fused<X>(m, x, r, pbuf, q, part_a, part_b, st, (j + 1) & 1, ss);
        else enqueue_iteration<X>(m, x, r, p, q, part_a, part_b, st, vdt, ss, spws);
    };
    // the fused loop detects convergence at the start of the next iteration
    const long long cap = maxit + (fused ? 1 : 0);
    std::string key;
    if (use_graph) {
        const Payload &P = m->P;
        char buf[512];
        snprintf(buf, sizeof buf, "cg|%p|%d|%d|%d|%lld|%lld|%lld|%lld|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%d|%d|%p|%lld|%d|%p",
                 (void *)m, P.fmt, P.vdt, m->variant, (long long)P.ndiag, (long long)P.K, (long long)P.csr_nnz,
                 (long long)P.coo_nnz, (void *)P.rp, (void *)P.dval, (void *)P.evl, (void *)P.cval, (void *)x,
                 (void *)r, (void *)p, (void *)q, (void *)p2, (void *)part_a, (void *)part_b, vdt, check_every,
                 spws.p, (long long)n, (int)fused, (void *)st);
        key = buf;
    }
    return run_chunks(cgws, key, use_graph, check_every, cap, st, s, enqueue);
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

// Jacobi-preconditioned CG (z = D^-1 r formed on the fly), with the plain
// loop's execution: the SpMV writes the p.q partials where its format can,
// and the iterations are replayed in chunks from a captured graph.
static CgState run_pcg(dsm_matrix m, const double *b, double *x, CgBuffers &B, double tol, long long maxit,
                       int every, hipStream_t s, Workspace &spws, Workspace &cgws, bool use_graph) {
    const i64 n = m->nrows;
    diagonal_op(m, B.dinv, 0, s);
    int *zero = (int *)B.norms;
    DSM_HIP(hipMemsetAsync(zero, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_invert_diag, dim3(grid_for(n, 256)), dim3(256), 0, s, n, B.dinv, zero);
    int hz = 0;
    DSM_HIP(hipMemcpyAsync(&hz, zero, sizeof(int), hipMemcpyDeviceToHost, s));
    DSM_HIP(hipStreamSynchronize(s));
    DSM_CHECK(hz == 0, DSM_E_INVALID, "Jacobi preconditioner needs a non-zero finite diagonal");
    const unsigned G = vec_grid(n);
    spmv(m, m->P, x, B.q, DSM_F64, m->variant, s, &spws);
    hipLaunchKernelGGL(k_pcg_init, dim3(G), dim3(CGB), 0, s, n, b, B.q, B.dinv, B.r, B.p, B.part_b, B.part_c);
    hipLaunchKernelGGL(k_pcg_init_state, dim3(1), dim3(CGB), 0, s, B.part_b, B.part_c, (int)G, B.st, tol, maxit);
    DSM_HIP(hipGetLastError());
    auto enqueue = [&](int, hipStream_t ss) {
        int npq = spmv_dot(m, m->P, B.p, B.q, DSM_F64, m->variant, ss, B.part_a, &B.st->iters, &B.st->done);
        if (npq == 0) {
            spmv(m, m->P, B.p, B.q, DSM_F64, m->variant, ss, &spws, &B.st->done);
            hipLaunchKernelGGL((k_cg_dot_pq<double>), dim3(G), dim3(CGB), 0, ss, n, B.p, B.q, B.part_a, B.st);
            npq = (int)G;
        }
        hipLaunchKernelGGL(k_pcg_update_xr, dim3(G), dim3(CGB), 0, ss, n, x, B.r, B.p, B.q, B.dinv, B.part_a, npq,
                           B.part_b, B.part_c, B.st);
        hipLaunchKernelGGL(k_pcg_update_p, dim3(G), dim3(CGB), 0, ss, n, B.r, B.p, B.dinv, B.part_b, B.part_c,
                           (int)G, B.st);
        DSM_HIP(hipGetLastError());
    };
    std::string key;
    if (use_graph) {
        const Payload &P = m->P;
        char buf[512];
        snprintf(buf, sizeof buf, "pcgj|%p|%d|%d|%d|%lld|%lld|%lld|%lld|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%d|%p|%lld",
                 (void *)m, P.fmt, P.vdt, m->variant, (long long)P.ndiag, (long long)P.K, (long long)P.csr_nnz,
                 (long long)P.coo_nnz, (void *)P.rp, (void *)P.dval, (void *)P.evl, (void *)P.cval, (void *)x,
                 (void *)B.r, (void *)B.p, (void *)B.q, (void *)B.dinv, (void *)B.part_a, (void *)B.part_b,
                 (void *)B.part_c, (void *)B.st, every, spws.p, (long long)n);
        key = buf;
    }
    return run_chunks(cgws, key, use_graph, every, maxit, B.st, s, enqueue);
}

static int default_check_every(i64 n) { return n < 100000 ? 32 : 8; }

void cg_solve_ws(dsm_matrix m, const double *b, double *x, const dsm_cg_opts &o, dsm_cg_result *res, hipStream_t s,
                 Workspace &cgws, Workspace &spws, bool use_graph) {
    DSM_CHECK(m->nrows == m->ncols, DSM_E_UNSUPPORTED, "CG needs a square matrix");
    const i64 n = m->nrows;
    long long maxit = o.maxit > 0 ? o.maxit : std::min<long long>(10 * std::max<i64>(n, 1), 20000);
    int every = o.check_every > 0 ? o.check_every : default_check_every(n);
    dsm_cg_result R{};
    const bool ir = o.mode == DSM_CG_IR || o.mode == DSM_CG_IR_CONT;
    DSM_CHECK(o.mode == DSM_CG_F64 || ir || o.mode == DSM_CG_JACOBI, DSM_E_INVALID, "unknown CG mode");
    DSM_CHECK(!ir || m->P.vdt != DSM_F64, DSM_E_UNSUPPORTED,
              "iterative refinement needs F32 or BF16 matrix values (convert with value_dtype)");
    CgBuffers B = cg_buffers(m, ir, cgws, s);
    // the SpMV scratch is sized before anything is enqueued (no allocation
    // while an iteration chunk is captured)
    if (const size_t sb = spmv_scratch_bytes(m, m->P, DSM_F64)) ws_get(m->ctx, spws, sb, s);
    if (n == 0) {
        R.status = DSM_OK;
        *res = R;
        return;
    }
    if (o.mode == DSM_CG_JACOBI) {
        // replayed on a workspace copy of x, as the plain loop below
        const bool graphed = use_graph && cg_graphs_enabled();
        double *xi = graphed ? B.xw : x;
        if (graphed) DSM_HIP(hipMemcpyAsync(xi, x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
        CgState h = run_pcg(m, b, xi, B, o.tol, maxit, every, s, spws, cgws, graphed);
        if (graphed) DSM_HIP(hipMemcpyAsync(x, xi, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
        R.iters = h.iters;
        R.relres = h.relres;
        R.status = h.done == 1 ? DSM_OK : h.done == 3 ? DSM_E_BREAKDOWN : DSM_E_NOT_CONVERGED;
        R.relres_true = true_relres(m, b, x, B, s, spws);
        *res = R;
        return;
    }
    if (!ir) {
        // The graph-replayed loop iterates on a workspace copy of x, copied
        // back at the end: the captured graph then holds only workspace
        // buffers and stays valid from solve to solve, whatever x the caller
        // passes (with the caller's x in it, a new x meant a new capture).
        const bool graphed = use_graph && cg_graphs_enabled();
        double *xi = graphed ? B.xw : x;
        if (graphed) DSM_HIP(hipMemcpyAsync(xi, x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
        CgState h = run_cg<double>(m, b, xi, B.r, B.p, B.q, B.p2, B.part_a, B.part_b, B.st, DSM_F64, o.tol, maxit,
                                   every, s, spws, cgws, use_graph);
        if (graphed) DSM_HIP(hipMemcpyAsync(x, xi, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
        R.iters = h.iters;
        R.relres = h.relres;
        R.status = h.done == 1 ? DSM_OK : h.done == 3 ? DSM_E_BREAKDOWN : DSM_E_NOT_CONVERGED;
        R.relres_true = true_relres(m, b, x, B, s, spws);
        *res = R;
        return;
    }
    // iterative refinement
    // Default inner tolerances, measured at 128^3 with BF16 values.
    // Restarted inner solves: 1e-5 (HPCG 301 inner iterations against 345
    // at 1e-4 and 389 at 1e-2; ANISO7 869 / 875 / 887).  Continued
    // directions: 1e-2 (HPCG 264, ANISO7 805, against 797 for FP64 CG); a
    // larger reduction per step lets the FP64 residual drift from the
    // recursive one, and the continuation then falls back to a restart.
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : (o.mode == DSM_CG_IR_CONT ? 1e-2 : 1e-5);
    const int max_outer = o.max_outer > 0 ? o.max_outer : 50;
    long long inner_total = 0;
    int status = DSM_E_NOT_CONVERGED;
    double relres = 1.0;
    // continued directions: the last inner solve's state and the outer
    // relative residual its right-hand side was scaled by
    CgState last{};
    bool have_last = false;
    double relres_last = 0;
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
        // the inner solve need not reduce the residual further than the
        // outer tolerance asks (with a factor 2 of margin): the last outer
        // step usually needs far less than inner_tol
        const double tau = std::min(0.5, std::max(inner_tol, 0.5 * o.tol / relres));
        // Continued direction.  The previous inner solve (right-hand side
        // r_k/||r_k||) stopped after iteration j with p_j in p32 and
        // rho_{j-1} = r_{j-1}.r_{j-1}; its next direction would have been
        // r_j + (rho_j / rho_{j-1}) p_j.  With r_j replaced by the FP64
        // residual, r_{k+1}/||r_k|| = rhat/s (rhat = r_{k+1}/||r_{k+1}||,
        // s = ||r_k||/||r_{k+1}||, rho_j = 1/s^2), that direction scaled by s
        // into the new right-hand side's units is rhat + p_j/(s rho_{j-1}).
        // The continuation holds only while the FP64 residual still is the
        // recursive one (rounding has not taken over): 1/s within a factor 2
        // of sqrt(rho_j); otherwise the inner solve starts afresh (with a
        // tight inner tolerance the continued direction cost ANISO7 128^3
        // 4818 inner iterations instead of 869).
        double pc = 0;
        if (o.mode == DSM_CG_IR_CONT && have_last && last.done != 3 && last.iters >= 1) {
            const double rho_prev = last.rho[(last.iters - 1) & 1];
            const double rho_last = last.rho[last.iters & 1];
            const double sc = relres_last / relres;
            const double drift = 1.0 / (sc * std::sqrt(rho_last));
            const double c = 1.0 / (sc * rho_prev);
            if (std::isfinite(c) && rho_prev > 0 && rho_last > 0 && sc > 0 && drift <= 2.0 && drift >= 0.5) pc = c;
        }
        CgState h = run_cg<float>(m, B.r32, B.d32, B.ri32, B.p32, B.q32, B.p32b, B.part_a, B.part_b, B.st2, DSM_F32,
                                  tau, std::max<long long>(1, maxit - inner_total), every, s, spws,
                                  cgws, use_graph, pc);
        inner_total += h.iters;
        last = h;
        have_last = true;
        relres_last = relres;
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
    o->inner_tol = 0;
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
