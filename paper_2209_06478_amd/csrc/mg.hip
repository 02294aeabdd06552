// HPCG's preconditioner on the device: symmetric Gauss-Seidel smoothing
// inside a multigrid V-cycle, and CG preconditioned by one V-cycle per
// iteration (the benchmark's PCG, Section II-B; the paper's port switches
// it off, Section IV-B).  The cycle follows the HPCG specification: one
// pre- and one post-smoothing sweep per level, restriction by injection of
// the residual at the coarse points, prolongation by adding the coarse
// correction back at those points, one sweep on the coarsest level.
//
// Gauss-Seidel is sequential by nature; on the GPU every level carries a
// colouring in which rows of one colour are not coupled, so a colour's rows
// are updated together by one launch.  The forward sweep visits the colours
// in ascending order, the backward sweep in descending order: the result is
// that of a sequential sweep over rows ordered by (colour, index).  The
// backward sweep starts at the second-highest colour: re-updating the last
// colour right after the forward sweep reproduces the same values (its
// rows see no changed neighbour), so it is skipped.
//
// Levels hold CSR or DIA matrices with FP64 values.  CSR rows are reduced
// by 8 lanes each; DIA rows by one thread sweeping the diagonals in
// ascending offset (ascending column) order, over a colour-ordered copy of
// the diagonals made at set-up (the smoother's values are read at set-up:
// later value updates of a DIA level are not seen by the smoother).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "cg_common.hpp"

namespace dsm {

// threads per workgroup: 128 measured 8% faster per V-cycle than 256 or 512
// (a colour's rows spread over more CUs; 64 was no faster)
constexpr int MB = 128;
constexpr int GSW = 8;       // CSR lanes per row in the smoother
constexpr int GSR = 1;       // DIA rows per thread in the smoother
constexpr int MG_MAX_LEVELS = 8;

}  // namespace dsm

struct dsm_mg_s {
    struct Level {
        dsm_matrix A = nullptr;
        int fmt = 0;
        const void *payload = nullptr;  // A's value array at create (format guard)
        int64_t n = 0;
        std::vector<int64_t> cstart;    // colour c owns rows[cstart[c] .. cstart[c+1])
        int32_t *rows = nullptr;        // rows grouped by colour, ascending inside a colour
        double *diag = nullptr;
        int32_t *f2c = nullptr;         // next level's rows -> rows of this level
        int64_t f2c_t0 = -1;            // >= 0: f2c lists rows[f2c_t0 ...] (one colour, in order)
        double *dperm = nullptr;        // DIA: diagonals in colour order (same pitch), the main diagonal last
        int32_t *offnd = nullptr;       // DIA: offsets of the other diagonals, ascending
        int kd = -1;                    // DIA: index of offset 0 among the ascending offsets
        double *rec = nullptr;          // DIA levels swept in LDS: one record of lds_rw doubles per slot
        int lds_nd = 0;                 // > 0: the level takes the LDS sweep with this many diagonals
        int64_t guard = 0;              // largest |offset| (zero guard band around x in LDS)
        int64_t *cstart_d = nullptr;    // cstart on the device (one-workgroup sweep)
        double *r = nullptr, *x = nullptr;
        dsm::Workspace spws;
    };
    dsm_ctx ctx = nullptr;
    std::vector<Level> L;
    std::vector<std::pair<void *, size_t>> bufs;
    // PCG vectors and state (xw: the iterate of the graph-replayed loop)
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *xw = nullptr;
    double *part_a = nullptr, *part_b = nullptr, *part_c = nullptr;
    dsm::CgState *st = nullptr;
    dsm::Workspace gws;

    void *alloc(size_t b) {
        if (b == 0) b = 16;
        void *p = dsm::dev_alloc(ctx, b);
        bufs.push_back({p, b});
        return p;
    }
    void release() {
        for (auto &l : L) dsm::ws_release(ctx, l.spws);
        dsm::ws_release_host(gws);
        for (auto &b : bufs) dsm::dev_free(ctx, b.first, b.second);
        bufs.clear();
    }
};

namespace dsm {

// ---------------------------------------------------------------- kernels
__device__ __forceinline__ bool stopped(const int *stop) { return stop && *(volatile const int *)stop; }

// The multi-launch kernels below read the done flag at their start but test
// it only before their stores, so the flag's load overlaps the kernel's own
// loads instead of adding a round trip (the flag is written only by other
// launches, so every thread sees the same value).

template <int W>
__global__ void __launch_bounds__(MB) k_symgs_csr(i64 cnt, const i32 *__restrict__ rows, const i32 *__restrict__ rp,
                                                  const i32 *__restrict__ col, const double *__restrict__ val,
                                                  const double *__restrict__ diag, const double *__restrict__ r,
                                                  double *__restrict__ x, const int *stop) {
    const bool halt = stopped(stop);
    constexpr int U = 4;        // entries a lane loads before its x gathers
    const i64 g = ((i64)blockIdx.x * MB + threadIdx.x) / W;
    const int lane = threadIdx.x % W;
    double s = 0;
    i64 i = 0;
    if (g < cnt) {
        i = rows[g];
        const i64 e1 = rp[i + 1];
        for (i64 base = rp[i] + lane; base < e1; base += (i64)U * W) {
            // entries past the row and the diagonal entry take their x
            // operand from the zero word (the diagonal is finite, so its
            // product is a zero that leaves s unchanged): with selects on
            // loaded values the compiler branched around each load
            i32 c[U];
            double v[U], xv[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const i64 k = base + (i64)u * W;
                c[u] = *(k < e1 ? col + k : sentinel_ptr<i32>());
                v[u] = *(k < e1 ? val + k : zero_ptr<double>());
            }
#pragma unroll
            for (int u = 0; u < U; u++) xv[u] = *(c[u] >= 0 && c[u] != i ? x + c[u] : zero_ptr<double>());
#pragma unroll
            for (int u = 0; u < U; u++) s += v[u] * xv[u];
        }
    }
    s = group_sum<W>(s);
    if (g < cnt && lane == 0 && !halt) x[i] = (r[i] - s) / diag[i];
}

// DIA levels keep a colour-ordered copy of the diagonals: slot t of copy
// k holds A(rows[t], rows[t] + offnd_k) for the off-diagonals in ascending
// offset order, and the last copy holds the main diagonal A(rows[t],
// rows[t]).  A colour's rows are then a contiguous, coalesced range of
// every copy (in the natural layout they would be every other slot,
// wasting half of each line fetched), and the divisor is read with them
// instead of gathered at row rows[t].  nod = ndiag - 1 off-diagonals.
__device__ __forceinline__ i64 slot_of(i64 k, i64 kd, i64 ndiag) { return k < kd ? k : (k == kd ? ndiag - 1 : k - 1); }

template <int R>
__global__ void __launch_bounds__(MB) k_symgs_dia(i64 t0, i64 cnt, const i32 *__restrict__ rows, i64 n, i64 nod,
                                                  const i32 *__restrict__ offnd, const double *__restrict__ dperm,
                                                  i64 pitch, const double *__restrict__ r, double *__restrict__ x,
                                                  const int *stop) {
    const bool halt = stopped(stop);
    // R rows per thread, each with its own sum, and the diagonal loop
    // unrolled: several independent loads in flight per thread
    // Loads are unconditional, at clamped in-range addresses, and the
    // products of out-of-range or diagonal slots are selected away: no load
    // sits behind a branch, so the unrolled iterations' loads are all in
    // flight together instead of one round trip per diagonal.
    const i64 g0 = (i64)blockIdx.x * MB * R + threadIdx.x;
    i64 i[R], gq[R];
    double s[R];
#pragma unroll
    for (int q = 0; q < R; q++) {
        const i64 g = g0 + (i64)q * MB;
        gq[q] = g < cnt ? g : 0;
        i[q] = g < cnt ? rows[t0 + g] : -1;
        s[q] = 0;
    }
    double d[R];
#pragma unroll
    for (int q = 0; q < R; q++) d[q] = dperm[nod * pitch + t0 + gq[q]];
#pragma unroll 26
    for (i64 k = 0; k < nod; k++) {
        const i64 off = offnd[k];
        const double *dk = dperm + k * pitch + t0;
#pragma unroll
        for (int q = 0; q < R; q++) {
            const i64 j = i[q] + off;
            const bool ok = i[q] >= 0 && j >= 0 && j < n;
            const double v = dk[gq[q]];
            const double xv = x[ok ? j : 0];
            s[q] += ok ? v * xv : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < R; q++)
        if (i[q] >= 0 && !halt) x[i[q]] = (r[i[q]] - s[q]) / d[q];
}

// The per-colour sweep for levels of ND diagonals (7 or 27): the ND values
// of the thread's slot (off-diagonals, then the main diagonal) are loaded
// first, since they do not depend on the row index; then the row index,
// then every x gather and r.  The loads go into arrays in separate loops so
// that all of them are in flight together (the runtime-length loop above
// lets the compiler interleave loads and products, which reuses registers
// and keeps only a few loads in flight).
template <int ND>
__global__ void __launch_bounds__(MB) k_symgs_dia_nd(i64 t0, i64 cnt, const i32 *__restrict__ rows, i64 n,
                                                     const i32 *__restrict__ offnd, const double *__restrict__ dperm,
                                                     i64 pitch, const double *__restrict__ r, double *__restrict__ x,
                                                     const int *stop) {
#pragma clang fp contract(off)
    const bool halt = stopped(stop);
    // XCD-aware order: each XCD sweeps one contiguous range of the colour,
    // so the x lines its rows gather stay in its own L2 (590 against 618 us
    // per V-cycle at HPCG 104^3 in launch order; streaming the values with a
    // nontemporal hint gained nothing on top)
    const u32 b = xcd_tile(blockIdx.x, gridDim.x);
    const i64 g = (i64)b * MB + threadIdx.x;
    if (g >= cnt) return;
    const i64 t = t0 + g;
    double v[ND];
    const double *p = dperm + t;
#pragma unroll
    for (int k = 0; k < ND; k++) {
        v[k] = *p;
        p += pitch;
    }
    const i64 i = rows[t];
    double xv[ND - 1];
#pragma unroll
    for (int k = 0; k < ND - 1; k++) {
        const i64 j = i + offnd[k];
        xv[k] = x[(j >= 0 && j < n) ? j : 0];
    }
    const double ri = r[i];
    double s = 0;
#pragma unroll
    for (int k = 0; k < ND - 1; k++) {
        const i64 j = i + offnd[k];
        s = s + ((j >= 0 && j < n) ? v[k] * xv[k] : 0.0);
    }
    if (!halt) x[i] = (ri - s) / v[ND - 1];
}

__global__ void k_dia_colour_order(i64 n, i64 ndiag, i64 kd, const double *__restrict__ dval, i64 pitch,
                                   const i32 *__restrict__ rows, double *__restrict__ dperm) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const i64 i = rows[t];
    for (i64 k = 0; k < ndiag; k++) dperm[slot_of(k, kd, ndiag) * pitch + t] = dval[k * pitch + i];
}

// Records of the LDS sweep: slot t holds the ND values of row rows[t] in the
// colour-ordered copy's order (off-diagonals ascending, then the main
// diagonal) followed by the row index itself, so one contiguous record load
// gives a thread everything about its row but x and r.
template <int ND>
__global__ void k_lds_records(i64 n, i64 kd, const double *__restrict__ dval, i64 pitch, const i32 *__restrict__ rows,
                              double *__restrict__ rec) {
    constexpr int RW = ND + 1;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const i64 i = rows[t];
    for (i64 k = 0; k < ND; k++) rec[t * RW + slot_of(k, kd, ND)] = dval[k * pitch + i];
    rec[t * RW + ND] = __builtin_bit_cast(double, i);
}

// DSM_MG_LDS=0 turns the LDS sweep off (small levels then take the
// one-workgroup sweep through the L2), DSM_MG_ND=0 the fixed-length colour
// sweeps (the runtime-length sweep then runs), to time one against the other.
static bool lds_sweep_on();
static bool nd_sweep_on();

// Small levels: the whole sweep (every colour, forward then backward) in
// one workgroup, colours separated by barriers, instead of one launch per
// colour (a launch costs more than a small colour's work).
constexpr int SBT = 1024;                 // threads of the one-workgroup sweep
constexpr i64 BLOCK_LEVEL_ROWS = 8192;    // levels up to this size use it

__device__ __forceinline__ int sweep_colour(int step, int nc) { return step < nc ? step : 2 * nc - 2 - step; }

__global__ void __launch_bounds__(SBT) k_symgs_dia_block(int nc, const i64 *__restrict__ cstart,
                                                         const i32 *__restrict__ rows, i64 n, i64 nod,
                                                         const i32 *__restrict__ offnd,
                                                         const double *__restrict__ dperm, i64 pitch,
                                                         const double *__restrict__ r, double *x, const int *stop,
                                                         int from_zero) {
    if (stopped(stop)) return;
    if (from_zero) {
        for (i64 i = threadIdx.x; i < n; i += SBT) x[i] = 0.0;
        __syncthreads();
    }
    for (int step = 0; step < 2 * nc - 1; step++) {
        const int c = sweep_colour(step, nc);
        const i64 t1 = cstart[c + 1];
        for (i64 t = cstart[c] + threadIdx.x; t < t1; t += SBT) {
            const i64 i = rows[t];
            double s = 0;
#pragma unroll 9
            for (i64 k = 0; k < nod; k++) {
                const i64 j = i + offnd[k];
                const bool ok = j >= 0 && j < n;
                const double v = dperm[k * pitch + t];
                const double xv = x[ok ? j : 0];
                s += ok ? v * xv : 0.0;
            }
            x[i] = (r[i] - s) / dperm[nod * pitch + t];
        }
        __syncthreads();  // the next colour reads this colour's updates
    }
}

// Small DIA levels whose colours have at most LT rows: the whole sweep in
// one workgroup of LT threads with the level's x and r held in LDS (x with
// a zero guard band of the largest |offset| on each side, so a neighbour
// outside the matrix reads +0 and needs no test).  Each step updates one
// colour, a thread owning at most one of its rows: it loads the row's
// record (values and row index; fourteen 16-byte loads in flight at once),
// reads x and r in LDS and writes its x there.  Per step the critical path
// is one record load, the LDS reads and a barrier that orders LDS only,
// instead of the row index, then gathers of x and r from the L2, then a
// store of x to it.  The sums are the same products in the same order as
// the other sweeps (no fused multiply-add).
constexpr int LT = 512;
constexpr i64 LDS_WORDS = 20000;  // 160,000 bytes: x with its guard bands, then r

template <int ND>
__device__ __forceinline__ void load_record(const double *__restrict__ rec, i64 t, double (&v)[ND + 1]) {
    constexpr int RW = ND + 1;
    static_assert(RW % 2 == 0, "records are whole 16-byte words");
    const double2 *p = (const double2 *)(rec + t * RW);
#pragma unroll
    for (int k = 0; k < RW / 2; k++) {
        const double2 w = p[k];
        v[2 * k] = w.x;
        v[2 * k + 1] = w.y;
    }
}

template <int ND>
__global__ void __launch_bounds__(LT) k_symgs_dia_lds(int nc, const i64 *__restrict__ cstart, i64 n, i64 G,
                                                      const i32 *__restrict__ offnd, const double *__restrict__ rec,
                                                      const double *__restrict__ r, double *x, const int *stop,
                                                      int from_zero) {
#pragma clang fp contract(off)
    __shared__ double sm[LDS_WORDS];
    double *xs = sm + G;           // x[j] at xs[j], j in [-G, n + G)
    double *rs = sm + n + 2 * G;   // r[i] at rs[i]
    if (stopped(stop)) return;
    for (i64 k = threadIdx.x; k < n + 2 * G; k += LT) {
        const i64 j = k - G;
        sm[k] = (from_zero || j < 0 || j >= n) ? 0.0 : x[j];
    }
    for (i64 k = threadIdx.x; k < n; k += LT) rs[k] = r[k];
    i32 o[ND - 1];
#pragma unroll
    for (int k = 0; k < ND - 1; k++) o[k] = offnd[k];
    __syncthreads();
    for (int step = 0; step < 2 * nc - 1; step++) {
        const int c = sweep_colour(step, nc);
        const i64 t = cstart[c] + threadIdx.x;
        if (t < cstart[c + 1]) {
            double v[ND + 1];
            load_record<ND>(rec, t, v);
            const i64 i = __builtin_bit_cast(i64, v[ND]);
            double s = 0;
#pragma unroll
            for (int k = 0; k < ND - 1; k++) s = s + v[k] * xs[i + o[k]];
            xs[i] = (rs[i] - s) / v[ND - 1];
        }
        // orders the LDS updates only (no global store is read in the sweep)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
    __syncthreads();
    for (i64 i = threadIdx.x; i < n; i += LT) x[i] = xs[i];
}

template <int W>
__global__ void __launch_bounds__(SBT) k_symgs_csr_block(int nc, const i64 *__restrict__ cstart,
                                                         const i32 *__restrict__ rows, const i32 *__restrict__ rp,
                                                         const i32 *__restrict__ col,
                                                         const double *__restrict__ val,
                                                         const double *__restrict__ diag,
                                                         const double *__restrict__ r, double *x, const int *stop,
                                                         i64 n, int from_zero) {
    if (stopped(stop)) return;
    if (from_zero) {
        for (i64 i = threadIdx.x; i < n; i += SBT) x[i] = 0.0;
        __syncthreads();
    }
    const int lane = threadIdx.x % W, grp = threadIdx.x / W;
    constexpr int G = SBT / W;
    for (int step = 0; step < 2 * nc - 1; step++) {
        const int c = sweep_colour(step, nc);
        const i64 t0 = cstart[c], t1 = cstart[c + 1];
        // every lane of a row group runs the same number of rounds (the
        // shuffle reduction needs all W lanes)
        for (i64 tb = t0; tb < t1; tb += G) {
            const i64 t = tb + grp;
            double s = 0;
            i64 i = 0;
            if (t < t1) {
                i = rows[t];
                const i64 e1 = rp[i + 1];
                for (i64 k = rp[i] + lane; k < e1; k += W) {
                    const i32 cc = col[k];
                    const double v = val[k], xv = *(cc != i ? x + cc : zero_ptr<double>());
                    s += v * xv;
                }
            }
            s = group_sum<W>(s);
            if (t < t1 && lane == 0) x[i] = (r[i] - s) / diag[i];
        }
        __syncthreads();
    }
}

// The first colour of a sweep that starts from x = 0, for every level row at
// once: rows of colour 0 see only zero neighbours, so their update is
// r_i / a_ii exactly as the sweep computes it ((r_i - (+0)) / a_ii); every
// other row starts at 0.  Replaces the zeroing launch and the first colour
// launch.  t walks the colour-ordered rows, colour 0 being [0, n0).
__global__ void k_symgs_first_from_zero(i64 n, i64 n0, const i32 *__restrict__ rows,
                                        const double *__restrict__ diag, int by_slot,
                                        const double *__restrict__ r, double *__restrict__ x, const int *stop) {
    const bool halt = stopped(stop);
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const i64 i = rows[t];
    const double v = t < n0 ? (r[i] - 0.0) / diag[by_slot ? t : i] : 0.0;
    if (!halt) x[i] = v;
}

__global__ void k_mg_zero(i64 n, double *x, const int *stop) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !stopped(stop)) x[i] = 0.0;
}

// rc = (r - A x) at the coarse points, computing A x only for those rows
// (an eighth of the level's rows in the 2:1 coarsening) instead of a full
// SpMV followed by a gather.  Row sums in ascending column order, as in the
// level's SpMV.  Loads unconditional at in-range addresses, products of
// out-of-range slots selected away (as in the SpMV sweeps).
__global__ void __launch_bounds__(MB) k_restrict_dia(i64 nc, const i32 *__restrict__ f2c, i64 n, i64 ndiag,
                                                     const i32 *__restrict__ offs, const double *__restrict__ dval,
                                                     i64 pitch, const double *__restrict__ x,
                                                     const double *__restrict__ r, double *__restrict__ rc,
                                                     const int *stop) {
    const bool halt = stopped(stop);
    const i64 c = (i64)blockIdx.x * MB + threadIdx.x;
    if (c >= nc) return;
    const i64 i = f2c[c];
    double s = 0;
#pragma unroll 27
    for (i64 k = 0; k < ndiag; k++) {
        const i64 j = i + offs[k];
        const bool ok = j >= 0 && j < n;
        const double v = dval[k * pitch + i];
        const double xv = x[ok ? j : 0];
        s += ok ? v * xv : 0.0;
    }
    if (!halt) rc[c] = r[i] - s;
}

// The same residual when the coarse points are exactly one colour of the
// level, listed in the colour's row order: coarse row c sits on slot
// t0 + c of the colour-ordered diagonals, so the values come from one
// contiguous range of each diagonal instead of every other row of every
// other grid line.  Same products in the same order as k_restrict_dia.
__global__ void __launch_bounds__(MB) k_restrict_dia_perm(i64 nc, i64 t0, const i32 *__restrict__ f2c, i64 n,
                                                          i64 ndiag, i64 kd, const i32 *__restrict__ offs,
                                                          const double *__restrict__ dperm, i64 pitch,
                                                          const double *__restrict__ x, const double *__restrict__ r,
                                                          double *__restrict__ rc, const int *stop) {
    const bool halt = stopped(stop);
    const i64 c = (i64)blockIdx.x * MB + threadIdx.x;
    if (c >= nc) return;
    const i64 i = f2c[c];
    const double *dp = dperm + t0 + c;
    double s = 0;
#pragma unroll 27
    for (i64 k = 0; k < ndiag; k++) {
        const i64 j = i + offs[k];
        const bool ok = j >= 0 && j < n;
        const double v = dp[slot_of(k, kd, ndiag) * pitch];
        const double xv = x[ok ? j : 0];
        s += ok ? v * xv : 0.0;
    }
    if (!halt) rc[c] = r[i] - s;
}

template <int W>
__global__ void __launch_bounds__(MB) k_restrict_csr(i64 nc, const i32 *__restrict__ f2c, const i32 *__restrict__ rp,
                                                     const i32 *__restrict__ col, const double *__restrict__ val,
                                                     const double *__restrict__ x, const double *__restrict__ r,
                                                     double *__restrict__ rc, const int *stop) {
    const bool halt = stopped(stop);
    const i64 g = ((i64)blockIdx.x * MB + threadIdx.x) / W;
    const int lane = threadIdx.x % W;
    double s = 0;
    i64 i = 0;
    if (g < nc) {
        i = f2c[g];
        const i64 e1 = rp[i + 1];
        for (i64 k = rp[i] + lane; k < e1; k += W) {
            const double v = val[k], xv = x[col[k]];
            s += v * xv;
        }
    }
    s = group_sum<W>(s);
    if (g < nc && lane == 0 && !halt) rc[g] = r[i] - s;
}

// x += xc at the coarse points (f2c is injective)
__global__ void k_prolong(i64 nc, const i32 *__restrict__ f2c, const double *__restrict__ xc, double *__restrict__ x,
                          const int *stop) {
    const bool halt = stopped(stop);
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) {
        const i32 f = f2c[i];
        const double v = x[f] + xc[i];
        if (!halt) x[f] = v;
    }
}

// colouring check: a stored off-diagonal entry between two rows of one colour
__global__ void k_colour_check_csr(i64 n, const i32 *rp, const i32 *col, const i32 *colour, int *bad) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = 0;
    for (i64 k = rp[i]; k < rp[i + 1]; k++) {
        const i32 c = col[k];
        if (c != i && colour[c] == colour[i]) b = 1;
    }
    if (b) atomicAdd(bad, 1);
}

__global__ void k_colour_check_dia(i64 n, i64 ndiag, const i32 *offs, const double *dval, i64 pitch, const i32 *colour,
                                   int *bad) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = 0;
    for (i64 k = 0; k < ndiag; k++) {
        const i64 j = i + offs[k];
        if (offs[k] != 0 && j >= 0 && j < n && dval[k * pitch + i] != 0.0 && colour[j] == colour[i]) b = 1;
    }
    if (b) atomicAdd(bad, 1);
}

__global__ void k_count_bad_diag(i64 n, const double *d, int *bad) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(d[i] != 0.0 && isfinite(d[i]))) atomicAdd(bad, 1);
}

// ---- preconditioned CG (z = M r from one V-cycle)
// r = b - A x0 and partials of r.r
__global__ void __launch_bounds__(CGB) k_pmg_init(i64 n, const double *b, const double *ax, double *r, double *part) {
    __shared__ double lds[CGB / WAVE];
    double acc = 0;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x) {
        const double ri = b[i] - ax[i];
        r[i] = ri;
        acc += ri * ri;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(CGB) k_pmg_init_state(const double *part, CgState *st, double tol, long long maxit) {
    __shared__ double lds[CGB / WAVE];
    const double rr = reduce_partials(part, lds);
    if (threadIdx.x == 0) {
        st->rho[0] = st->rho[1] = 0;
        st->nr0 = sqrt(rr);
        st->pq = 0;
        st->relres = rr > 0 ? 1.0 : 0.0;
        st->tol = tol;
        st->iters = 0;
        st->maxit = maxit;
        st->done = rr == 0 ? 1 : (!isfinite(rr) ? 3 : (maxit <= 0 ? 2 : 0));
    }
}

// partials of ||b - ax||^2 and ||b||^2
__global__ void __launch_bounds__(CGB) k_pmg_norms(i64 n, const double *b, const double *ax, double *part_rr,
                                                   double *part_bb) {
    __shared__ double lds[CGB / WAVE];
    double rr = 0, bb = 0;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x) {
        const double ri = b[i] - ax[i];
        rr += ri * ri;
        bb += b[i] * b[i];
    }
    rr = block_sum(rr, lds);
    bb = block_sum(bb, lds);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = rr;
        part_bb[blockIdx.x] = bb;
    }
}

// partials of r.z
__global__ void __launch_bounds__(CGB) k_pmg_rz(i64 n, const double *r, const double *z, double *part, CgState *st) {
    __shared__ double lds[CGB / WAVE];
    if (wg_done(&st->done)) return;
    double acc = 0;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x)
        acc += r[i] * z[i];
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// rho_k = r.z; p = z (first iteration) or z + (rho_k / rho_{k-1}) p.  With
// k iterations completed, rho_k goes to slot k & 1, rho_{k-1} is in the other.
__global__ void __launch_bounds__(CGB) k_pmg_update_p(i64 n, const double *z, double *p, const double *part_rz,
                                                      CgState *st) {
    __shared__ double lds[CGB / WAVE];
    if (wg_done(&st->done)) return;
    const double rz = reduce_partials(part_rz, lds);
    const long long k = st->iters;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->rho[k & 1] = rz;
    const bool first = k == 0;
    const double beta = first ? 0.0 : rz / st->rho[(k & 1) ^ 1];
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x)
        p[i] = first ? z[i] : z[i] + beta * p[i];
}

// alpha = rho / p.q; x += alpha p; r -= alpha q; partials of r.r (the SpMV
// before this kernel counted the iteration: rho is in slot (iters - 1) & 1)
__global__ void __launch_bounds__(CGB) k_pmg_update_xr(i64 n, double *x, double *r, const double *p, const double *q,
                                                       const double *part_pq, int npq, double *part_rr, CgState *st) {
    __shared__ double lds[CGB / WAVE];
    if (wg_done(&st->done)) return;
    const double pq = reduce_partials(part_pq, lds, npq);
    const double rho = st->rho[(st->iters - 1) & 1];
    if (!(pq > 0) || !isfinite(pq) || !isfinite(rho)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->done = 3;
        }
        return;
    }
    const double alpha = rho / pq;
    double acc = 0;
    for (i64 i = slice_lo(n) + threadIdx.x, iend = slice_hi(n); i < iend; i += blockDim.x) {
        x[i] = x[i] + alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = acc;
        if (blockIdx.x == 0) st->pq = pq;
    }
}

// convergence test after the update (one workgroup)
__global__ void __launch_bounds__(CGB) k_pmg_check(const double *part_rr, CgState *st) {
    __shared__ double lds[CGB / WAVE];
    if (wg_done(&st->done)) return;
    const double rr = reduce_partials(part_rr, lds);
    if (threadIdx.x == 0) {
        const double nr = sqrt(rr);
        st->relres = st->nr0 > 0 ? nr / st->nr0 : 0.0;
        if (!isfinite(rr)) st->done = 3;
        else if (nr <= st->tol * st->nr0) st->done = 1;
        else if (st->iters >= st->maxit) st->done = 2;
    }
}

template <class X>
__global__ void __launch_bounds__(CGB) k_pmg_dot_pq(i64 n, const X *p, const X *q, double *part, CgState *st) {
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

// ---------------------------------------------------------------- host side
static unsigned vgrid(i64 n) { return (unsigned)std::max<i64>(1, std::min<i64>(CGG, (n + CGB - 1) / CGB)); }

static void check_level_format(const dsm_mg_s::Level &l) {
    DSM_CHECK(l.A->P.fmt == l.fmt && l.A->P.vdt == DSM_F64 &&
                  (l.fmt == DSM_CSR ? (const void *)l.A->P.val : (const void *)l.A->P.dval) == l.payload,
              DSM_E_INVALID, "a level matrix changed format or values array since dsm_mg_create");
}

// One symmetric Gauss-Seidel sweep on level l: x <- S(x) for A_l x = r.
// One symmetric sweep on level l.  from_zero: x is first set to zero (the
// pre-smoothing of a V-cycle), folded into the sweep's first launch.
static void symgs(dsm_mg_s *mg, int l, const double *r, double *x, hipStream_t s, const int *stop,
                  bool from_zero = false) {
    auto &lv = mg->L[l];
    const Payload &P = lv.A->P;
    const int nc = (int)lv.cstart.size() - 1;
    if (nc == 0) return;
    if (lv.lds_nd > 0 && lds_sweep_on()) {
        if (lv.lds_nd == 27)
            hipLaunchKernelGGL(k_symgs_dia_lds<27>, dim3(1), dim3(LT), 0, s, nc, lv.cstart_d, lv.n, lv.guard,
                               lv.offnd, lv.rec, r, x, stop, (int)from_zero);
        else
            hipLaunchKernelGGL(k_symgs_dia_lds<7>, dim3(1), dim3(LT), 0, s, nc, lv.cstart_d, lv.n, lv.guard,
                               lv.offnd, lv.rec, r, x, stop, (int)from_zero);
        DSM_HIP(hipGetLastError());
        return;
    }
    if (lv.n <= BLOCK_LEVEL_ROWS) {
        if (lv.fmt == DSM_CSR)
            hipLaunchKernelGGL(k_symgs_csr_block<GSW>, dim3(1), dim3(SBT), 0, s, nc, lv.cstart_d, lv.rows, P.rp,
                               P.col, (const double *)P.val, lv.diag, r, x, stop, lv.n, (int)from_zero);
        else
            hipLaunchKernelGGL(k_symgs_dia_block, dim3(1), dim3(SBT), 0, s, nc, lv.cstart_d, lv.rows, lv.n,
                               P.ndiag - 1, lv.offnd, lv.dperm, P.pitch, r, x, stop, (int)from_zero);
        DSM_HIP(hipGetLastError());
        return;
    }
    auto colour = [&](int c) {
        const i64 c0 = lv.cstart[c], cnt = lv.cstart[c + 1] - c0;
        if (cnt == 0) return;
        if (lv.fmt == DSM_CSR)
            hipLaunchKernelGGL(k_symgs_csr<GSW>, dim3(grid_for(cnt * GSW, MB)), dim3(MB), 0, s, cnt, lv.rows + c0,
                               P.rp, P.col, (const double *)P.val, lv.diag, r, x, stop);
        else if (P.ndiag == 27 && nd_sweep_on())
            hipLaunchKernelGGL(k_symgs_dia_nd<27>, dim3(grid_for(cnt, MB)), dim3(MB), 0, s, c0, cnt, lv.rows, lv.n,
                               lv.offnd, lv.dperm, P.pitch, r, x, stop);
        else if (P.ndiag == 7 && nd_sweep_on())
            hipLaunchKernelGGL(k_symgs_dia_nd<7>, dim3(grid_for(cnt, MB)), dim3(MB), 0, s, c0, cnt, lv.rows, lv.n,
                               lv.offnd, lv.dperm, P.pitch, r, x, stop);
        else
            hipLaunchKernelGGL(k_symgs_dia<GSR>, dim3(grid_for(cnt, MB * GSR)), dim3(MB), 0, s, c0, cnt, lv.rows,
                               lv.n, P.ndiag - 1, lv.offnd, lv.dperm, P.pitch, r, x, stop);
    };
    int c_first = 0;
    if (from_zero) {
        const bool dia = lv.fmt == DSM_DIA;
        hipLaunchKernelGGL(k_symgs_first_from_zero, dim3(grid_for(lv.n, MB)), dim3(MB), 0, s, lv.n, lv.cstart[1],
                           lv.rows, dia ? lv.dperm + (P.ndiag - 1) * P.pitch : lv.diag, (int)dia, r, x, stop);
        c_first = 1;
    }
    for (int c = c_first; c < nc; c++) colour(c);
    for (int c = nc - 2; c >= 0; c--) colour(c);
    DSM_HIP(hipGetLastError());
}

static bool nd_sweep_on() {
    static const bool v = [] {
        const char *e = getenv("DSM_MG_ND");
        return !(e && e[0] == '0');
    }();
    return v;
}

static bool lds_sweep_on() {
    static const bool v = [] {
        const char *e = getenv("DSM_MG_LDS");
        return !(e && e[0] == '0');
    }();
    return v;
}

// x = M r on level l (x is overwritten; one V-cycle from zero)
static void vcycle(dsm_mg_s *mg, int l, const double *r, double *x, hipStream_t s, const int *stop) {
    auto &lv = mg->L[l];
    if (lv.cstart.size() > 1) symgs(mg, l, r, x, s, stop, true);
    else hipLaunchKernelGGL(k_mg_zero, dim3(grid_for(lv.n, MB)), dim3(MB), 0, s, lv.n, x, stop);
    if (l + 1 == (int)mg->L.size()) return;
    auto &cv = mg->L[l + 1];
    const Payload &P = lv.A->P;
    if (lv.fmt == DSM_DIA && lv.f2c_t0 >= 0)
        hipLaunchKernelGGL(k_restrict_dia_perm, dim3(grid_for(cv.n, MB)), dim3(MB), 0, s, cv.n, lv.f2c_t0, lv.f2c,
                           lv.n, P.ndiag, (i64)lv.kd, P.offs, lv.dperm, P.pitch, x, r, cv.r, stop);
    else if (lv.fmt == DSM_DIA)
        hipLaunchKernelGGL(k_restrict_dia, dim3(grid_for(cv.n, MB)), dim3(MB), 0, s, cv.n, lv.f2c, lv.n, P.ndiag,
                           P.offs, (const double *)P.dval, P.pitch, x, r, cv.r, stop);
    else
        hipLaunchKernelGGL(k_restrict_csr<GSW>, dim3(grid_for(cv.n * GSW, MB)), dim3(MB), 0, s, cv.n, lv.f2c, P.rp,
                           P.col, (const double *)P.val, x, r, cv.r, stop);
    vcycle(mg, l + 1, cv.r, cv.x, s, stop);
    hipLaunchKernelGGL(k_prolong, dim3(grid_for(cv.n, MB)), dim3(MB), 0, s, cv.n, lv.f2c, cv.x, x, stop);
    symgs(mg, l, r, x, s, stop);
    DSM_HIP(hipGetLastError());
}

static void build_level(dsm_mg_s *mg, int l, dsm_matrix A, const int32_t *colour_h, const int32_t *f2c_h,
                        int64_t n_next, hipStream_t s) {
    auto &lv = mg->L[l];
    lv.A = A;
    lv.n = A->nrows;
    lv.fmt = A->P.fmt;
    lv.payload = lv.fmt == DSM_CSR ? (const void *)A->P.val : (const void *)A->P.dval;
    const i64 n = lv.n;
    // colours: host counting sort (stable, so ascending rows inside a colour)
    DSM_CHECK(colour_h || n == 0, DSM_E_INVALID, "null colour array");
    int ncol = 0;
    for (i64 i = 0; i < n; i++) {
        DSM_CHECK(colour_h[i] >= 0 && colour_h[i] < 256, DSM_E_INVALID, "colours must lie in [0, 255]");
        ncol = std::max(ncol, colour_h[i] + 1);
    }
    lv.cstart.assign(ncol + 1, 0);
    for (i64 i = 0; i < n; i++) lv.cstart[colour_h[i] + 1]++;
    for (int c = 0; c < ncol; c++) lv.cstart[c + 1] += lv.cstart[c];
    std::vector<int32_t> rows((size_t)std::max<i64>(n, 1));
    {
        std::vector<int64_t> pos(lv.cstart.begin(), lv.cstart.end() - 1);
        for (i64 i = 0; i < n; i++) rows[pos[colour_h[i]]++] = (int32_t)i;
    }
    lv.rows = (int32_t *)mg->alloc(sizeof(int32_t) * rows.size());
    lv.cstart_d = (int64_t *)mg->alloc(sizeof(int64_t) * lv.cstart.size());
    DSM_HIP(hipMemcpyAsync(lv.cstart_d, lv.cstart.data(), sizeof(int64_t) * lv.cstart.size(), hipMemcpyHostToDevice,
                           s));
    lv.diag = (double *)mg->alloc(sizeof(double) * (size_t)std::max<i64>(n, 1));
    int32_t *col_d = (int32_t *)dev_alloc(mg->ctx, sizeof(int32_t) * (size_t)std::max<i64>(n, 1));
    int *bad = (int *)dev_alloc(mg->ctx, 2 * sizeof(int));
    auto cleanup = [&] {
        (void)hipStreamSynchronize(s);
        dev_free(mg->ctx, col_d, sizeof(int32_t) * (size_t)std::max<i64>(n, 1));
        dev_free(mg->ctx, bad, 2 * sizeof(int));
    };
    try {
        DSM_HIP(hipMemcpyAsync(lv.rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice, s));
        if (n > 0)
            DSM_HIP(hipMemcpyAsync(col_d, colour_h, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
        DSM_HIP(hipMemsetAsync(bad, 0, 2 * sizeof(int), s));
        diagonal_op(A, lv.diag, 0, s);
        if (n > 0) {
            const Payload &P = A->P;
            if (lv.fmt == DSM_CSR)
                hipLaunchKernelGGL(k_colour_check_csr, dim3(grid_for(n, MB)), dim3(MB), 0, s, n, P.rp, P.col, col_d,
                                   bad);
            else
                hipLaunchKernelGGL(k_colour_check_dia, dim3(grid_for(n, MB)), dim3(MB), 0, s, n, P.ndiag, P.offs,
                                   (const double *)P.dval, P.pitch, col_d, bad);
            hipLaunchKernelGGL(k_count_bad_diag, dim3(grid_for(n, MB)), dim3(MB), 0, s, n, lv.diag, bad + 1);
            DSM_HIP(hipGetLastError());
        }
        int hb[2] = {0, 0};
        DSM_HIP(hipMemcpyAsync(hb, bad, sizeof(hb), hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
        DSM_CHECK(hb[0] == 0, DSM_E_INVALID,
                  "level " + std::to_string(l) + ": " + std::to_string(hb[0]) +
                      " rows are coupled to a row of their own colour");
        DSM_CHECK(hb[1] == 0, DSM_E_INVALID,
                  "level " + std::to_string(l) + ": " + std::to_string(hb[1]) +
                      " rows have a zero, missing or non-finite diagonal");
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
    if (lv.fmt == DSM_DIA && n > 0) {
        const Payload &P = A->P;
        // the main diagonal's position among the ascending offsets (every
        // row has a nonzero diagonal, checked above, so offset 0 is stored)
        std::vector<int32_t> offs((size_t)P.ndiag);
        DSM_HIP(hipMemcpyAsync(offs.data(), P.offs, sizeof(int32_t) * offs.size(), hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
        std::vector<int32_t> offnd;
        for (i64 k = 0; k < P.ndiag; k++) {
            if (offs[k] == 0) lv.kd = (int)k;
            else offnd.push_back(offs[k]);
            lv.guard = std::max<int64_t>(lv.guard, std::abs((int64_t)offs[k]));
        }
        DSM_CHECK(lv.kd >= 0, DSM_E_INVALID, "level " + std::to_string(l) + " stores no main diagonal");
        lv.offnd = (int32_t *)mg->alloc(sizeof(int32_t) * std::max<size_t>(offnd.size(), 1));
        if (!offnd.empty())
            DSM_HIP(hipMemcpyAsync(lv.offnd, offnd.data(), sizeof(int32_t) * offnd.size(), hipMemcpyHostToDevice, s));
        lv.dperm = (double *)mg->alloc(sizeof(double) * (size_t)std::max<i64>(P.ndiag * P.pitch, 1));
        hipLaunchKernelGGL(k_dia_colour_order, dim3(grid_for(n, MB)), dim3(MB), 0, s, n, P.ndiag, (i64)lv.kd,
                           (const double *)P.dval, P.pitch, lv.rows, lv.dperm);
        DSM_HIP(hipGetLastError());
        // the LDS sweep: a 7- or 27-diagonal level whose colours have at
        // most LT rows and whose x (with guard bands) and r fit the LDS
        i64 maxc = 0;
        for (size_t c = 0; c + 1 < lv.cstart.size(); c++) maxc = std::max<i64>(maxc, lv.cstart[c + 1] - lv.cstart[c]);
        if ((P.ndiag == 27 || P.ndiag == 7) && maxc <= LT && 2 * n + 2 * lv.guard <= LDS_WORDS) {
            lv.lds_nd = (int)P.ndiag;
            const int rw = lv.lds_nd + 1;
            lv.rec = (double *)mg->alloc(sizeof(double) * (size_t)(n * rw));
            if (lv.lds_nd == 27)
                hipLaunchKernelGGL(k_lds_records<27>, dim3(grid_for(n, MB)), dim3(MB), 0, s, n, (i64)lv.kd,
                                   (const double *)P.dval, P.pitch, lv.rows, lv.rec);
            else
                hipLaunchKernelGGL(k_lds_records<7>, dim3(grid_for(n, MB)), dim3(MB), 0, s, n, (i64)lv.kd,
                                   (const double *)P.dval, P.pitch, lv.rows, lv.rec);
            DSM_HIP(hipGetLastError());
        }
        DSM_HIP(hipStreamSynchronize(s));
    }
    if (l > 0) {
        lv.r = (double *)mg->alloc(sizeof(double) * (size_t)std::max<i64>(n, 1));
        lv.x = (double *)mg->alloc(sizeof(double) * (size_t)std::max<i64>(n, 1));
    }
    if (f2c_h) {
        // injective map into this level's rows
        std::vector<uint8_t> seen((size_t)std::max<i64>(n, 1), 0);
        for (i64 i = 0; i < n_next; i++) {
            const int32_t f = f2c_h[i];
            DSM_CHECK(f >= 0 && f < n && !seen[f], DSM_E_INVALID,
                      "f2c of level " + std::to_string(l) + " must map coarse rows to distinct rows of the level");
            seen[f] = 1;
        }
        // the coarse points are one whole colour, in that colour's row order
        for (size_t c = 0; c + 1 < lv.cstart.size(); c++) {
            const i64 t0 = lv.cstart[c];
            if (lv.cstart[c + 1] - t0 != n_next || n_next == 0) continue;
            bool same = true;
            for (i64 k = 0; k < n_next && same; k++) same = rows[t0 + k] == f2c_h[k];
            if (same) lv.f2c_t0 = t0;
        }
        lv.f2c = (int32_t *)mg->alloc(sizeof(int32_t) * (size_t)std::max<i64>(n_next, 1));
        if (n_next > 0)
            DSM_HIP(hipMemcpyAsync(lv.f2c, f2c_h, sizeof(int32_t) * (size_t)n_next, hipMemcpyHostToDevice, s));
        DSM_HIP(hipStreamSynchronize(s));
    }
}

static CgState run_pcg_mg(dsm_mg_s *mg, const double *b, double *x, double tol, long long maxit, int every,
                          hipStream_t s) {
    auto &l0 = mg->L[0];
    dsm_matrix A = l0.A;
    const i64 n = l0.n;
    CgState *st = mg->st;
    spmv(A, A->P, x, mg->q, DSM_F64, A->variant, s, &l0.spws);
    hipLaunchKernelGGL(k_pmg_init, dim3(CGG), dim3(CGB), 0, s, n, b, mg->q, mg->r, mg->part_b);
    hipLaunchKernelGGL(k_pmg_init_state, dim3(1), dim3(CGB), 0, s, mg->part_b, st, tol, maxit);
    DSM_HIP(hipGetLastError());
    const int *stop = &st->done;
    // the replayed chunks update a copy of x the hierarchy owns (copied back
    // below), so the captured graph holds no caller buffer and serves every
    // solve whatever x is passed
    const bool graphed = cg_graphs_enabled();
    double *xi = graphed ? mg->xw : x;
    if (graphed) DSM_HIP(hipMemcpyAsync(xi, x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    auto enqueue = [&](int, hipStream_t ss) {
        vcycle(mg, 0, mg->r, mg->z, ss, stop);
        hipLaunchKernelGGL(k_pmg_rz, dim3(CGG), dim3(CGB), 0, ss, n, mg->r, mg->z, mg->part_c, st);
        hipLaunchKernelGGL(k_pmg_update_p, dim3(CGG), dim3(CGB), 0, ss, n, mg->z, mg->p, mg->part_c, st);
        int npq = spmv_dot(A, A->P, mg->p, mg->q, DSM_F64, A->variant, ss, mg->part_a, &st->iters, stop);
        if (npq == 0) {
            spmv(A, A->P, mg->p, mg->q, DSM_F64, A->variant, ss, &l0.spws, stop);
            hipLaunchKernelGGL(k_pmg_dot_pq<double>, dim3(CGG), dim3(CGB), 0, ss, n, mg->p, mg->q, mg->part_a, st);
            npq = CGG;
        }
        hipLaunchKernelGGL(k_pmg_update_xr, dim3(CGG), dim3(CGB), 0, ss, n, xi, mg->r, mg->p, mg->q, mg->part_a,
                           npq, mg->part_b, st);
        hipLaunchKernelGGL(k_pmg_check, dim3(1), dim3(CGB), 0, ss, mg->part_b, st);
        DSM_HIP(hipGetLastError());
    };
    char key[256];
    snprintf(key, sizeof key, "pmg|%p|%p|%d|%d", (void *)mg, (void *)xi, A->variant, every);
    const CgState h = run_chunks(mg->gws, key, true, every, maxit, st, s, enqueue);
    if (graphed) DSM_HIP(hipMemcpyAsync(x, xi, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    return h;
}

}  // namespace dsm

using namespace dsm;

static size_t pcg_partials(int64_t n) { return (size_t)dot_partials_cap(n); }

DSM_API dsm_status dsm_mg_create(dsm_ctx ctx, int32_t nlevels, const dsm_matrix *levels, const int32_t *const *f2c,
                                 const int32_t *const *colour, void *stream, dsm_mg *out) {
    return guard([&] {
        DSM_CHECK(ctx && levels && colour && out, DSM_E_INVALID, "null argument");
        DSM_CHECK(nlevels >= 1 && nlevels <= MG_MAX_LEVELS, DSM_E_INVALID, "nlevels must be in [1, 8]");
        DSM_CHECK(nlevels == 1 || f2c, DSM_E_INVALID, "f2c is needed with more than one level");
        for (int l = 0; l < nlevels; l++) {
            dsm_matrix A = levels[l];
            DSM_CHECK(A && A->ctx == ctx, DSM_E_INVALID, "null level matrix or one of another context");
            DSM_CHECK(A->nrows == A->ncols, DSM_E_UNSUPPORTED, "level matrices must be square");
            DSM_CHECK((A->P.fmt == DSM_CSR || A->P.fmt == DSM_DIA) && A->P.vdt == DSM_F64, DSM_E_UNSUPPORTED,
                      "level matrices must be CSR or DIA with FP64 values");
        }
        for (int l = 0; l + 1 < nlevels; l++)
            DSM_CHECK(f2c[l] || levels[l + 1]->nrows == 0, DSM_E_INVALID, "null f2c array");
        DSM_HIP(hipSetDevice(ctx->device));
        hipStream_t s = (hipStream_t)stream;
        auto *mg = new dsm_mg_s();
        mg->ctx = ctx;
        mg->L.resize(nlevels);
        try {
            for (int l = 0; l < nlevels; l++)
                build_level(mg, l, levels[l], colour[l], l + 1 < nlevels ? f2c[l] : nullptr,
                            l + 1 < nlevels ? levels[l + 1]->nrows : 0, s);
            const int64_t n = levels[0]->nrows;
            const size_t nb = sizeof(double) * (size_t)std::max<int64_t>(n, 1);
            mg->r = (double *)mg->alloc(nb);
            mg->z = (double *)mg->alloc(nb);
            mg->p = (double *)mg->alloc(nb);
            mg->q = (double *)mg->alloc(nb);
            mg->xw = (double *)mg->alloc(nb);
            mg->part_a = (double *)mg->alloc(sizeof(double) * pcg_partials(n));
            mg->part_b = (double *)mg->alloc(sizeof(double) * pcg_partials(n));
            mg->part_c = (double *)mg->alloc(sizeof(double) * pcg_partials(n));
            mg->st = (CgState *)mg->alloc(sizeof(CgState));
        } catch (...) {
            (void)hipStreamSynchronize(s);
            mg->release();
            delete mg;
            throw;
        }
        *out = mg;
    });
}

DSM_API dsm_status dsm_mg_destroy(dsm_mg mg) {
    return guard([&] {
        if (!mg) return;
        (void)hipSetDevice(mg->ctx->device);
        (void)hipDeviceSynchronize();
        mg->release();
        delete mg;
    });
}

DSM_API dsm_status dsm_mg_symgs(dsm_mg mg, int32_t level, const double *r, double *x, void *stream) {
    return guard([&] {
        DSM_CHECK(mg, DSM_E_INVALID, "null hierarchy");
        DSM_CHECK(level >= 0 && level < (int)mg->L.size(), DSM_E_INVALID, "no such level");
        auto &lv = mg->L[level];
        DSM_CHECK((r && x) || lv.n == 0, DSM_E_INVALID, "null vector");
        DSM_CHECK(r != x || lv.n == 0, DSM_E_INVALID, "r and x must not alias");
        check_level_format(lv);
        DSM_HIP(hipSetDevice(mg->ctx->device));
        if (lv.n > 0) symgs(mg, level, r, x, (hipStream_t)stream, nullptr);
    });
}

DSM_API dsm_status dsm_mg_apply(dsm_mg mg, const double *r, double *z, void *stream) {
    return guard([&] {
        DSM_CHECK(mg, DSM_E_INVALID, "null hierarchy");
        const int64_t n = mg->L[0].n;
        DSM_CHECK((r && z) || n == 0, DSM_E_INVALID, "null vector");
        DSM_CHECK(r != z || n == 0, DSM_E_INVALID, "r and z must not alias");
        for (auto &lv : mg->L) check_level_format(lv);
        DSM_HIP(hipSetDevice(mg->ctx->device));
        if (n > 0) vcycle(mg, 0, r, z, (hipStream_t)stream, nullptr);
    });
}

DSM_API dsm_status dsm_pcg_mg_solve(dsm_mg mg, const double *b, double *x, const dsm_cg_opts *opts,
                                    dsm_cg_result *result, void *stream) {
    dsm_cg_result R{};
    dsm_status st = guard([&] {
        DSM_CHECK(mg && result, DSM_E_INVALID, "null argument");
        const int64_t n = mg->L[0].n;
        DSM_CHECK((b && x) || n == 0, DSM_E_INVALID, "null vector");
        for (auto &lv : mg->L) check_level_format(lv);
        DSM_HIP(hipSetDevice(mg->ctx->device));
        dsm_cg_opts o;
        dsm_cg_opts_default(&o);
        if (opts) o = *opts;
        DSM_CHECK(o.tol >= 0, DSM_E_INVALID, "negative tolerance");
        hipStream_t s = (hipStream_t)stream;
        if (n == 0) {
            R.status = DSM_OK;
            return;
        }
        const long long maxit = o.maxit > 0 ? o.maxit : std::min<long long>(10 * n, 20000);
        const int every = o.check_every > 0 ? o.check_every : 4;
        CgState h = run_pcg_mg(mg, b, x, o.tol, maxit, every, s);
        R.iters = h.iters;
        R.relres = h.relres;
        R.status = h.done == 1 ? DSM_OK : h.done == 3 ? DSM_E_BREAKDOWN : DSM_E_NOT_CONVERGED;
        // true residual ||b - A x|| / ||b|| with the level-0 matrix
        auto &l0 = mg->L[0];
        spmv(l0.A, l0.A->P, x, mg->q, DSM_F64, l0.A->variant, s, &l0.spws);
        hipLaunchKernelGGL(k_pmg_norms, dim3(CGG), dim3(CGB), 0, s, n, b, mg->q, mg->part_b, mg->part_c);
        DSM_HIP(hipGetLastError());
        std::vector<double> pa(CGG), pb(CGG);
        DSM_HIP(hipMemcpyAsync(pa.data(), mg->part_b, sizeof(double) * CGG, hipMemcpyDeviceToHost, s));
        DSM_HIP(hipMemcpyAsync(pb.data(), mg->part_c, sizeof(double) * CGG, hipMemcpyDeviceToHost, s));
        DSM_HIP(hipStreamSynchronize(s));
        double rr = 0, bb = 0;
        for (int i = 0; i < CGG; i++) {
            rr += pa[i];
            bb += pb[i];
        }
        R.relres_true = bb > 0 ? std::sqrt(rr) / std::sqrt(bb) : std::sqrt(rr);
    });
    if (result) *result = R;
    if (st != DSM_OK) return st;
    return R.status;
}
