// Host-side objects of libdsm: the context (device + HBM budget), the
// dynamic matrix handle with its single active payload, and the interfaces
// between the translation units (scan, conversion, SpMV, CG, selection).
#pragma once

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

struct dsm_ctx_s {
    // Effective bandwidth (GB/s) of the selection model's kernel classes
    // (COO, CSR, DIA, ELL sweeps), learned from every timed selection on
    // this context; seeded with MI355X values measured on the HPCG 27-point
    // matrix at 104^3.  model_variant: the last best kernel variant per format.
    double model_bw[4] = {2700.0, 3400.0, 5700.0, 3950.0};
    int model_variant[6] = {0, 0, 4, 0, 0, 0};
    int device = 0;
    size_t budget = 0;                  // 0: no cap
    std::atomic<size_t> in_use{0};
    std::atomic<int> live_matrices{0};
    std::mutex cache_mu;                // selection cache
    std::map<std::string, std::pair<int, int>> select_cache;  // fingerprint -> (format, variant)
};

#include "admission.hpp"

namespace dsm {

// Device memory charged against the context budget.
void *dev_alloc(dsm_ctx ctx, size_t bytes);
void dev_free(dsm_ctx ctx, void *p, size_t bytes);

// One storage format's arrays.  HYB uses the ELL and COO members, HDC the
// DIA and CSR members; the others use their own.
struct Payload {
    int fmt = DSM_CSR;
    int vdt = DSM_F64;
    // CSR (HDC remainder)
    i32 *rp = nullptr, *col = nullptr;
    void *val = nullptr;
    i64 csr_nnz = 0;
    i32 *rblocks = nullptr;  // adaptive row blocks: nrblocks + 1 row indices
    i64 nrblocks = 0;
    // COO (HYB overflow)
    i32 *crow = nullptr, *ccol = nullptr;
    void *cval = nullptr;
    i64 coo_nnz = 0;
    // DIA (HDC)
    i32 *offs = nullptr;
    void *dval = nullptr;
    i64 ndiag = 0;
    // diagonals grouped into clusters of up to DIA_CLUSTER_K consecutive
    // diagonals whose offsets span at most DIA_CLUSTER_SPAN: nclu records of
    // CLU_REC ints {first diagonal, one past the last, lowest offset, highest
    // offset, offsets of its diagonals relative to the lowest} (clusters.hpp)
    i32 *clu = nullptr;
    i64 nclu = 0;
    // ELL (HYB)
    i32 *ecol = nullptr;
    void *evl = nullptr;
    i64 K = 0;
    i64 pitch = 0;
    double theta = 0.5;
    // owned allocations
    std::vector<std::pair<void *, size_t>> bufs;
    size_t bytes = 0;

    void *alloc(dsm_ctx ctx, size_t b) {
        if (b == 0) b = 16;
        void *p = dev_alloc(ctx, b);
        bufs.push_back({p, b});
        bytes += b;
        return p;
    }
    void release(dsm_ctx ctx) {
        for (auto &pb : bufs) dev_free(ctx, pb.first, pb.second);
        bufs.clear();
        bytes = 0;
        *this = Payload();
    }
};

// Scratch buffers the SpMV/CG paths reuse between calls.  A CG workspace
// also keeps the last captured iteration chunk (a HIP graph) with the key it
// was captured for, and a private stream to replay it on.
struct Workspace {
    void *p = nullptr;
    size_t bytes = 0;
    void *graph = nullptr;  // hipGraphExec_t
    std::string graph_key;
    hipStream_t stream = nullptr;
    void *host = nullptr;         // pinned host staging (hipHostMalloc)
    void *events[2] = {nullptr, nullptr};  // hipEvent_t, for the staging slots
    bool grow_pow2 = false;       // grow to the next power of two (ws_round)
    // When set, device bytes this workspace holds are added here before they
    // are allocated and taken off after they are freed, so a reader that
    // subtracts it from the context's bytes in use never counts a workspace
    // as memory of someone else.
    std::atomic<size_t> *live = nullptr;
    // Memory the workspace does not own (the allocation-free entry point's
    // static buffer): ws_get never frees, replaces or grows it.
    bool fixed = false;
};

}  // namespace dsm

struct dsm_matrix_s {
    dsm_ctx ctx = nullptr;
    int64_t nrows = 0, ncols = 0, nnz = 0;
    dsm::Payload P;
    int variant = 0;
    int batch_lanes = 0;  // CSR lanes per row in the one-workgroup solver (0 = by mean row length)
    hipStream_t last_stream = nullptr;
    dsm::Workspace ws;   // SpMV scratch (COO tile carries)
    dsm::Workspace cgws; // CG vectors and scalars
};

namespace dsm {

// Grows (never shrinks) a workspace; contents are not preserved.  A
// workspace is used on one stream at a time: before its memory is replaced,
// the stream `s` of the call and the workspace's own replay stream are
// synchronised (not the whole device).
void *ws_get(dsm_ctx ctx, Workspace &w, size_t bytes, hipStream_t s);
void ws_release(dsm_ctx ctx, Workspace &w);
// Releases a workspace's graph, stream, events and pinned host staging;
// its device memory stays.
void ws_release_host(Workspace &w);

// ---------------------------------------------------------------- scan.hip
// Exclusive prefix sum of n int32 counts into out[0..n] (out[n] = total);
// returns the total (blocking read-back when `want_total`).
i64 exclusive_scan_i32(dsm_ctx ctx, const i32 *in, i32 *out, i64 n, hipStream_t s, bool want_total);
i64 exclusive_scan_i64(dsm_ctx ctx, const i64 *in, i64 *out, i64 n, hipStream_t s, bool want_total);
// max over n int32 values (blocking)
i32 reduce_max_i32(dsm_ctx ctx, const i32 *in, i64 n, hipStream_t s);

// ---------------------------------------------------------------- convert.hip
// Validates canonical CSR on the device; fails with DSM_E_INVALID.
void validate_csr(dsm_ctx ctx, i64 nrows, i64 ncols, i64 nnz, const i32 *rp, const i32 *col,
                  hipStream_t s);
// Builds the adaptive row blocks of a CSR part.
void build_row_blocks(dsm_ctx ctx, Payload &P, i64 nrows, hipStream_t s);
// Any payload -> canonical CSR payload (values keep their dtype).
Payload to_csr(dsm_matrix m, const Payload &src, hipStream_t s);
// Canonical CSR payload -> payload of `fmt` with values cast to `vdt`.
Payload from_csr(dsm_matrix m, const Payload &csr, int fmt, int vdt, const dsm_convert_opts &o,
                 hipStream_t s);
// Same dtype cast of a CSR payload (returns a new CSR payload).
Payload cast_csr(dsm_matrix m, const Payload &csr, int vdt, hipStream_t s);
// COO triplets (sorted or not) -> canonical CSR payload with F64 values.
Payload coo_to_csr_payload(dsm_matrix m, const i32 *row, const i32 *col, const double *val,
                           i64 nnz, bool sorted, hipStream_t s);
void row_stats(dsm_matrix m, i64 *out, hipStream_t s);
// Whether every stored value of the active format casts to `to` and back
// unchanged (blocking)
bool values_exact(dsm_matrix m, int to, hipStream_t s);
// Structure of a CSR payload that decides every format's size, computed
// on the device without building the formats: longest row, HYB width and
// overflow, number of diagonals, HDC's well-filled diagonals and the entries
// on them, and the entries within `window` of the diagonal.
struct StructFeatures {
    i64 nnz = 0, max_len = 0, hyb_width = 0, hyb_coo = 0, ndiag = 0, hdc_ndiag = 0, hdc_dia_nnz = 0, near = 0;
};
StructFeatures structure_features(dsm_matrix m, const Payload &C, double theta, i64 window, hipStream_t s);

// ---------------------------------------------------------------- spmv.hip
// y = A x for one payload; vector dtype F64 or F32.  `scratch` holds the
// COO tile partials (the matrix's own workspace when null).  When `stop`
// is given, every kernel returns at once if *stop is non-zero (the CG loop's
// convergence flag).  With `acc` the product is added to y (y += A x).
// Allocation-free SpMV: the COO tile partials live in a static device
// buffer of NOALLOC_SCRATCH_BYTES whose per-device address is taken once per
// device at context creation (noalloc_scratch_init, with the device current).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)2 << 20;
void noalloc_scratch_init(int device);
void spmv_noalloc(dsm_matrix m, const void *x, void *y, int vdt, hipStream_t s);
void spmv(dsm_matrix m, const Payload &P, const void *x, void *y, int vdt, int variant,
          hipStream_t s, Workspace *scratch = nullptr, const int *stop = nullptr, bool acc = false);
// diag.hip: mode 0 extracts A(i, i) into d (FP64, 0 where absent); mode 1
// writes d into the diagonal entries the structure holds (blocking).
void diagonal_op(dsm_matrix m, double *d, int mode, hipStream_t s);
// Partial slots the solvers allocate per dot product (at least the 512 of
// their vector kernels; one per 256-row tile of a sweep): spmv_dot writes at
// most this many.
inline i64 dot_partials_cap(i64 n) { return n / 256 + 2 > 512 ? n / 256 + 2 : 512; }
// Square DIA/ELL (and HDC/HYB whose CSR/COO part is empty), and square CSR
// when its launch has at most dot_partials_cap(n) workgroups: y = A x plus,
// per workgroup, the partial of x . y in part[]; *count (when given) is
// incremented once per launch.  Returns the number of partials written, or
// 0 (nothing launched) for other payloads.
int spmv_dot(dsm_matrix m, const Payload &P, const void *x, void *y, int vdt, int variant, hipStream_t s,
             double *part, long long *count, const int *stop);
// Algorithmic bytes one SpMV must move (x read once, y written once).
// Device scratch one SpMV of this payload needs with vec_dtype vectors (the
// COO tile carries of COO and HYB; 0 for the other formats).
size_t spmv_scratch_bytes(const dsm_matrix_s *m, const Payload &P, int vec_dtype);
double spmv_bytes(const dsm_matrix_s *m, const Payload &P, int vec_dtype);
// Number of CSR kernel variants (index 0 = adaptive) and of DIA/ELL sweep
// variants (tile order x row groups per thread x paired rows).
constexpr int CSR_VARIANTS = 16;
constexpr int CSR_VARIANT_NT = 8;
constexpr int SWEEP_VARIANT_COUNT = 16;
// DIA/HDC also take bit 4 (x staged in LDS per diagonal cluster) and bit 5
// (value loads marked nontemporal).
constexpr int DIA_VARIANT_COUNT = 64;
constexpr int DIA_VARIANT_NT = 32;

// Events attached to the kernel launches of one SpMV, for kernel-only
// timing: while t_launch_timing points at one on the calling thread, every
// SpMV launch records `stop` at its own end and the first also records
// `start` at its beginning (hipExtLaunchKernel), so no event packet or host
// gap between queued work and the SpMV is counted.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
    bool started = false;
};
extern thread_local LaunchTiming *t_launch_timing;
// Kernel-only duration (us) of one SpMV of the active payload and variant;
// blocks until it has finished.
double spmv_kernel_us(dsm_matrix m, const void *x, void *y, int vdt, hipStream_t s);
// Reads `bytes` (a multiple of 16) of buf with the streaming read kernel,
// writing DSM_PROBE_PARTIALS partial sums to part: evicts L2 and the
// Infinity Cache of what was there when bytes exceed their capacity.
void flush_read(const void *buf, i64 bytes, double *part, hipStream_t s);
// diagonal clusters of the LDS-staged DIA sweep: at most 9 diagonals whose
// offsets lie within 256 of the first (one z-plane of a 27-point stencil)
constexpr int DIA_CLUSTER_K = 9;
constexpr int DIA_CLUSTER_SPAN = 256;

// ---------------------------------------------------------------- cg.hip / batched.hip
// CG with caller-provided workspaces (vectors/scalars, SpMV scratch).
// `use_graph` replays the iteration chunks from a captured HIP graph; the
// multi-threaded callers (server workers, batched side stream) pass false,
// since a capture in one thread makes device-wide synchronisation in
// another thread fail.
void cg_solve_ws(dsm_matrix m, const double *b, double *x, const dsm_cg_opts &o, dsm_cg_result *res,
                 hipStream_t s, Workspace &cgws, Workspace &spws, bool use_graph);
size_t cg_workspace_bytes(i64 n, bool ir);
// One-workgroup solver: eligibility, per-request device bytes, and timing
// of one solve of `P` with `lanes` (CSR) for `iters` iterations (us).
bool batch_eligible(const dsm_matrix_s *m, i64 small_rows);
size_t batch_request_bytes(i64 n);
size_t batch_arena_fixed();
double time_batched_solve(dsm_matrix m, const Payload &P, int lanes, int iters, hipStream_t s);
struct BatchJob {
    std::vector<dsm_matrix> mats;
    std::vector<const double *> b;
    std::vector<double *> x;
    std::vector<dsm_cg_opts> opts;
};
// Runs one persistent launch for `job` on s and waits for it; fills
// results[0 .. job.mats.size()).
void run_batch(dsm_ctx ctx, const BatchJob &job, dsm_cg_result *results, Workspace &arena, hipStream_t s);

}  // namespace dsm
