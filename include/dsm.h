/*
 * dsm.h - dynamic sparse matrices on one MI355X (gfx950).
 *
 * A C ABI over a "dynamic matrix": one handle that holds a sparse matrix in
 * exactly one active storage format at a time and can switch that format at
 * run time (the DynamicMatrix of arXiv 2209.06478, Section III-A, whose
 * active state changes through activate()/convert, Sections III-A, III-B
 * and IV-B).  On top of the handle sit SpMV (Section III-D, "multiply"),
 * format selection by timed profiling runs (Section V-E, the naive
 * auto-tuner) or by a cost model (Section VII's future work), and the
 * conjugate-gradient loop of HPCG with the preconditioner disabled
 * (Sections II-B and IV-B).  Around them: mixed-precision iterative
 * refinement, a batched one-workgroup-per-system solver and a serving loop
 * with HBM-budget admission; diagonal extraction and update with Jacobi
 * PCG (Sections III-D, IV-B); HPCG's own preconditioner, a multicolour
 * symmetric Gauss-Seidel multigrid V-cycle (Section II-B); y += A x for a
 * matrix split into parts (Sections V-A, V-E); and streaming probes that
 * measure the bandwidth ceiling.
 *
 * Conventions shared by every entry point:
 *   - Indices are int32 (row pointers, rows, columns, offsets); linear slot
 *     indices inside the library are 64-bit.
 *   - A "device pointer" is memory on the handle's GPU (hipMalloc'd, e.g. a
 *     torch CUDA tensor's data_ptr()); a "host pointer" is ordinary memory.
 *     Vectors passed to the library are never owned by it (the paper's
 *     unmanaged containers, Section IV-A): the caller allocates and frees
 *     them and keeps them alive until the stream work that uses them is done.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Asynchronous calls enqueue work on it and return; calls marked
 *     "blocking" synchronise it before returning.
 *   - Every call returns a dsm_status.  No C++ exception and no abort cross
 *     this boundary.  On failure dsm_last_error() returns a thread-local
 *     message describing the most recent error of the calling thread.
 *   - Handles are not thread-safe; distinct handles may be used concurrently
 *     on distinct streams.
 */
#ifndef DSM_H
#define DSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dsm_ctx_s *dsm_ctx;
typedef struct dsm_matrix_s *dsm_matrix;
typedef struct dsm_server_s *dsm_server;
typedef int32_t dsm_status;

/* Storage formats.  Stable integer indices: activate/convert accept them
 * (Section III-A lets the active state be chosen by enum or by index). */
typedef enum {
    DSM_COO = 0, /* coordinate list, sorted by (row, col) (Section II-A)        */
    DSM_CSR = 1, /* compressed rows, ascending columns per row (Section II-A)   */
    DSM_DIA = 2, /* diagonals: offsets + one stored column per diagonal (II-A)  */
    DSM_ELL = 3, /* ELLPACK: K = longest row, K slots per row (Section VI)      */
    DSM_HYB = 4, /* ELL of width K_h + COO overflow (Section VI)                */
    DSM_HDC = 5  /* DIA over well-filled diagonals + CSR remainder (Section VI) */
} dsm_format;
#define DSM_NUM_FORMATS 6

/* Element types of matrix values and of dense vectors. */
typedef enum { DSM_F64 = 0, DSM_F32 = 1, DSM_BF16 = 2 } dsm_dtype;

/* Status codes. */
#define DSM_OK 0
#define DSM_E_INVALID (-1)       /* bad argument or malformed structure         */
#define DSM_E_NOMEM (-2)         /* device allocation failed or budget exceeded */
#define DSM_E_INFEASIBLE (-3)    /* padding above max_pad_ratio                 */
#define DSM_E_UNSUPPORTED (-4)   /* operation not defined for these arguments   */
#define DSM_E_NOT_CONVERGED (-5) /* iteration limit reached, result filled      */
#define DSM_E_BREAKDOWN (-6)     /* p.q <= 0 or a non-finite scalar in CG       */
#define DSM_E_PENDING (-7)       /* server request not finished yet             */
#define DSM_E_DEVICE (-8)        /* HIP runtime error                           */

const char *dsm_status_string(dsm_status s);
/* Message of the calling thread's most recent error ("" if none).  The
 * pointer stays valid until the thread's next dsm_* call. */
const char *dsm_last_error(void);
/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t dsm_version(void);

/* ------------------------------------------------------------------ */
/* Context: device binding and HBM budget.                             */
/* ------------------------------------------------------------------ */
/* Binds to HIP device `device`.  hbm_budget_bytes caps the bytes held by
 * all matrices of this context (payloads plus solver workspaces); 0 means
 * no cap beyond what hipMalloc can give.  Exceeding it fails with
 * DSM_E_NOMEM before anything is allocated. */
dsm_status dsm_ctx_create(int device, size_t hbm_budget_bytes, dsm_ctx *out);
/* Frees the context.  All its matrices must have been destroyed. */
dsm_status dsm_ctx_destroy(dsm_ctx ctx);
/* Bytes currently charged against the budget. */
dsm_status dsm_ctx_bytes_in_use(dsm_ctx ctx, size_t *out);

/* ------------------------------------------------------------------ */
/* Creation (deep copy in, Section III-B).                             */
/* ------------------------------------------------------------------ */
/* Builds a handle whose active format is CSR with FP64 values from
 * canonical CSR arrays: row_ptr[nrows+1] (row_ptr[0] = 0, non-decreasing,
 * row_ptr[nrows] = nnz), col[nnz] strictly ascending inside each row and in
 * [0, ncols), val[nnz].  The arrays are host pointers if on_device == 0,
 * device pointers otherwise; they are copied and remain owned by the caller
 * (free them once `stream` has completed).  The structure is validated on
 * the device; a violation (including duplicate columns) gives
 * DSM_E_INVALID and no handle.  Blocking. */
dsm_status dsm_create_csr(dsm_ctx ctx, int64_t nrows, int64_t ncols, int64_t nnz,
                          const int32_t *row_ptr, const int32_t *col, const double *val,
                          int on_device, void *stream, dsm_matrix *out);

/* Same from COO triplets row[nnz], col[nnz], val[nnz].  If `sorted` is
 * non-zero the triplets must already be in ascending (row, col) order;
 * otherwise they are sorted on the device first.  Duplicate (row, col)
 * pairs give DSM_E_INVALID.  The active format is CSR.  Blocking. */
dsm_status dsm_create_coo(dsm_ctx ctx, int64_t nrows, int64_t ncols, int64_t nnz,
                          const int32_t *row, const int32_t *col, const double *val,
                          int sorted, int on_device, void *stream, dsm_matrix *out);

/* Synchronises the handle's last stream, then frees everything it owns. */
dsm_status dsm_matrix_destroy(dsm_matrix m);

/* ------------------------------------------------------------------ */
/* Format switching (Section III-B "convert", Section IV-B in-place    */
/* conversion of the dynamic matrix).                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    dsm_dtype value_dtype; /* values after conversion: F64, F32 (round to nearest
                              even) or BF16 (round to nearest even of the F32
                              value).  Narrowing is one-way. */
    double hdc_theta;      /* HDC keeps diagonal d in DIA iff count_d >= theta*L_d
                              (L_d = in-range positions on d); <= 0 means 0.5 */
    double max_pad_ratio;  /* DIA/ELL refuse (DSM_E_INFEASIBLE) when stored slots
                              exceed max_pad_ratio * nnz; <= 0 means 16 */
    int32_t hyb_width;     /* HYB ELL width K_h; < 0 means the default rule (the
                              largest k reached by at least ceil(nrows/3) rows) */
} dsm_convert_opts;

/* Fills *o with the defaults (value_dtype = the handle's current dtype is
 * NOT implied: defaults use F64). */
void dsm_convert_opts_default(dsm_convert_opts *o);

/* Converts the handle in place to `fmt` (opts NULL = defaults with the
 * handle's current value dtype).  Transactional: the new payload is built
 * completely, then the old one is freed; on any error the old format stays
 * active and usable.  Peak memory is old + new payload.  Blocking (sizes of
 * the new payload are read back from the device). */
dsm_status dsm_convert(dsm_matrix m, dsm_format fmt, const dsm_convert_opts *opts, void *stream);

/* ------------------------------------------------------------------ */
/* Inspection and export (HostMirror deep copy, Section III-C).        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t format;      /* dsm_format */
    int32_t value_dtype; /* dsm_dtype */
    int64_t nrows, ncols, nnz;
    int64_t ndiag;       /* DIA: diagonals; HDC: DIA-part diagonals; else 0 */
    int64_t ell_width;   /* ELL: K; HYB: K_h; else 0 */
    int64_t coo_nnz;     /* COO: nnz; HYB: entries in the COO part; else 0 */
    int64_t csr_nnz;     /* CSR: nnz; HDC: entries in the CSR part; else 0 */
    int64_t bytes;       /* device bytes held by the active payload */
    int64_t pitch;       /* device row pitch of DIA/ELL arrays (>= nrows) */
    double hdc_theta;
} dsm_info;

dsm_status dsm_get_info(dsm_matrix m, dsm_info *out);

/* Host buffers for dsm_export; size each from dsm_info (value arrays use
 * the handle's value dtype: 8, 4 or 2 bytes per element).  Pointers not
 * used by the active format are ignored and may be NULL.  DIA/ELL arrays
 * are exported with pitch = nrows, diagonal-/slot-major: element (k, i) at
 * k*nrows + i.
 *   COO: row, col, val (coo_nnz)
 *   CSR: row_ptr (nrows+1), col, val (csr_nnz)
 *   DIA: offsets (ndiag), dia_val (ndiag*nrows)
 *   ELL: ell_col, ell_val (ell_width*nrows; empty slot: col -1, value +0)
 *   HYB: ell_col, ell_val (K_h*nrows) + row, col, val (coo_nnz)
 *   HDC: offsets, dia_val (ndiag*nrows) + row_ptr, col, val (csr_nnz) */
typedef struct {
    int32_t *row_ptr;
    int32_t *row;
    int32_t *col;
    void *val;
    int32_t *offsets;
    void *dia_val;
    int32_t *ell_col;
    void *ell_val;
} dsm_export_bufs;

/* Copies the canonical arrays of the active format to host memory.
 * Blocking. */
dsm_status dsm_export(dsm_matrix m, const dsm_export_bufs *bufs, void *stream);

/* Structure statistics of the matrix (computed on the device from the
 * active payload's row structure): out[0..4] = max row length, min row
 * length, sum of lengths, sum of squared lengths, number of empty rows;
 * out[5 + b] for b in 0..32 = number of rows with length in [2^(b-1), 2^b)
 * (bin 0 = empty rows).  `out` is a host array of 38 int64.  Blocking. */
dsm_status dsm_row_stats(dsm_matrix m, int64_t *out, void *stream);
/* Whether storing the values in `to` loses nothing (Sec. III-A: a container
 * is parameterised by the type of the values it holds).  *exact = 1 when
 * every stored value of the active format, cast to `to` as dsm_convert
 * casts (round to nearest even, BF16 through FP32) and widened back, is
 * bit for bit the same; a wider or equal `to` is always exact.  Then an SpMV
 * that accumulates in FP64 over the narrowed values computes the same
 * products as over the original ones, with fewer value bytes (the HPCG
 * matrix: 26 and -1 are exact in BF16).  Runs on `stream` and blocks until
 * the answer is known; allocates one int of scratch. */
dsm_status dsm_values_exact(dsm_matrix m, dsm_dtype to, int32_t *exact, void *stream);

/* ------------------------------------------------------------------ */
/* Diagonal extraction and update (Section III-D lists both; HPCG's    */
/* TestCG edits the system matrix's diagonal, Section IV-B).           */
/* ------------------------------------------------------------------ */
/* d[i] = A(i, i) for i < min(nrows, ncols), 0 where the structure has no
 * diagonal entry; d is a device FP64 vector of that length.  Blocking. */
dsm_status dsm_extract_diagonal(dsm_matrix m, double *d, void *stream);

/* A(i, i) <- d[i] (rounded to the value dtype as in dsm_convert) for every
 * diagonal entry held by the active format; d is a device FP64 vector of
 * length min(nrows, ncols).  A non-zero d[i] for an entry the structure
 * lacks gives DSM_E_INVALID and leaves the matrix unchanged (the structure
 * is never changed; in DIA/HDC a stored zero there would vanish on the next
 * conversion, see dsm_convert).  Blocking. */
dsm_status dsm_update_diagonal(dsm_matrix m, const double *d, void *stream);

/* ------------------------------------------------------------------ */
/* SpMV (Section III-D "multiply").                                    */
/* ------------------------------------------------------------------ */
/* y = A x with x (ncols) and y (nrows) device vectors of `vec_dtype` (F64
 * or F32; they must not alias).  Products are accumulated in vec_dtype;
 * stored F32/BF16 values are widened exactly.  y is written, not read.
 * Non-finite x entries reach only the rows that store an entry in their
 * column: ELL/HYB padding is marked by column -1, and in DIA (and HDC's DIA
 * part) a zero slot is no entry (padding and a stored zero are the same
 * there, as in dsm_convert).  Asynchronous on `stream`. */
dsm_status dsm_spmv(dsm_matrix m, const void *x, void *y, dsm_dtype vec_dtype, void *stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A x
 * exactly as dsm_spmv (same kernels, same result bit for bit), but no call
 * allocates or frees memory.  The only device memory beyond A, x and y,
 * the COO part's per-tile partials (COO, and HYB's COO part), lives in a
 * static 2 MiB device buffer per GPU, set up when the first context on
 * that GPU is created and held until the process ends.  F64 vectors take
 * 16 bytes per 256 COO entries, F32 vectors 8: a COO part beyond about
 * 33.5M entries (F64) or 67M (F32) gives DSM_E_NOMEM and launches nothing.
 * Every call on one GPU shares that buffer: calls that overlap on one GPU
 * (other streams, other threads, other contexts) race on it and must be
 * serialised by the caller.  Asynchronous on `stream`. */
dsm_status dsm_spmv_noalloc(dsm_matrix m, const void *x, void *y, dsm_dtype vec_dtype, void *stream);

/* y += A x, otherwise as dsm_spmv.  Lets a matrix split into parts held in
 * different formats - a rank's regular local block and its irregular ghost
 * block (Section V-A, Fig. 2; Section V-E) - add into one y. */
dsm_status dsm_spmv_accumulate(dsm_matrix m, const void *x, void *y, dsm_dtype vec_dtype, void *stream);

/* Kernel variant used for SpMV.  CSR (0..15): 0 = adaptive row blocks in
 * XCD-aware order, 1..6 = vector kernel with 2^v lanes per row, 7 = adaptive
 * row blocks in launch order; bit 3 (8..15) loads the column indices and
 * values with a nontemporal hint (identical results).  DIA, ELL and the DIA/ELL parts of HDC/HYB
 * (0..15): bit 0 = launch order instead of XCD-aware order, bits 1-2 =
 * log2 of the row groups per thread (1, 2, 4, 4), bit 3 = groups of two
 * adjacent rows fetched with double-width loads.  DIA and HDC also take
 * bit 4 (16..31): x is staged in LDS once per cluster of up to 3 nearby
 * diagonals instead of gathered per diagonal (bits 0-3 keep their meaning),
 * and bit 5 (32..63): the stored values are loaded with a nontemporal hint
 * (faster when the sweep starts with cold caches, slower back to back when
 * the matrix would stay in the Infinity Cache; identical results; the dot
 * form inside CG uses plain loads).  COO: 0.  Set by dsm_select or directly; an out-of-range value gives
 * DSM_E_INVALID. */
dsm_status dsm_set_variant(dsm_matrix m, int32_t variant);
dsm_status dsm_get_variant(dsm_matrix m, int32_t *variant);

/* ------------------------------------------------------------------ */
/* Format selection by timed profiling runs (Section V-E).             */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t warmup;        /* untimed runs per candidate (default 3)          */
    int32_t reps;          /* timed runs per candidate, median kept (def. 20);
                              0 = no profiling runs: pick by the context's
                              cost model (the bytes each format would move,
                              computed from the matrix structure on the
                              device, over per-format bandwidths learned from
                              the context's earlier timed selections) - the
                              online selection Section VII leaves open      */
    int32_t use_cache;     /* reuse a previous choice for the same structure  */
    int32_t tune_variant;  /* also time CSR kernel variants (default 1)       */
    dsm_dtype vec_dtype;   /* vector type the SpMVs are timed with            */
    dsm_dtype value_dtype; /* value type of every candidate                   */
    double max_pad_ratio;  /* as in dsm_convert_opts                          */
    double bytes_prefilter;/* skip candidates moving more than this many times
                              the bytes of the leanest candidate timed so far
                              (CSR is timed first; default 2)                 */
    int32_t target;        /* what the timing measures: 0 = device-wide SpMV;
                              1 = one FP64 CG solve of this matrix inside one
                              workgroup, the path dsm_cg_solve_batched takes
                              (candidates CSR/DIA/ELL; for CSR the lanes per
                              row are tuned too)                              */
    int64_t flush_bytes;   /* 0 (default): warm timing, back-to-back SpMVs as
                              an iterative solver runs them.  > 0 (target 0
                              only): cold timing for an SpMV that finds none
                              of its operands in the caches - before every
                              timed SpMV the selection reads a device buffer
                              of this many bytes (allocated for the call
                              and counted in the context's budget; more than
                              L2 plus the 256 MB Infinity Cache, e.g. 1 GiB),
                              and each time is kernel-only, as
                              dsm_spmv_kernel_time measures it              */
} dsm_select_opts;

void dsm_select_opts_default(dsm_select_opts *o);

typedef struct {
    int32_t chosen;                      /* dsm_format now active           */
    int32_t chosen_variant;              /* kernel variant now active       */
    int32_t cache_hit;                   /* 1 if the cached choice was used */
    int32_t status[DSM_NUM_FORMATS];     /* per candidate: DSM_OK, or why it
                                            was skipped (INFEASIBLE, NOMEM,
                                            UNSUPPORTED = not in mask or
                                            pruned by bytes)                */
    double median_us[DSM_NUM_FORMATS];   /* median SpMV time (0 if skipped) */
    double convert_us[DSM_NUM_FORMATS];  /* conversion time from CSR        */
    double bytes[DSM_NUM_FORMATS];       /* algorithmic bytes per SpMV      */
} dsm_select_report;

/* Converts the handle to each candidate of `candidate_mask` (bit f =
 * format f) that passes the feasibility prefilter, times SpMV, and leaves
 * the fastest one active (ties within 2% go to fewer bytes).  The original
 * payload is kept until the end, so a failure leaves the handle unchanged.
 * Every timed selection also updates the context's cost model.  With
 * reps = 0 the report's median_us holds the model's predictions and only
 * the chosen format is built.  Blocking. */
dsm_status dsm_select(dsm_matrix m, uint32_t candidate_mask, const dsm_select_opts *opts,
                      dsm_select_report *report, void *stream);

/* One profiling run of the active format and kernel variant, the
 * measurement the selection above makes per candidate (Section V-E:
 * profiling runs decide the format): `warmup` untimed SpMVs y = A x, then
 * `reps` SpMVs each bracketed by a pair of events on `stream`; *median_us
 * receives the median of the bracketed durations in microseconds.  x and y
 * are as in dsm_spmv (device vectors of vec_dtype, not aliased); y holds
 * A x afterwards.  reps >= 1, warmup >= 0, otherwise DSM_E_INVALID.
 * Blocking. */
dsm_status dsm_time_spmv(dsm_matrix m, const void *x, void *y, dsm_dtype vec_dtype, int32_t warmup, int32_t reps,
                         double *median_us, void *stream);

/* Kernel-only duration of one SpMV y = A x (as dsm_spmv) in the active
 * format and variant: *us receives the time from the start of its first
 * kernel to the end of its last, from HIP events that its launches record
 * themselves (hipExtLaunchKernel), so neither separate event packets nor
 * the gap after work queued earlier on `stream` are counted; 0 when there
 * is nothing to launch.  Work queued earlier on `stream` (for example a read
 * that evicts the caches) runs first and is not part of the time.
 * Blocking. */
dsm_status dsm_spmv_kernel_time(dsm_matrix m, const void *x, void *y, dsm_dtype vec_dtype, double *us,
                                void *stream);

/* Drops all cached selections of a context. */
dsm_status dsm_select_cache_clear(dsm_ctx ctx);

/* ------------------------------------------------------------------ */
/* Conjugate gradients (HPCG's CG without preconditioner, Section IV-B)*/
/* ------------------------------------------------------------------ */
typedef enum {
    DSM_CG_F64 = 0,   /* FP64 vectors, dots and updates; SpMV accumulates in
                         FP64 over the stored values (any value dtype)       */
    DSM_CG_IR = 1,    /* iterative refinement: outer FP64 residual, dots and
                         update; inner CG in FP32 vectors with FP32 SpMV
                         accumulation and FP64 dot accumulation (values must
                         be F32 or BF16)                                      */
    DSM_CG_JACOBI = 2, /* FP64 CG preconditioned with M = diag(A) (the
                         diagonal from dsm_extract_diagonal; a zero diagonal
                         entry gives DSM_E_INVALID); stops on
                         ||r|| <= tol ||r0||                                   */
    DSM_CG_IR_CONT = 3 /* iterative refinement as DSM_CG_IR, but every inner
                         solve after the first continues the previous one's
                         search direction: its first direction is the new
                         scaled residual plus the last inner direction times
                         the CG step coefficient, as if the previous inner CG
                         had gone on with its recursive residual replaced by
                         the FP64 one (a reliable update), so the Krylov
                         space is not restarted at every outer step        */
} dsm_cg_mode;

typedef struct {
    double tol;          /* stop when ||r|| <= tol * ||r0|| (2-norms)          */
    int64_t maxit;       /* SpMV limit (outer iterations for F64; inner total
                            for IR); <= 0 means min(10*n, 20000)              */
    int32_t mode;        /* dsm_cg_mode                                        */
    double inner_tol;    /* IR: inner relative tolerance; <= 0 (the default)
                            takes the mode's: 1e-5 for DSM_CG_IR, 1e-2 for
                            DSM_CG_IR_CONT; an
                            inner solve stops at max(inner_tol,
                            tol / (2 * current outer residual)), so the last
                            outer step reduces no further than needed         */
    int32_t check_every; /* iterations per chunk between host reads of the
                            device solver state (default: chosen by size);
                            the next chunk is queued before the host waits
                            unless the residual trend predicts convergence, so
                            at most one chunk of early-exiting kernels runs
                            past convergence (results are unaffected)         */
    int32_t max_outer;   /* IR: outer iteration limit (default 50)             */
} dsm_cg_opts;

void dsm_cg_opts_default(dsm_cg_opts *o);

typedef struct {
    int64_t iters;          /* SpMVs inside the iteration (F64), or total inner
                               iterations (IR)                                  */
    int64_t outer_iters;    /* IR refinement steps (F64: 0)                     */
    double relres;          /* final recursive (F64) or true outer (IR) relres  */
    double relres_true;     /* ||b - A x|| / ||b|| recomputed in FP64 at the end */
    int32_t status;         /* DSM_OK, DSM_E_NOT_CONVERGED or DSM_E_BREAKDOWN   */
} dsm_cg_result;

/* Solves A x = b for square A.  b and x are FP64 device vectors of length
 * nrows (8-byte aligned; a 16-byte aligned x lets the FP64 loop's vector
 * updates load two elements at a time, with the same results up to the
 * order of the per-lane partial sums); x holds x0 on entry and the last
 * iterate on return.  The result is filled for OK, NOT_CONVERGED and
 * BREAKDOWN.  Blocking.  Two environment switches pick between equivalent
 * executions of the same iteration: DSM_CG_GRAPH=0 launches the loop
 * eagerly instead of replaying captured graphs (bitwise the same result),
 * and DSM_CG_FUSED=1 runs the two-kernel iteration on square DIA/ELL
 * payloads (slower on MI355X at the HPCG sizes). */
dsm_status dsm_cg_solve(dsm_matrix m, const double *b, double *x, const dsm_cg_opts *opts,
                        dsm_cg_result *result, void *stream);

/* ------------------------------------------------------------------ */
/* Batched solves: many independent CG problems in one launch.          */
/* ------------------------------------------------------------------ */
/* Solves A_k x_k = b_k for k < count with plain FP64 CG, each system with
 * its own matrix handle (square; any format), device vectors b[k], x[k]
 * (x holds x0) and tolerance/maxit from opts[k] (mode must be F64).
 * Systems small enough run whole inside one persistent workgroup each;
 * larger ones are solved one after another on `stream`.  Each system's
 * result is bitwise the same as when it is solved alone.  Blocking. */
dsm_status dsm_cg_solve_batched(int32_t count, const dsm_matrix *mats, const double *const *b,
                                double *const *x, const dsm_cg_opts *opts,
                                dsm_cg_result *results, void *stream);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching of CG solves under an HBM budget.       */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t slots;           /* requests in flight at once (default 64)        */
    size_t hbm_budget;       /* bound on the matrix bytes of the requests in
                                flight plus the device workspaces the workers
                                hold (kept between requests, grown to powers
                                of two); 0 = the context's budget, or no bound
                                when the context has none                    */
    int32_t streams;         /* HIP streams for large requests (default 4)     */
    int64_t small_rows;      /* requests with at most this many rows go to the
                                persistent batched kernel (default 4096, at
                                most 40000)                                   */
    int32_t batch_max;       /* max requests per persistent launch (def. 256)  */
} dsm_server_opts;

void dsm_server_opts_default(dsm_server_opts *o);

typedef struct {
    double arrival_s;  /* submit time, seconds on the server's clock */
    double start_s;    /* first device work enqueued                  */
    double finish_s;   /* result known on the host                    */
} dsm_timestamps;

/* Creates a server with `streams` worker threads, each with its own HIP
 * stream (default priority) and its own workspaces. */
dsm_status dsm_server_create(dsm_ctx ctx, const dsm_server_opts *opts, dsm_server *out);

/* Queues a solve of m x = b (b, x device FP64 vectors; x holds x0).  The
 * matrix and both vectors must stay alive and untouched until the request
 * completes.  A request that could not run on an idle server within the
 * budget (its matrix bytes plus the workspaces it needs) fails with
 * DSM_E_NOMEM at submit; otherwise it waits in arrival order until a slot
 * and budget are free.  Workspace allocations go through the context's
 * budget too: one that fails sends the request back to the head of the
 * queue while other requests are in flight, and fails it with DSM_E_NOMEM
 * (in its result) when none is.  *ticket identifies the request. */
dsm_status dsm_server_submit(dsm_server s, dsm_matrix m, const double *b, double *x,
                             const dsm_cg_opts *opts, uint64_t *ticket);

/* DSM_E_PENDING while the request runs; otherwise DSM_OK and the result and
 * timestamps are filled (the request's solver status is in result->status).
 * A finished ticket can be polled again until dsm_server_destroy. */
dsm_status dsm_server_poll(dsm_server s, uint64_t ticket, dsm_cg_result *result,
                           dsm_timestamps *ts);

/* Blocks until the request finishes, then behaves like dsm_server_poll. */
dsm_status dsm_server_wait(dsm_server s, uint64_t ticket, dsm_cg_result *result,
                           dsm_timestamps *ts);

/* Seconds on the server's clock (the clock of dsm_timestamps). */
double dsm_server_now(dsm_server s);

typedef struct {
    uint64_t submitted;          /* requests accepted by dsm_server_submit       */
    uint64_t completed;          /* requests finished (any status)               */
    uint64_t budget_waits;       /* requests that reached the head of the queue
                                    and waited there for budget with a slot and
                                    a worker free                                */
    uint64_t requeued;           /* units of work sent back to the queue after a
                                    failed workspace allocation                  */
    uint64_t peak_charged_bytes; /* most matrix + workspace bytes charged at once */
    uint64_t workspace_bytes;    /* device workspace the workers hold now        */
    double busy_s;               /* time with at least one unit of work running
                                    (from its start to its result on the host)  */
    double elapsed_s;            /* time since dsm_server_create                 */
} dsm_server_stats;

/* Counters of the server since its creation.  Non-blocking. */
dsm_status dsm_server_get_stats(dsm_server s, dsm_server_stats *out);

/* Waits for every queued request, stops the scheduler and frees the server. */
dsm_status dsm_server_destroy(dsm_server s);

/* ------------------------------------------------------------------ */
/* HPCG's preconditioner (Section II-B: PCG with a symmetric Gauss-     */
/* Seidel smoother inside a multigrid V-cycle; the paper's port turns   */
/* it off, Section IV-B): one pre- and one post-smoothing sweep per     */
/* level, restriction by injection of the residual, prolongation by     */
/* adding the coarse correction back at the injected points, one sweep  */
/* on the coarsest level.                                                */
/* ------------------------------------------------------------------ */
typedef struct dsm_mg_s *dsm_mg;

/* Builds a hierarchy of nlevels (1..8) levels.  levels[0] is the system
 * matrix, levels[l+1] the next coarser one: square matrices of `ctx` in CSR
 * or DIA format with FP64 values and a non-zero diagonal.  They are held,
 * not copied: each must outlive the hierarchy and keep its format and
 * values array (a later dsm_convert makes the calls below fail with
 * DSM_E_INVALID).  The smoother reads the diagonal, and for DIA levels all
 * values (kept in colour order), here: a later dsm_update_diagonal is seen
 * by the level's SpMV but not by its smoother.
 * f2c[l] (l < nlevels - 1; host array of levels[l+1]->nrows entries): the
 * row of level l under each row of level l + 1, all distinct.
 * colour[l] (host array of levels[l]->nrows entries in [0, 255]): rows of
 * one colour must not be coupled by a stored off-diagonal entry.  The sweep
 * updates one colour at a time, ascending forward and descending backward,
 * which equals a sequential Gauss-Seidel sweep over rows in (colour, row)
 * order.  Invalid structure (ranges, coupled colours, zero diagonal) gives
 * DSM_E_INVALID; other formats or dtypes DSM_E_UNSUPPORTED.  Blocking.
 * DIA levels keep a colour-ordered copy of their diagonals (the level's
 * value bytes again); 7- and 27-diagonal levels whose colours have at most
 * 512 rows also keep a record of (diagonals + 1) x 8 bytes per row and sweep in
 * one workgroup with x in LDS.  Two environment switches pick equivalent
 * executions (same results), for timing one against the other:
 * DSM_MG_LDS=0 (small levels sweep through the L2 instead of LDS) and
 * DSM_MG_ND=0 (the runtime-length colour sweep for 7/27 diagonals). */
dsm_status dsm_mg_create(dsm_ctx ctx, int32_t nlevels, const dsm_matrix *levels, const int32_t *const *f2c,
                         const int32_t *const *colour, void *stream, dsm_mg *out);

/* Waits for the device and frees the hierarchy (not the level matrices). */
dsm_status dsm_mg_destroy(dsm_mg mg);

/* One symmetric Gauss-Seidel sweep on level `level`: x <- S(x) for
 * A_level x = r (forward then backward; r, x device FP64 vectors of the
 * level's size, not aliased).  Asynchronous on `stream`. */
dsm_status dsm_mg_symgs(dsm_mg mg, int32_t level, const double *r, double *x, void *stream);

/* z = M r: one V-cycle from z = 0 (r, z device FP64 vectors of
 * levels[0]->nrows, not aliased).  Asynchronous on `stream`; calls that
 * overlap on one hierarchy race (it owns the coarse-level vectors). */
dsm_status dsm_mg_apply(dsm_mg mg, const double *r, double *z, void *stream);

/* CG on levels[0] x = b preconditioned by one V-cycle per iteration (HPCG's
 * solver): b, x device FP64 vectors, x holds x0.  opts: tol, maxit,
 * check_every as for dsm_cg_solve (mode is ignored).  The result and
 * return value follow dsm_cg_solve; result->relres is the recursive
 * ||r||/||r0||, relres_true = ||b - A x|| / ||b||.  Blocking. */
dsm_status dsm_pcg_mg_solve(dsm_mg mg, const double *b, double *x, const dsm_cg_opts *opts,
                            dsm_cg_result *result, void *stream);

/* ------------------------------------------------------------------ */
/* Streaming probes (measurement only): the practical HBM ceiling that  */
/* SpMV bandwidth is compared with.                                     */
/* ------------------------------------------------------------------ */
#define DSM_PROBE_READ 0      /* read `bytes` of src; dst gets DSM_PROBE_PARTIALS FP64 partial sums */
#define DSM_PROBE_COPY 1      /* dst[0, bytes) = src[0, bytes) */
#define DSM_PROBE_WRITE 2     /* dst[0, bytes) = 0 (src unused, may be NULL) */
#define DSM_PROBE_PARTIALS 4096

/* One streaming kernel over device buffers on `stream` (asynchronous).
 * `bytes` must be a multiple of 16 and both buffers 16-byte aligned; src and
 * dst must not overlap.  In read mode dst must hold DSM_PROBE_PARTIALS
 * doubles (their sum is the sum of src read as FP64 words).  Bad arguments
 * give DSM_E_INVALID before anything is launched. */
dsm_status dsm_stream_probe(int32_t mode, const void *src, void *dst, int64_t bytes, void *stream);

/* The gather ceiling of irregular SpMV: reads idx[0, n) (int32, device) and
 * x[idx[k]] (FP64, device, xlen entries; an index outside [0, xlen) reads
 * nothing and adds 0) and writes DSM_PROBE_PARTIALS FP64 partial sums of the
 * gathered values to part (device).  With idx = a CSR column array it moves
 * the x-operand traffic of that matrix's SpMV alone.  Asynchronous on
 * `stream`; bad arguments give DSM_E_INVALID before anything is launched. */
dsm_status dsm_gather_probe(const double *x, int64_t xlen, const int32_t *idx, int64_t n, double *part,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DSM_H */
