/*
 * Reference oracle for dynamic sparse matrices (arXiv 2209.06478).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU statement of what the library computes.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the library
 * itself never links, loads or calls it, and the two share no code.
 *
 * Everything is FP64 and written as loops that follow the definitions:
 *
 *   - Storage formats COO, CSR and DIA follow Section II-A (storage formats).
 *     The canonical encodings fixed here (sorted COO, ascending columns
 *     within a CSR row, row-aligned DIA) are readings of that prose; ELL,
 *     HYB and HDC are only named in Section VI (related work) and their
 *     encodings below are readings of the published formats they cite.
 *   - Conversions (Section III-B, "convert": element-wise copy between
 *     formats) are written directly as "build the canonical encoding of the
 *     same matrix"; the bit-exact contract is on the encodings, not on the
 *     route taken.
 *   - SpMV is the textbook y = A x, summed per row in ascending column
 *     order with a separate multiply and add (no FMA contraction: built with
 *     -ffp-contract=off).  A compensated reference (Ogita, Rump and Oishi's
 *     Dot2, SISC 2005) and the row scale S_i = sum_j |a_ij||x_j| give the
 *     row-scaled acceptance test.
 *   - CG is Hestenes-Stiefel conjugate gradients, i.e. HPCG's solver with
 *     the preconditioner disabled as in the paper's port (Section IV-B), in
 *     plain FP64 with left-to-right dot products.  The preconditioned forms
 *     (Jacobi; HPCG's symmetric Gauss-Seidel / multigrid V-cycle of
 *     Section II-B) use the same loop with z = M r.
 *
 * Parity pins: every function here is checked by the CPU tests against
 * closed forms of the HPCG matrix, dense brute force on tiny inputs,
 * round-trip identities and library routines.  None is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef int32_t i32;
typedef int64_t i64;

/* ------------------------------------------------------------------ */
/* threads (timing mode); results never depend on the thread count     */
/* ------------------------------------------------------------------ */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* CSR validation (Section II-A: row pointers mark row boundaries and   */
/* the last one equals the number of nonzeros).  Canonical form adds:   */
/* columns strictly ascending inside a row, all in [0, ncols).          */
/* returns 0 if valid, a positive code naming the first violation.      */
/* ------------------------------------------------------------------ */
int orc_csr_validate(i64 nrows, i64 ncols, i64 nnz, const i32 *rp, const i32 *col)
{
    if (nrows < 0 || ncols < 0 || nnz < 0) return 1;
    if (rp[0] != 0) return 2;
    if ((i64)rp[nrows] != nnz) return 3;
    for (i64 i = 0; i < nrows; i++) {
        if (rp[i + 1] < rp[i]) return 4;
        for (i64 k = rp[i]; k < rp[i + 1]; k++) {
            if (col[k] < 0 || (i64)col[k] >= ncols) return 5;
            if (k > rp[i] && col[k] <= col[k - 1]) return 6;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* SpMV by definition                                                  */
/* ------------------------------------------------------------------ */
void orc_spmv_csr(i64 nrows, const i32 *rp, const i32 *col, const double *val,
                  const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < nrows; i++) {
        double s = 0.0;
        for (i64 k = rp[i]; k < rp[i + 1]; k++) {
            double p = val[k] * x[col[k]];
            s = s + p;
        }
        y[i] = s;
    }
}

/* Error-free transformations (Knuth's TwoSum; TwoProduct via an exact FMA). */
static void two_sum(double a, double b, double *s, double *e)
{
    double t = a + b;
    double bb = t - a;
    *e = (a - (t - bb)) + (b - bb);
    *s = t;
}

static void two_prod(double a, double b, double *p, double *e)
{
    double t = a * b;
    *e = fma(a, b, -t);
    *p = t;
}

/* Dot2-compensated y*_i = sum_j a_ij x_j and row scale S_i = sum_j |a_ij x_j|. */
void orc_spmv_csr_ref(i64 nrows, const i32 *rp, const i32 *col, const double *val,
                      const double *x, double *yref, double *scale)
{
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < nrows; i++) {
        double s = 0.0, c = 0.0, a = 0.0;
        for (i64 k = rp[i]; k < rp[i + 1]; k++) {
            double p, ep, es;
            two_prod(val[k], x[col[k]], &p, &ep);
            two_sum(s, p, &s, &es);
            c = c + (ep + es);
            a = a + fabs(val[k] * x[col[k]]);
        }
        yref[i] = s + c;
        scale[i] = a;
    }
}

/* ------------------------------------------------------------------ */
/* COO (Section II-A: row, column and value per nonzero).  Canonical  */
/* COO is sorted by (row, col).                                        */
/* ------------------------------------------------------------------ */
void orc_csr_to_coo(i64 nrows, const i32 *rp, i32 *row_out)
{
    for (i64 i = 0; i < nrows; i++)
        for (i64 k = rp[i]; k < rp[i + 1]; k++)
            row_out[k] = (i32)i;
}

/* COO in any order -> canonical CSR by counting sort on rows, then an
 * insertion sort of each row on columns.  Returns 0, or -1 on an index out
 * of range, -2 on a duplicate (row, col). */
int orc_coo_to_csr(i64 nrows, i64 ncols, i64 nnz, const i32 *row, const i32 *col,
                   const double *val, i32 *rp, i32 *col_out, double *val_out)
{
    for (i64 i = 0; i <= nrows; i++) rp[i] = 0;
    for (i64 k = 0; k < nnz; k++) {
        if (row[k] < 0 || row[k] >= nrows || col[k] < 0 || col[k] >= ncols) return -1;
        rp[row[k] + 1]++;
    }
    for (i64 i = 0; i < nrows; i++) rp[i + 1] += rp[i];
    i32 *next = (i32 *)malloc(sizeof(i32) * (size_t)(nrows + 1));
    for (i64 i = 0; i <= nrows; i++) next[i] = rp[i];
    for (i64 k = 0; k < nnz; k++) {
        i32 p = next[row[k]]++;
        col_out[p] = col[k];
        val_out[p] = val[k];
    }
    free(next);
    for (i64 i = 0; i < nrows; i++) {
        for (i64 a = rp[i] + 1; a < rp[i + 1]; a++) {
            i32 c = col_out[a];
            double v = val_out[a];
            i64 b = a - 1;
            while (b >= rp[i] && col_out[b] > c) {
                col_out[b + 1] = col_out[b];
                val_out[b + 1] = val_out[b];
                b--;
            }
            col_out[b + 1] = c;
            val_out[b + 1] = v;
        }
        for (i64 a = rp[i] + 1; a < rp[i + 1]; a++)
            if (col_out[a] == col_out[a - 1]) return -2;
    }
    return 0;
}

void orc_spmv_coo(i64 nrows, i64 nnz, const i32 *row, const i32 *col, const double *val,
                  const double *x, double *y)
{
    for (i64 i = 0; i < nrows; i++) y[i] = 0.0;
    for (i64 k = 0; k < nnz; k++) y[row[k]] = y[row[k]] + val[k] * x[col[k]];
}

/* ------------------------------------------------------------------ */
/* DIA (Section II-A: one stored column per diagonal plus an offset    */
/* array).  Canonical reading: offsets = sorted distinct (col - row)   */
/* over stored entries; vals[k * nrows + i] = A(i, i + off_k) when that */
/* entry is stored, else +0.0 (row-aligned, diagonal-major).            */
/* ------------------------------------------------------------------ */

/* Number of distinct diagonals; writes them ascending if offsets != NULL. */
i64 orc_dia_count(i64 nrows, i64 ncols, const i32 *rp, const i32 *col, i32 *offsets)
{
    i64 span = nrows + ncols - 1;
    if (span <= 0) return 0;
    unsigned char *seen = (unsigned char *)calloc((size_t)span, 1);
    for (i64 i = 0; i < nrows; i++)
        for (i64 k = rp[i]; k < rp[i + 1]; k++)
            seen[(i64)col[k] - i + (nrows - 1)] = 1;
    i64 nd = 0;
    for (i64 d = 0; d < span; d++) {
        if (seen[d]) {
            if (offsets) offsets[nd] = (i32)(d - (nrows - 1));
            nd++;
        }
    }
    free(seen);
    return nd;
}

void orc_csr_to_dia(i64 nrows, i64 ncols, const i32 *rp, const i32 *col, const double *val,
                    i64 ndiag, const i32 *offsets, double *vals)
{
    for (i64 k = 0; k < ndiag * nrows; k++) vals[k] = 0.0;
    for (i64 i = 0; i < nrows; i++) {
        for (i64 e = rp[i]; e < rp[i + 1]; e++) {
            i64 off = (i64)col[e] - i;
            i64 k = 0;
            while (offsets[k] != off) k++; /* linear search: plain and slow */
            vals[k * nrows + i] = val[e];
        }
    }
    (void)ncols;
}

/* DIA -> CSR: walk each row's diagonals in ascending offset (hence ascending
 * column) order and keep in-range slots whose value is not +-0.0 (padding
 * cannot be told apart from a stored zero).  Returns nnz. */
i64 orc_dia_to_csr(i64 nrows, i64 ncols, i64 ndiag, const i32 *offsets, const double *vals,
                   i32 *rp, i32 *col, double *val)
{
    i64 nz = 0;
    rp[0] = 0;
    for (i64 i = 0; i < nrows; i++) {
        for (i64 k = 0; k < ndiag; k++) {
            i64 j = i + offsets[k];
            if (j < 0 || j >= ncols) continue;
            double v = vals[k * nrows + i];
            if (v == 0.0) continue;
            if (col) col[nz] = (i32)j;
            if (val) val[nz] = v;
            nz++;
        }
        rp[i + 1] = (i32)nz;
    }
    return nz;
}

/* y = A x over the DIA slots.  A slot holding +0 or -0 is no entry of the
 * matrix (padding and a stored zero cannot be told apart, the reading the
 * conversion out of DIA follows too), so its x operand does not enter the
 * row sum: with finite x that changes nothing, and an infinite or NaN x_j
 * reaches only the rows that store a nonzero in column j, as in CSR. */
void orc_spmv_dia(i64 nrows, i64 ncols, i64 ndiag, const i32 *offsets, const double *vals,
                  const double *x, double *y)
{
    for (i64 i = 0; i < nrows; i++) {
        double s = 0.0;
        for (i64 k = 0; k < ndiag; k++) {
            i64 j = i + offsets[k];
            double a = (j >= 0 && j < ncols) ? vals[k * nrows + i] : 0.0;
            if (a != 0.0) s = s + a * x[j];
        }
        y[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* ELL: width K = longest row; slot (k, i) at k * nrows + i holds the  */
/* k-th entry of row i (ascending column order); empty slots carry the */
/* sentinel column -1 and value +0.0.                                   */
/* ------------------------------------------------------------------ */
i32 orc_ell_width(i64 nrows, const i32 *rp)
{
    i32 K = 0;
    for (i64 i = 0; i < nrows; i++)
        if (rp[i + 1] - rp[i] > K) K = rp[i + 1] - rp[i];
    return K;
}

void orc_csr_to_ell_part(i64 nrows, const i32 *rp, const i32 *col, const double *val, i32 K,
                         i32 *ecol, double *evals)
{
    for (i64 k = 0; k < (i64)K; k++) {
        for (i64 i = 0; i < nrows; i++) {
            i64 len = rp[i + 1] - rp[i];
            if (k < len) {
                ecol[k * nrows + i] = col[rp[i] + k];
                evals[k * nrows + i] = val[rp[i] + k];
            } else {
                ecol[k * nrows + i] = -1;
                evals[k * nrows + i] = 0.0;
            }
        }
    }
}

/* ELL -> CSR: slots in k order per row, stopping at nothing: every
 * non-sentinel slot is an entry.  Returns nnz. */
i64 orc_ell_to_csr(i64 nrows, i32 K, const i32 *ecol, const double *evals, i32 *rp, i32 *col,
                   double *val)
{
    i64 nz = 0;
    rp[0] = 0;
    for (i64 i = 0; i < nrows; i++) {
        for (i64 k = 0; k < (i64)K; k++) {
            i32 c = ecol[k * nrows + i];
            if (c < 0) continue;
            if (col) col[nz] = c;
            if (val) val[nz] = evals[k * nrows + i];
            nz++;
        }
        rp[i + 1] = (i32)nz;
    }
    return nz;
}

void orc_spmv_ell(i64 nrows, i32 K, const i32 *ecol, const double *evals, const double *x,
                  double *y)
{
    for (i64 i = 0; i < nrows; i++) {
        double s = 0.0;
        for (i64 k = 0; k < (i64)K; k++) {
            i32 c = ecol[k * nrows + i];
            if (c >= 0) s = s + evals[k * nrows + i] * x[c];
        }
        y[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* HYB = ELL of width K_h + COO overflow.  K_h rule: the largest k for  */
/* which at least ceil(nrows / 3) rows have length >= k (the "one third */
/* of the rows" heuristic of the published HYB format).                 */
/* ------------------------------------------------------------------ */
i32 orc_hyb_width(i64 nrows, const i32 *rp)
{
    if (nrows == 0) return 0;
    i64 need = (nrows + 2) / 3;
    i32 K = orc_ell_width(nrows, rp);
    /* count[k] = rows of length exactly k; walking k down accumulates the
     * number of rows with length >= k */
    i64 *count = (i64 *)calloc((size_t)K + 1, sizeof(i64));
    for (i64 i = 0; i < nrows; i++) count[rp[i + 1] - rp[i]]++;
    i64 ge = 0;
    i32 k = K;
    for (; k > 0; k--) {
        ge += count[k];
        if (ge >= need) break;
    }
    free(count);
    return k;
}

/* Number of entries that overflow into the COO part of HYB(K_h). */
i64 orc_hyb_coo_count(i64 nrows, const i32 *rp, i32 Kh)
{
    i64 c = 0;
    for (i64 i = 0; i < nrows; i++) {
        i64 len = rp[i + 1] - rp[i];
        if (len > Kh) c += len - Kh;
    }
    return c;
}

void orc_csr_to_hyb(i64 nrows, const i32 *rp, const i32 *col, const double *val, i32 Kh,
                    i32 *ecol, double *evals, i32 *crow, i32 *ccol, double *cval)
{
    orc_csr_to_ell_part(nrows, rp, col, val, Kh, ecol, evals);
    i64 c = 0;
    for (i64 i = 0; i < nrows; i++) {
        for (i64 e = rp[i] + Kh; e < rp[i + 1]; e++) {
            crow[c] = (i32)i;
            ccol[c] = col[e];
            cval[c] = val[e];
            c++;
        }
    }
}

/* HYB -> CSR: per row, the ELL slots then that row's COO entries. */
i64 orc_hyb_to_csr(i64 nrows, i32 Kh, const i32 *ecol, const double *evals, i64 ncoo,
                   const i32 *crow, const i32 *ccol, const double *cval, i32 *rp, i32 *col,
                   double *val)
{
    i64 nz = 0, c = 0;
    rp[0] = 0;
    for (i64 i = 0; i < nrows; i++) {
        for (i64 k = 0; k < (i64)Kh; k++) {
            i32 cc = ecol[k * nrows + i];
            if (cc < 0) continue;
            col[nz] = cc;
            val[nz] = evals[k * nrows + i];
            nz++;
        }
        while (c < ncoo && crow[c] == i) {
            col[nz] = ccol[c];
            val[nz] = cval[c];
            nz++;
            c++;
        }
        rp[i + 1] = (i32)nz;
    }
    return nz;
}

/* ------------------------------------------------------------------ */
/* HDC = DIA over the "true" diagonals + CSR remainder.  Diagonal d is  */
/* true when its stored count c_d satisfies c_d >= theta * L_d, with    */
/* L_d the number of in-range positions on d (both in FP64).            */
/* ------------------------------------------------------------------ */
static i64 diag_len(i64 nrows, i64 ncols, i64 d)
{
    i64 lo = d < 0 ? -d : 0;           /* first row with 0 <= i + d */
    i64 hi = ncols - d;                 /* rows i < ncols - d */
    if (hi > nrows) hi = nrows;
    return hi > lo ? hi - lo : 0;
}

/* Writes the true offsets ascending (if out != NULL); returns their count. */
i64 orc_hdc_true_diags(i64 nrows, i64 ncols, const i32 *rp, const i32 *col, double theta,
                       i32 *out)
{
    i64 span = nrows + ncols - 1;
    if (span <= 0) return 0;
    i64 *cnt = (i64 *)calloc((size_t)span, sizeof(i64));
    for (i64 i = 0; i < nrows; i++)
        for (i64 k = rp[i]; k < rp[i + 1]; k++)
            cnt[(i64)col[k] - i + (nrows - 1)]++;
    i64 nt = 0;
    for (i64 s = 0; s < span; s++) {
        i64 d = s - (nrows - 1);
        if (cnt[s] > 0 && (double)cnt[s] >= theta * (double)diag_len(nrows, ncols, d)) {
            if (out) out[nt] = (i32)d;
            nt++;
        }
    }
    free(cnt);
    return nt;
}

/* Splits canonical CSR into HDC: DIA part (canonical DIA over the true
 * offsets, pitch nrows) and CSR part (entries on other diagonals). */
i64 orc_csr_to_hdc(i64 nrows, i64 ncols, const i32 *rp, const i32 *col, const double *val,
                   i64 ntrue, const i32 *offs, double *dvals, i32 *crp, i32 *ccol, double *cval)
{
    for (i64 k = 0; k < ntrue * nrows; k++) dvals[k] = 0.0;
    i64 nz = 0;
    crp[0] = 0;
    for (i64 i = 0; i < nrows; i++) {
        for (i64 e = rp[i]; e < rp[i + 1]; e++) {
            i64 off = (i64)col[e] - i;
            i64 k = 0;
            while (k < ntrue && offs[k] != off) k++;
            if (k < ntrue) {
                dvals[k * nrows + i] = val[e];
            } else {
                if (ccol) ccol[nz] = col[e];
                if (cval) cval[nz] = val[e];
                nz++;
            }
        }
        crp[i + 1] = (i32)nz;
    }
    (void)ncols;
    return nz;
}

/* HDC -> CSR: merge each row's DIA slots (nonzero, in range) with its CSR
 * entries by ascending column. */
i64 orc_hdc_to_csr(i64 nrows, i64 ncols, i64 ntrue, const i32 *offs, const double *dvals,
                   const i32 *crp, const i32 *ccol, const double *cval, i32 *rp, i32 *col,
                   double *val)
{
    i64 nz = 0;
    rp[0] = 0;
    for (i64 i = 0; i < nrows; i++) {
        i64 k = 0, e = crp[i];
        for (;;) {
            /* next DIA candidate */
            while (k < ntrue) {
                i64 j = i + offs[k];
                if (j >= 0 && j < ncols && dvals[k * nrows + i] != 0.0) break;
                k++;
            }
            int have_d = k < ntrue, have_c = e < crp[i + 1];
            if (!have_d && !have_c) break;
            i64 jd = have_d ? i + offs[k] : INT64_MAX;
            i64 jc = have_c ? (i64)ccol[e] : INT64_MAX;
            if (jd < jc) {
                col[nz] = (i32)jd;
                val[nz] = dvals[k * nrows + i];
                k++;
            } else {
                col[nz] = (i32)jc;
                val[nz] = cval[e];
                e++;
            }
            nz++;
        }
        rp[i + 1] = (i32)nz;
    }
    return nz;
}

/* ------------------------------------------------------------------ */
/* Value casts for reduced-precision storage: FP32 = round-to-nearest- */
/* even of the FP64 value; BF16 = round-to-nearest-even of that FP32    */
/* value to the upper 16 bits.                                          */
/* ------------------------------------------------------------------ */
void orc_cast_f32(i64 n, const double *in, float *out)
{
    for (i64 i = 0; i < n; i++) out[i] = (float)in[i]; /* C conversion: current mode, RNE */
}

static uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u); /* NaN stays NaN */
    /* add half an ulp of the kept part, plus one more if the kept part is odd */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

void orc_cast_bf16(i64 n, const double *in, uint16_t *out)
{
    for (i64 i = 0; i < n; i++) out[i] = f32_to_bf16_rne((float)in[i]);
}

void orc_bf16_to_f64(i64 n, const uint16_t *in, double *out)
{
    for (i64 i = 0; i < n; i++) {
        uint32_t u = (uint32_t)in[i] << 16;
        float f;
        memcpy(&f, &u, 4);
        out[i] = (double)f;
    }
}

/* ------------------------------------------------------------------ */
/* Structure statistics: row-length extremes and sums, log2 histogram  */
/* (bin b holds lengths in [2^(b-1), 2^b), bin 0 holds empty rows).     */
/* ------------------------------------------------------------------ */
void orc_row_stats(i64 nrows, const i32 *rp, i64 *out /* [5 + 33] */)
{
    i64 mx = 0, mn = nrows ? INT64_MAX : 0, s = 0, s2 = 0, empty = 0;
    for (int b = 0; b < 33; b++) out[5 + b] = 0;
    for (i64 i = 0; i < nrows; i++) {
        i64 len = rp[i + 1] - rp[i];
        if (len > mx) mx = len;
        if (len < mn) mn = len;
        s += len;
        s2 += len * len;
        if (len == 0) empty++;
        int b = 0;
        while (b < 32 && ((i64)1 << b) <= len) b++;
        out[5 + b]++;
    }
    out[0] = mx;
    out[1] = mn;
    out[2] = s;
    out[3] = s2;
    out[4] = empty;
}

/* ------------------------------------------------------------------ */
/* Conjugate gradients (HPCG's solver with the preconditioner off).    */
/*   r = b - A x0, p = r, rho = r.r, stop when ||r|| <= tol ||r0||.     */
/*   each iteration: q = A p; alpha = rho / p.q; x += alpha p;          */
/*   r -= alpha q; rho' = r.r; test; beta = rho'/rho; p = r + beta p.   */
/* Status: 0 converged, 1 not converged (maxit), 2 breakdown (p.q <= 0 */
/* or a non-finite scalar).  iters counts the SpMVs in the loop.        */
/* ------------------------------------------------------------------ */
static double dot_lr(i64 n, const double *a, const double *b)
{
    double s = 0.0;
    for (i64 i = 0; i < n; i++) s = s + a[i] * b[i];
    return s;
}

/* q = A x by definition.  Rows are independent and each is summed by one
 * thread in ascending column order, so the result does not depend on the
 * number of threads; only the dot products (dot_lr) stay sequential. */
static void spmv_rows(i64 n, const i32 *rp, const i32 *col, const double *val,
                      const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < n; i++) {
        double s = 0.0;
        for (i64 k = rp[i]; k < rp[i + 1]; k++) s = s + val[k] * x[col[k]];
        y[i] = s;
    }
}

int orc_cg(i64 n, const i32 *rp, const i32 *col, const double *val, const double *b,
           double *x, double tol, i64 maxit, i64 *iters_out, double *relres_out)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    spmv_rows(n, rp, col, val, x, q);
    for (i64 i = 0; i < n; i++) r[i] = b[i] - q[i];
    for (i64 i = 0; i < n; i++) p[i] = r[i];
    double rho = dot_lr(n, r, r);
    double nr0 = sqrt(rho);
    int status = 1;
    i64 it = 0;
    double relres = nr0 > 0.0 ? 1.0 : 0.0;
    if (nr0 == 0.0) {
        status = 0;
    } else if (!isfinite(nr0)) {
        status = 2;
    } else {
        while (it < maxit) {
            spmv_rows(n, rp, col, val, p, q);
            it++;
            double pq = dot_lr(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) {
                status = 2;
                break;
            }
            double alpha = rho / pq;
#pragma omp parallel for schedule(static)
            for (i64 i = 0; i < n; i++) {
                x[i] = x[i] + alpha * p[i];
                r[i] = r[i] - alpha * q[i];
            }
            double rho1 = dot_lr(n, r, r);
            if (!isfinite(rho1)) {
                status = 2;
                break;
            }
            relres = sqrt(rho1) / nr0;
            if (sqrt(rho1) <= tol * nr0) {
                status = 0;
                break;
            }
            double beta = rho1 / rho;
#pragma omp parallel for schedule(static)
            for (i64 i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
            rho = rho1;
        }
    }
    free(r);
    free(p);
    free(q);
    *iters_out = it;
    *relres_out = relres;
    return status;
}

/* True relative residual ||b - A x|| / ||b|| with each r_i formed by a
 * compensated sum (Dot2 over the terms b_i and -a_ij x_j). */
double orc_true_relres(i64 n, const i32 *rp, const i32 *col, const double *val,
                       const double *b, const double *x)
{
    double nr = 0.0, nb = 0.0;
    for (i64 i = 0; i < n; i++) {
        double s = b[i], c = 0.0;
        for (i64 k = rp[i]; k < rp[i + 1]; k++) {
            double p, ep, es;
            two_prod(-val[k], x[col[k]], &p, &ep);
            two_sum(s, p, &s, &es);
            c = c + (ep + es);
        }
        double ri = s + c;
        nr = nr + ri * ri;
        nb = nb + b[i] * b[i];
    }
    return nb > 0.0 ? sqrt(nr) / sqrt(nb) : sqrt(nr);
}

/* ------------------------------------------------------------------ */
/* Diagonal extraction and update (Section III-D lists both; HPCG's    */
/* TestCG edits the diagonal, Section IV-B).  d[i] = A(i,i) for         */
/* i < min(nrows, ncols), 0 where the structure has no such entry.      */
/* ------------------------------------------------------------------ */
void orc_extract_diagonal(i64 nrows, i64 ncols, const i32 *rp, const i32 *col, const double *val, double *d)
{
    i64 nd = nrows < ncols ? nrows : ncols;
    for (i64 i = 0; i < nd; i++) {
        d[i] = 0.0;
        for (i64 k = rp[i]; k < rp[i + 1]; k++)
            if (col[k] == i) d[i] = val[k];
    }
}

/* A(i,i) <- d[i] where the entry exists; returns the number of rows whose
 * diagonal entry is missing while d[i] != 0 (then nothing is written). */
i64 orc_update_diagonal(i64 nrows, i64 ncols, const i32 *rp, const i32 *col, double *val, const double *d)
{
    i64 nd = nrows < ncols ? nrows : ncols, bad = 0;
    for (i64 i = 0; i < nd; i++) {
        int found = 0;
        for (i64 k = rp[i]; k < rp[i + 1]; k++)
            if (col[k] == i) found = 1;
        if (!found && d[i] != 0.0) bad++;
    }
    if (bad) return bad;
    for (i64 i = 0; i < nd; i++)
        for (i64 k = rp[i]; k < rp[i + 1]; k++)
            if (col[k] == i) val[k] = d[i];
    return 0;
}

/* ------------------------------------------------------------------ */
/* Jacobi-preconditioned CG (M = diag(A)), textbook form:               */
/*   r = b - A x0, z = M^-1 r, p = z, rho = r.z                          */
/*   loop: q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q;       */
/*         stop when ||r|| <= tol ||r0||; z = M^-1 r; rho' = r.z;        */
/*         beta = rho'/rho; p = z + beta p.                              */
/* Status as orc_cg, plus 3 = a zero diagonal entry.                     */
/* ------------------------------------------------------------------ */
int orc_pcg_jacobi(i64 n, const i32 *rp, const i32 *col, const double *val, const double *b, double *x,
                   double tol, i64 maxit, i64 *iters_out, double *relres_out)
{
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *dg = (double *)malloc(sz), *r = (double *)malloc(sz), *z = (double *)malloc(sz);
    double *p = (double *)malloc(sz), *q = (double *)malloc(sz);
    orc_extract_diagonal(n, n, rp, col, val, dg);
    int status = 1;
    i64 it = 0;
    double relres = 1.0;
    for (i64 i = 0; i < n; i++)
        if (dg[i] == 0.0) status = 3;
    if (status == 3) goto out;
    spmv_rows(n, rp, col, val, x, q);
    for (i64 i = 0; i < n; i++) r[i] = b[i] - q[i];
    for (i64 i = 0; i < n; i++) z[i] = r[i] / dg[i];
    for (i64 i = 0; i < n; i++) p[i] = z[i];
    double rho = dot_lr(n, r, z);
    double nr0 = sqrt(dot_lr(n, r, r));
    if (nr0 == 0.0) {
        status = 0;
        relres = 0.0;
        goto out;
    }
    if (!isfinite(nr0) || !isfinite(rho)) {
        status = 2;
        goto out;
    }
    while (it < maxit) {
        spmv_rows(n, rp, col, val, p, q);
        it++;
        double pq = dot_lr(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = 2;
            break;
        }
        double alpha = rho / pq;
        for (i64 i = 0; i < n; i++) x[i] = x[i] + alpha * p[i];
        for (i64 i = 0; i < n; i++) r[i] = r[i] - alpha * q[i];
        double nr = sqrt(dot_lr(n, r, r));
        if (!isfinite(nr)) {
            status = 2;
            break;
        }
        relres = nr / nr0;
        if (nr <= tol * nr0) {
            status = 0;
            break;
        }
        for (i64 i = 0; i < n; i++) z[i] = r[i] / dg[i];
        double rho1 = dot_lr(n, r, z);
        double beta = rho1 / rho;
        for (i64 i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        rho = rho1;
    }
out:
    free(dg);
    free(r);
    free(z);
    free(p);
    free(q);
    *iters_out = it;
    *relres_out = relres;
    return status;
}

/* ------------------------------------------------------------------ */
/* HPCG's preconditioner (Section II-B: PCG with a symmetric            */
/* Gauss-Seidel smoother inside a multigrid V-cycle; the paper's port   */
/* disables it, Section IV-B).  The structure follows the published     */
/* HPCG specification (Dongarra, Heroux, Luszczek, SAND2013-8752):      */
/* one pre- and one post-smoothing sweep per level, restriction by      */
/* injection of the residual at the coarse points, prolongation by      */
/* adding the coarse correction back at those points, one smoothing     */
/* sweep on the coarsest level.                                         */
/*                                                                      */
/* The Gauss-Seidel sweep visits rows in a given order (HPCG leaves the */
/* order to the implementation; a multicolour order makes rows of one   */
/* colour independent).  Forward: x_i <- (r_i - sum_{j != i} a_ij x_j) / */
/* a_ii for i in order, each row seeing the values already updated;     */
/* backward: the same in reverse order.  The off-diagonal sum runs in   */
/* ascending column order.  Returns the number of rows with a zero or   */
/* missing diagonal (then x is left untouched).                         */
/* ------------------------------------------------------------------ */
static double row_offdiag(const i32 *rp, const i32 *col, const double *val, const double *x, i64 i,
                          double *aii)
{
    double s = 0.0;
    *aii = 0.0;
    for (i64 k = rp[i]; k < rp[i + 1]; k++) {
        if (col[k] == i) *aii = val[k];
        else s = s + val[k] * x[col[k]];
    }
    return s;
}

static i64 count_bad_diag(i64 n, const i32 *rp, const i32 *col, const double *val)
{
    i64 bad = 0;
    for (i64 i = 0; i < n; i++) {
        double aii = 0.0;
        for (i64 k = rp[i]; k < rp[i + 1]; k++)
            if (col[k] == i) aii = val[k];
        if (aii == 0.0) bad++;
    }
    return bad;
}

i64 orc_symgs(i64 n, const i32 *rp, const i32 *col, const double *val, const double *r, double *x,
              const i32 *order)
{
    i64 bad = count_bad_diag(n, rp, col, val);
    if (bad) return bad;
    for (i64 t = 0; t < n; t++) {
        i64 i = order ? order[t] : t;
        double aii, s = row_offdiag(rp, col, val, x, i, &aii);
        x[i] = (r[i] - s) / aii;
    }
    for (i64 t = n - 1; t >= 0; t--) {
        i64 i = order ? order[t] : t;
        double aii, s = row_offdiag(rp, col, val, x, i, &aii);
        x[i] = (r[i] - s) / aii;
    }
    return 0;
}

/* One V-cycle x = M r from x = 0 on level `l` of `nlev` levels.  Level l
 * has n[l] rows, CSR arrays rp[l], col[l], val[l] and sweep order ord[l];
 * f2c[l] (l < nlev - 1) lists, for each row of level l + 1, the row of
 * level l it sits on. */
static void mg_level(int l, int nlev, const i64 *n, const i32 *const *rp, const i32 *const *col,
                     const double *const *val, const i32 *const *ord, const i32 *const *f2c, const double *r,
                     double *x)
{
    const i64 nf = n[l];
    for (i64 i = 0; i < nf; i++) x[i] = 0.0;
    orc_symgs(nf, rp[l], col[l], val[l], r, x, ord[l]);
    if (l == nlev - 1) return;
    const i64 nc = n[l + 1];
    double *ax = (double *)malloc(sizeof(double) * (size_t)(nf > 0 ? nf : 1));
    double *rc = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    double *xc = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    spmv_rows(nf, rp[l], col[l], val[l], x, ax);
    for (i64 i = 0; i < nc; i++) rc[i] = r[f2c[l][i]] - ax[f2c[l][i]];
    mg_level(l + 1, nlev, n, rp, col, val, ord, f2c, rc, xc);
    for (i64 i = 0; i < nc; i++) x[f2c[l][i]] = x[f2c[l][i]] + xc[i];
    orc_symgs(nf, rp[l], col[l], val[l], r, x, ord[l]);
    free(ax);
    free(rc);
    free(xc);
}

void orc_mg(int nlev, const i64 *n, const i32 *const *rp, const i32 *const *col, const double *const *val,
            const i32 *const *ord, const i32 *const *f2c, const double *r, double *x)
{
    mg_level(0, nlev, n, rp, col, val, ord, f2c, r, x);
}

/* PCG with the V-cycle as preconditioner (HPCG's CG), textbook form:
 *   r = b - A x0; loop: z = M r; rho = r.z; p = z (first) or z + (rho /
 *   rho_prev) p; q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q;
 *   stop when ||r|| <= tol ||r0||.
 * Status as orc_cg, plus 3 = a zero or missing diagonal on some level. */
int orc_pcg_mg(int nlev, const i64 *n, const i32 *const *rp, const i32 *const *col, const double *const *val,
               const i32 *const *ord, const i32 *const *f2c, const double *b, double *x, double tol, i64 maxit,
               i64 *iters_out, double *relres_out)
{
    const i64 nn = n[0];
    size_t sz = sizeof(double) * (size_t)(nn > 0 ? nn : 1);
    double *r = (double *)malloc(sz), *z = (double *)malloc(sz), *p = (double *)malloc(sz);
    double *q = (double *)malloc(sz);
    int status = 1;
    i64 it = 0;
    double relres = 1.0, rho = 0.0;
    for (int l = 0; l < nlev; l++)
        if (count_bad_diag(n[l], rp[l], col[l], val[l])) status = 3;
    if (status == 3) goto out;
    spmv_rows(nn, rp[0], col[0], val[0], x, q);
    for (i64 i = 0; i < nn; i++) r[i] = b[i] - q[i];
    double nr0 = sqrt(dot_lr(nn, r, r));
    if (nr0 == 0.0) {
        status = 0;
        relres = 0.0;
        goto out;
    }
    if (!isfinite(nr0)) {
        status = 2;
        goto out;
    }
    while (it < maxit) {
        mg_level(0, nlev, n, rp, col, val, ord, f2c, r, z);
        double rho1 = dot_lr(nn, r, z);
        if (it == 0) {
            for (i64 i = 0; i < nn; i++) p[i] = z[i];
        } else {
            double beta = rho1 / rho;
            for (i64 i = 0; i < nn; i++) p[i] = z[i] + beta * p[i];
        }
        rho = rho1;
        spmv_rows(nn, rp[0], col[0], val[0], p, q);
        it++;
        double pq = dot_lr(nn, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = 2;
            break;
        }
        double alpha = rho / pq;
        for (i64 i = 0; i < nn; i++) x[i] = x[i] + alpha * p[i];
        for (i64 i = 0; i < nn; i++) r[i] = r[i] - alpha * q[i];
        double nr = sqrt(dot_lr(nn, r, r));
        if (!isfinite(nr)) {
            status = 2;
            break;
        }
        relres = nr / nr0;
        if (nr <= tol * nr0) {
            status = 0;
            break;
        }
    }
out:
    free(r);
    free(z);
    free(p);
    free(q);
    *iters_out = it;
    *relres_out = relres;
    return status;
}
