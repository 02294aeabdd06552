/* Exercises every oracle routine on small hand-made and pseudo-random
 * matrices (empty rows, rectangular, 1x1, empty) so that a sanitizer build
 * can check the oracle for memory and undefined-behaviour errors. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef int32_t i32;
typedef int64_t i64;

int orc_csr_validate(i64, i64, i64, const i32 *, const i32 *);
void orc_spmv_csr(i64, const i32 *, const i32 *, const double *, const double *, double *);
void orc_spmv_csr_ref(i64, const i32 *, const i32 *, const double *, const double *, double *, double *);
void orc_csr_to_coo(i64, const i32 *, i32 *);
int orc_coo_to_csr(i64, i64, i64, const i32 *, const i32 *, const double *, i32 *, i32 *, double *);
void orc_spmv_coo(i64, i64, const i32 *, const i32 *, const double *, const double *, double *);
i64 orc_dia_count(i64, i64, const i32 *, const i32 *, i32 *);
void orc_csr_to_dia(i64, i64, const i32 *, const i32 *, const double *, i64, const i32 *, double *);
i64 orc_dia_to_csr(i64, i64, i64, const i32 *, const double *, i32 *, i32 *, double *);
void orc_spmv_dia(i64, i64, i64, const i32 *, const double *, const double *, double *);
i32 orc_ell_width(i64, const i32 *);
void orc_csr_to_ell_part(i64, const i32 *, const i32 *, const double *, i32, i32 *, double *);
i64 orc_ell_to_csr(i64, i32, const i32 *, const double *, i32 *, i32 *, double *);
void orc_spmv_ell(i64, i32, const i32 *, const double *, const double *, double *);
i32 orc_hyb_width(i64, const i32 *);
i64 orc_hyb_coo_count(i64, const i32 *, i32);
void orc_csr_to_hyb(i64, const i32 *, const i32 *, const double *, i32, i32 *, double *, i32 *, i32 *, double *);
i64 orc_hyb_to_csr(i64, i32, const i32 *, const double *, i64, const i32 *, const i32 *, const double *, i32 *,
                   i32 *, double *);
i64 orc_hdc_true_diags(i64, i64, const i32 *, const i32 *, double, i32 *);
i64 orc_csr_to_hdc(i64, i64, const i32 *, const i32 *, const double *, i64, const i32 *, double *, i32 *, i32 *,
                   double *);
i64 orc_hdc_to_csr(i64, i64, i64, const i32 *, const double *, const i32 *, const i32 *, const double *, i32 *,
                   i32 *, double *);
void orc_cast_f32(i64, const double *, float *);
void orc_cast_bf16(i64, const double *, uint16_t *);
void orc_bf16_to_f64(i64, const uint16_t *, double *);
void orc_row_stats(i64, const i32 *, i64 *);
int orc_cg(i64, const i32 *, const i32 *, const double *, const double *, double *, double, i64, i64 *, double *);
double orc_true_relres(i64, const i32 *, const i32 *, const double *, const double *, const double *);

static uint64_t st = 88172645463325252ull;
static uint64_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }

static void *xm(size_t n) { return malloc(n ? n : 1); }

static void run(i64 n, i64 m, int dens_pct) {
    i32 *rp = xm(sizeof(i32) * (n + 1));
    i32 *col = xm(sizeof(i32) * (size_t)(n * m));
    double *val = xm(sizeof(double) * (size_t)(n * m));
    i64 nz = 0;
    rp[0] = 0;
    for (i64 i = 0; i < n; i++) {
        for (i64 j = 0; j < m; j++)
            if ((int)(rnd() % 100) < dens_pct) {
                col[nz] = (i32)j;
                val[nz] = 1.0 + (double)(rnd() % 1000) / 7.0;
                nz++;
            }
        rp[i + 1] = (i32)nz;
    }
    if (orc_csr_validate(n, m, nz, rp, col) != 0) abort();
    double *x = xm(sizeof(double) * m), *y = xm(sizeof(double) * n), *y2 = xm(sizeof(double) * n);
    double *s = xm(sizeof(double) * n);
    for (i64 j = 0; j < m; j++) x[j] = (double)(rnd() % 100) / 13.0;
    orc_spmv_csr(n, rp, col, val, x, y);
    orc_spmv_csr_ref(n, rp, col, val, x, y2, s);
    i32 *row = xm(sizeof(i32) * nz);
    orc_csr_to_coo(n, rp, row);
    i32 *rp2 = xm(sizeof(i32) * (n + 1)), *c2 = xm(sizeof(i32) * nz);
    double *v2 = xm(sizeof(double) * nz);
    if (orc_coo_to_csr(n, m, nz, row, col, val, rp2, c2, v2) != 0) abort();
    orc_spmv_coo(n, nz, row, col, val, x, y2);
    i64 nd = orc_dia_count(n, m, rp, col, NULL);
    i32 *offs = xm(sizeof(i32) * nd);
    orc_dia_count(n, m, rp, col, offs);
    double *dv = xm(sizeof(double) * (size_t)(nd * n));
    orc_csr_to_dia(n, m, rp, col, val, nd, offs, dv);
    if (orc_dia_to_csr(n, m, nd, offs, dv, rp2, c2, v2) != nz) abort();
    orc_spmv_dia(n, m, nd, offs, dv, x, y2);
    i32 K = orc_ell_width(n, rp);
    i32 *ec = xm(sizeof(i32) * (size_t)(K * n));
    double *ev = xm(sizeof(double) * (size_t)(K * n));
    orc_csr_to_ell_part(n, rp, col, val, K, ec, ev);
    if (orc_ell_to_csr(n, K, ec, ev, rp2, c2, v2) != nz) abort();
    orc_spmv_ell(n, K, ec, ev, x, y2);
    i32 Kh = orc_hyb_width(n, rp);
    i64 nco = orc_hyb_coo_count(n, rp, Kh);
    i32 *hc = xm(sizeof(i32) * (size_t)(Kh * n)), *cr = xm(sizeof(i32) * nco), *cc = xm(sizeof(i32) * nco);
    double *hv = xm(sizeof(double) * (size_t)(Kh * n)), *cv = xm(sizeof(double) * nco);
    orc_csr_to_hyb(n, rp, col, val, Kh, hc, hv, cr, cc, cv);
    if (orc_hyb_to_csr(n, Kh, hc, hv, nco, cr, cc, cv, rp2, c2, v2) != nz) abort();
    i64 nt = orc_hdc_true_diags(n, m, rp, col, 0.5, NULL);
    i32 *to = xm(sizeof(i32) * nt);
    orc_hdc_true_diags(n, m, rp, col, 0.5, to);
    double *hd = xm(sizeof(double) * (size_t)(nt * n));
    i32 *hrp = xm(sizeof(i32) * (n + 1));
    i64 nr = orc_csr_to_hdc(n, m, rp, col, val, nt, to, hd, hrp, NULL, NULL);
    i32 *hcol = xm(sizeof(i32) * nr);
    double *hval = xm(sizeof(double) * nr);
    orc_csr_to_hdc(n, m, rp, col, val, nt, to, hd, hrp, hcol, hval);
    if (orc_hdc_to_csr(n, m, nt, to, hd, hrp, hcol, hval, rp2, c2, v2) != nz) abort();
    float *f = xm(sizeof(float) * nz);
    uint16_t *h = xm(sizeof(uint16_t) * nz);
    orc_cast_f32(nz, val, f);
    orc_cast_bf16(nz, val, h);
    orc_bf16_to_f64(nz, h, v2);
    i64 stats[38];
    orc_row_stats(n, rp, stats);
    if (n == m) {
        /* SPD by diagonal dominance: add a big diagonal via a fresh matrix */
        i64 it;
        double rr;
        double *b = xm(sizeof(double) * n), *xs = xm(sizeof(double) * n);
        for (i64 i = 0; i < n; i++) { b[i] = 1.0; xs[i] = 0.0; }
        orc_cg(n, rp, col, val, b, xs, 1e-8, 20, &it, &rr);
        orc_true_relres(n, rp, col, val, b, xs);
        free(b); free(xs);
    }
    free(rp); free(col); free(val); free(x); free(y); free(y2); free(s); free(row); free(rp2); free(c2); free(v2);
    free(offs); free(dv); free(ec); free(ev); free(hc); free(cr); free(cc); free(hv); free(cv); free(to); free(hd);
    free(hrp); free(hcol); free(hval); free(f); free(h);
}

int main(void) {
    int cases[][3] = {{1, 1, 100}, {0, 0, 50}, {7, 0, 50}, {0, 5, 50}, {5, 9, 0}, {13, 13, 30},
                      {40, 17, 20}, {17, 40, 60}, {64, 64, 5}, {33, 33, 100}};
    for (unsigned k = 0; k < sizeof cases / sizeof cases[0]; k++) run(cases[k][0], cases[k][1], cases[k][2]);
    puts("oracle driver ok");
    return 0;
}
