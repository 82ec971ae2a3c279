/*
 * oracle.c -- plain CPU reference for the two-phase SpGEMM hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code, header or table with the HIP
 * library.
 *
 * What it computes (Deveci et al., "Sparse Matrix-Matrix Multiplication on
 * Multilevel Memory Architectures", arXiv 1804.00695):
 *
 *  - C = A*B on CSR, row by row (Sec. 2.1, "Baseline SpGEMM method"): row i
 *    of C is the sum over the stored a_ik of a_ik times row k of B, visited
 *    in the order of Fig. "spgemmexp" (the entries of row i of A in stored
 *    order, each followed by all of row k of B). The two phases of the paper
 *    are kept: a symbolic pass that counts the distinct columns of each row
 *    of C, then a numeric pass that fills column indices and values.
 *    The accumulator is the dense one the paper names as the alternative to
 *    its hash maps (Sec. 3.1, access patterns): one slot per column of B,
 *    stamped with the current row so it never has to be cleared.
 *    Structural entries are kept even when their value sums to 0.0; columns
 *    of each output row are written in ascending order.
 *  - Triangle counting (Sec. 4.1.2): vertices relabelled by descending
 *    degree (ties by ascending id), L = strict lower triangle in the new
 *    labels, t_i = number of j in row i of (L*L) masked by L, T = sum t_i.
 *    Only the pattern is used; there is no output matrix.
 *  - The adjoint of the bilinear map (A, B) -> sum_ij W_ij (A*B)_ij, with W
 *    given on the pattern of C: dA_ik = sum_j W_ij b_kj on the pattern of A
 *    and dB_kj = sum_i a_ik W_ij on the pattern of B. This is not in the
 *    paper; it is the exact derivative of that loss.
 *
 * Floating point: fp64, every product rounded before it is added (the file
 * is compiled with -ffp-contract=off, so no fused multiply-add). Alongside
 * each value the oracle accumulates sum |a||b| over the same terms; a
 * computed value c is accepted against the oracle's c_ref when
 * |c - c_ref| <= tol * that sum.
 *
 * Threads: the count and fill passes run rows in parallel under OpenMP when
 * nthreads > 1 (one private accumulator per thread). Results do not depend
 * on the thread count: every row is computed by exactly one thread in the
 * same order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* CSR checks                                                              */
/* ---------------------------------------------------------------------- */

/* 0 = valid; 1 = row_ptr[0] != 0; 2 = row_ptr decreases; 3 = column out of
 * range; 4 = columns of a row not strictly increasing. */
int oracle_csr_check(int32_t nrows, int32_t ncols, const int32_t *rp, const int32_t *ci)
{
    if (rp[0] != 0) return 1;
    for (int32_t i = 0; i < nrows; ++i) {
        if (rp[i + 1] < rp[i]) return 2;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= ncols) return 3;
            if (p > rp[i] && ci[p] <= ci[p - 1]) return 4;
        }
    }
    return 0;
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    omp_set_num_threads(nthreads > 0 ? nthreads : 1);
#else
    (void)nthreads;
#endif
}

/* ---------------------------------------------------------------------- */
/* Symbolic phase: number of distinct columns in each selected row of C.   */
/* ---------------------------------------------------------------------- */

/* rows == NULL selects all rows 0..m-1 (then nr must equal m); otherwise
 * output entry t describes row rows[t] of C. Writes crp[0..nr] as an
 * exclusive prefix of the counts and returns crp[nr]. */
int64_t oracle_spgemm_count(int32_t m, const int32_t *arp, const int32_t *aci,
                            int32_t n, const int32_t *brp, const int32_t *bci,
                            const int32_t *rows, int32_t nr, int64_t *crp, int nthreads)
{
    (void)m;
    set_threads(nthreads);
    crp[0] = 0;
#pragma omp parallel
    {
        int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        for (int32_t j = 0; j < n; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 256)
        for (int32_t t = 0; t < nr; ++t) {
            int32_t i = rows ? rows[t] : t;
            int64_t cnt = 0;
            for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
                int32_t k = aci[p];
                for (int32_t q = brp[k]; q < brp[k + 1]; ++q) {
                    int32_t j = bci[q];
                    if (mark[j] != t) { mark[j] = t; ++cnt; }
                }
            }
            crp[t + 1] = cnt;
        }
        free(mark);
    }
    for (int32_t t = 0; t < nr; ++t) crp[t + 1] += crp[t];
    return crp[nr];
}

/* ---------------------------------------------------------------------- */
/* Numeric phase: column indices (ascending) and values of selected rows.  */
/* ---------------------------------------------------------------------- */

/* crp must be the result of oracle_spgemm_count for the same rows. aval,
 * bval may be NULL (pattern only; cval/cabs are then not written). cabs may
 * be NULL. */
void oracle_spgemm_fill(int32_t m, const int32_t *arp, const int32_t *aci, const double *aval,
                        int32_t n, const int32_t *brp, const int32_t *bci, const double *bval,
                        const int32_t *rows, int32_t nr, const int64_t *crp,
                        int32_t *cci, double *cval, double *cabs, int nthreads)
{
    (void)m;
    const int with_values = (aval != NULL && bval != NULL && cval != NULL);
    set_threads(nthreads);
#pragma omp parallel
    {
        size_t nn = (size_t)(n > 0 ? n : 1);
        int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * nn);
        int32_t *list = (int32_t *)malloc(sizeof(int32_t) * nn);
        double *spa = (double *)malloc(sizeof(double) * nn);
        double *sabs = (double *)malloc(sizeof(double) * nn);
        for (int32_t j = 0; j < n; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 256)
        for (int32_t t = 0; t < nr; ++t) {
            int32_t i = rows ? rows[t] : t;
            int32_t len = 0;
            for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
                int32_t k = aci[p];
                double a = with_values ? aval[p] : 0.0;
                for (int32_t q = brp[k]; q < brp[k + 1]; ++q) {
                    int32_t j = bci[q];
                    if (mark[j] != t) {
                        mark[j] = t;
                        spa[j] = 0.0;
                        sabs[j] = 0.0;
                        list[len++] = j;
                    }
                    if (with_values) {
                        double b = bval[q];
                        spa[j] += a * b;
                        sabs[j] += fabs(a) * fabs(b);
                    }
                }
            }
            qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
            int64_t base = crp[t];
            for (int32_t s = 0; s < len; ++s) {
                int32_t j = list[s];
                cci[base + s] = j;
                if (with_values) {
                    cval[base + s] = spa[j];
                    if (cabs) cabs[base + s] = sabs[j];
                }
            }
        }
        free(mark); free(list); free(spa); free(sabs);
    }
}

/* ---------------------------------------------------------------------- */
/* Triangle counting (Sec. 4.1.2)                                          */
/* ---------------------------------------------------------------------- */

static const int32_t *g_deg_for_sort;

static int cmp_degree_desc(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    int32_t da = g_deg_for_sort[a], db = g_deg_for_sort[b];
    if (da != db) return (da < db) - (da > db);   /* larger degree first */
    return (a > b) - (a < b);                     /* then smaller id */
}

/* Relabel the vertices of the symmetric pattern G (no self loops) by
 * descending degree, ties by ascending original id, and build L, the strict
 * lower triangle in the new labels: row i holds the new labels j < i of its
 * neighbours, ascending. perm[new] = old. lrp has nv+1 entries; lci has
 * nnz(G)/2 entries. Returns nnz(L). Not thread safe (qsort comparator). */
int64_t oracle_tc_lower(int32_t nv, const int32_t *grp, const int32_t *gci,
                        int32_t *perm, int32_t *lrp, int32_t *lci)
{
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
    int32_t *inv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
    for (int32_t v = 0; v < nv; ++v) { deg[v] = grp[v + 1] - grp[v]; perm[v] = v; }
    g_deg_for_sort = deg;
    qsort(perm, (size_t)nv, sizeof(int32_t), cmp_degree_desc);
    for (int32_t i = 0; i < nv; ++i) inv[perm[i]] = i;
    int64_t nnz = 0;
    lrp[0] = 0;
    for (int32_t i = 0; i < nv; ++i) {
        int32_t v = perm[i];
        int64_t start = nnz;
        for (int32_t p = grp[v]; p < grp[v + 1]; ++p) {
            int32_t j = inv[gci[p]];
            if (j < i) lci[nnz++] = j;
        }
        qsort(lci + start, (size_t)(nnz - start), sizeof(int32_t), cmp_i32);
        lrp[i + 1] = (int32_t)nnz;
    }
    free(deg); free(inv);
    return nnz;
}

/* t_i = sum over k in row i of L of |row k of L intersected with row i of L|,
 * which is row i of (L*L) masked by L, summed. rows == NULL selects all
 * rows (nr == nv). counts[t] receives t_{rows[t]}; returns the sum. */
int64_t oracle_tc_count(int32_t nv, const int32_t *lrp, const int32_t *lci,
                        const int32_t *rows, int32_t nr, int64_t *counts, int nthreads)
{
    int64_t total = 0;
    set_threads(nthreads);
#pragma omp parallel reduction(+ : total)
    {
        int32_t *flag = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
        for (int32_t j = 0; j < nv; ++j) flag[j] = -1;
#pragma omp for schedule(dynamic, 256)
        for (int32_t t = 0; t < nr; ++t) {
            int32_t i = rows ? rows[t] : t;
            for (int32_t p = lrp[i]; p < lrp[i + 1]; ++p) flag[lci[p]] = t;
            int64_t c = 0;
            for (int32_t p = lrp[i]; p < lrp[i + 1]; ++p) {
                int32_t k = lci[p];
                for (int32_t q = lrp[k]; q < lrp[k + 1]; ++q)
                    if (flag[lci[q]] == t) ++c;
            }
            counts[t] = c;
            total += c;
        }
        free(flag);
    }
    return total;
}

/* ---------------------------------------------------------------------- */
/* Adjoint of loss = sum_ij W_ij (A*B)_ij with W stored on the pattern of C */
/* ---------------------------------------------------------------------- */

/* B has kb rows and n columns. Writes dA (nnz(A)) and dB (nnz(B)); dA_abs / dB_abs (nullable) receive the
 * sums of |W_ij||b_kj| and |a_ik||W_ij| over the same terms. Returns 0, or 1
 * when W lacks a column that row i of A*B reaches. Sequential, rows in
 * ascending order, terms in the same order as the forward product. */
int oracle_spgemm_backward(int32_t m, const int32_t *arp, const int32_t *aci, const double *aval,
                           int32_t kb, int32_t n, const int32_t *brp, const int32_t *bci, const double *bval,
                           const int32_t *wrp, const int32_t *wci, const double *wval,
                           double *dA, double *dB, double *dA_abs, double *dB_abs)
{
    int64_t nnzA = arp[m], nnzB = brp[kb];
    for (int64_t p = 0; p < nnzA; ++p) { dA[p] = 0.0; if (dA_abs) dA_abs[p] = 0.0; }
    for (int64_t q = 0; q < nnzB; ++q) { dB[q] = 0.0; if (dB_abs) dB_abs[q] = 0.0; }
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * nn);
    double *w = (double *)malloc(sizeof(double) * nn);
    for (int32_t j = 0; j < n; ++j) mark[j] = -1;
    int err = 0;
    for (int32_t i = 0; i < m && !err; ++i) {
        for (int32_t r = wrp[i]; r < wrp[i + 1]; ++r) { mark[wci[r]] = i; w[wci[r]] = wval[r]; }
        for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
            int32_t k = aci[p];
            double a = aval[p];
            for (int32_t q = brp[k]; q < brp[k + 1]; ++q) {
                int32_t j = bci[q];
                if (mark[j] != i) { err = 1; break; }
                dA[p] += w[j] * bval[q];
                dB[q] += a * w[j];
                if (dA_abs) dA_abs[p] += fabs(w[j]) * fabs(bval[q]);
                if (dB_abs) dB_abs[q] += fabs(a) * fabs(w[j]);
            }
            if (err) break;
        }
    }
    free(mark); free(w);
    return err;
}
