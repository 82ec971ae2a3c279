/* Driver of the C oracle built with the address and undefined-behaviour
 * sanitizers: random CSR pairs through the count, fill and adjoint
 * functions, and random graphs through the relabelling and the triangle
 * count. Exit code 0 when every call returns consistent sizes. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_csr_check(int32_t nrows, int32_t ncols, const int32_t *rp, const int32_t *ci);
int64_t oracle_spgemm_count(int32_t m, const int32_t *arp, const int32_t *aci, int32_t n, const int32_t *brp,
                            const int32_t *bci, const int32_t *rows, int32_t nr, int64_t *crp, int nthreads);
void oracle_spgemm_fill(int32_t m, const int32_t *arp, const int32_t *aci, const double *aval, int32_t n,
                        const int32_t *brp, const int32_t *bci, const double *bval, const int32_t *rows, int32_t nr,
                        const int64_t *crp, int32_t *cci, double *cval, double *cabs, int nthreads);
int64_t oracle_tc_lower(int32_t nv, const int32_t *grp, const int32_t *gci, int32_t *perm, int32_t *lrp,
                        int32_t *lci);
int64_t oracle_tc_count(int32_t nv, const int32_t *lrp, const int32_t *lci, const int32_t *rows, int32_t nr,
                        int64_t *counts, int nthreads);
int oracle_spgemm_backward(int32_t m, const int32_t *arp, const int32_t *aci, const double *aval, int32_t kb,
                           int32_t n, const int32_t *brp, const int32_t *bci, const double *bval, const int32_t *wrp,
                           const int32_t *wci, const double *wval, double *dA, double *dB, double *dA_abs,
                           double *dB_abs);

static uint64_t state = 88172645463325252ull;
static double urand(void)
{
    state ^= state << 13; state ^= state >> 7; state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0;
}

/* random CSR: rows x cols, density d; arrays malloc'd */
static int64_t make_csr(int32_t rows, int32_t cols, double d, int32_t **rp, int32_t **ci, double **v)
{
    *rp = malloc(sizeof(int32_t) * (size_t)(rows + 1));
    int64_t cap = (int64_t)rows * cols + 1;
    *ci = malloc(sizeof(int32_t) * (size_t)cap);
    *v = malloc(sizeof(double) * (size_t)cap);
    int64_t nnz = 0;
    (*rp)[0] = 0;
    for (int32_t i = 0; i < rows; ++i) {
        for (int32_t j = 0; j < cols; ++j)
            if (urand() < d) { (*ci)[nnz] = j; (*v)[nnz] = urand() - 0.5; ++nnz; }
        (*rp)[i + 1] = (int32_t)nnz;
    }
    return nnz;
}

int main(void)
{
    int fails = 0;
    for (int it = 0; it < 200; ++it) {
        int32_t m = (int32_t)(urand() * 60), k = (int32_t)(urand() * 60) + 1, n = (int32_t)(urand() * 60) + 1;
        int32_t *arp, *aci, *brp, *bci;
        double *av, *bv;
        make_csr(m, k, urand() * 0.3, &arp, &aci, &av);
        make_csr(k, n, urand() * 0.3, &brp, &bci, &bv);
        if (oracle_csr_check(m, k, arp, aci) != 0 || oracle_csr_check(k, n, brp, bci) != 0) ++fails;
        int64_t *crp = malloc(sizeof(int64_t) * (size_t)(m + 1));
        int64_t nnzc = oracle_spgemm_count(m, arp, aci, n, brp, bci, NULL, m, crp, 1);
        int32_t *cci = malloc(sizeof(int32_t) * (size_t)(nnzc + 1));
        double *cv = malloc(sizeof(double) * (size_t)(nnzc + 1)), *ca = malloc(sizeof(double) * (size_t)(nnzc + 1));
        oracle_spgemm_fill(m, arp, aci, av, n, brp, bci, bv, NULL, m, crp, cci, cv, ca, 1);
        int32_t *wrp = malloc(sizeof(int32_t) * (size_t)(m + 1));
        for (int32_t i = 0; i <= m; ++i) wrp[i] = (int32_t)crp[i];
        double *dA = malloc(sizeof(double) * (size_t)(arp[m] + 1)), *dB = malloc(sizeof(double) * (size_t)(brp[k] + 1));
        if (oracle_spgemm_backward(m, arp, aci, av, k, n, brp, bci, bv, wrp, cci, cv, dA, dB, NULL, NULL) != 0) ++fails;
        free(arp); free(aci); free(av); free(brp); free(bci); free(bv);
        free(crp); free(cci); free(cv); free(ca); free(wrp); free(dA); free(dB);
    }
    for (int it = 0; it < 100; ++it) {
        int32_t nv = (int32_t)(urand() * 120);
        double p = urand() * 0.2;
        char *adj = calloc((size_t)nv * (size_t)nv + 1, 1);
        for (int32_t i = 0; i < nv; ++i)
            for (int32_t j = i + 1; j < nv; ++j)
                if (urand() < p) adj[(size_t)i * nv + j] = adj[(size_t)j * nv + i] = 1;
        int32_t *grp = malloc(sizeof(int32_t) * (size_t)(nv + 1)), *gci = malloc(sizeof(int32_t) * ((size_t)nv * nv + 1));
        int64_t nnz = 0;
        grp[0] = 0;
        for (int32_t i = 0; i < nv; ++i) {
            for (int32_t j = 0; j < nv; ++j)
                if (adj[(size_t)i * nv + j]) gci[nnz++] = j;
            grp[i + 1] = (int32_t)nnz;
        }
        int32_t *perm = malloc(sizeof(int32_t) * (size_t)(nv + 1)), *lrp = malloc(sizeof(int32_t) * (size_t)(nv + 1));
        int32_t *lci = malloc(sizeof(int32_t) * (size_t)(nnz / 2 + 1));
        int64_t nl = oracle_tc_lower(nv, grp, gci, perm, lrp, lci);
        if (nl != nnz / 2) ++fails;
        int64_t *cnt = malloc(sizeof(int64_t) * (size_t)(nv + 1));
        oracle_tc_count(nv, lrp, lci, NULL, nv, cnt, 1);
        free(adj); free(grp); free(gci); free(perm); free(lrp); free(lci); free(cnt);
    }
    printf("oracle driver: %d failed checks\n", fails);
    return fails == 0 ? 0 : 1;
}
