/* The C oracle (oracle/mttkrp_ref.c) on random small tensors, meant to be
 * built with AddressSanitizer and UBSan (tests/test_host_sanitized.py).
 * Besides memory safety it checks two closed forms: with all-ones factors,
 * MTTKRP along mode d is the per-row sum of the values (each rank column);
 * the loss equals the sum of the squared residuals it returns.  Exit status 0
 * when every check passes. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_mttkrp(int order, const int64_t *dims, int64_t nnz, const int32_t *idx, const double *val, int mode,
                   int R, const double *const *A, double *out);
double oracle_cp_loss(int order, int64_t nnz, const int32_t *idx, const double *val, int R,
                      const double *const *A, double *resid);

static uint64_t st = 88172645463325252ull;
static uint64_t next(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }

int main(void)
{
    int fails = 0;
    for (int c = 0; c < 60; ++c) {
        const int order = 2 + c % 4, R = 1 + (c * 7) % 33;
        const int64_t nnz = (c % 5 == 0) ? 0 : (int64_t)(next() % 400) + 1;
        int64_t dims[5];
        for (int w = 0; w < order; ++w) dims[w] = 1 + (int64_t)(next() % 23);
        int32_t *idx = malloc(sizeof(int32_t) * (size_t)(order * nnz + 1));
        double *val = malloc(sizeof(double) * (size_t)(nnz + 1));
        double *resid = malloc(sizeof(double) * (size_t)(nnz + 1));
        for (int64_t k = 0; k < nnz; ++k) {
            for (int w = 0; w < order; ++w) idx[w * nnz + k] = (int32_t)(next() % (uint64_t)dims[w]);
            val[k] = (double)(next() % 1000) / 250.0 - 2.0;
        }
        double *A[5];
        for (int w = 0; w < order; ++w) {
            A[w] = malloc(sizeof(double) * (size_t)(dims[w] * R));
            for (int64_t i = 0; i < dims[w] * R; ++i) A[w][i] = 1.0;
        }
        for (int d = 0; d < order; ++d) {
            double *out = malloc(sizeof(double) * (size_t)(dims[d] * R));
            double *rowsum = calloc((size_t)dims[d], sizeof(double));
            oracle_mttkrp(order, dims, nnz, idx, val, d, R, (const double *const *)A, out);
            for (int64_t k = 0; k < nnz; ++k) rowsum[idx[d * nnz + k]] += val[k];
            for (int64_t i = 0; i < dims[d]; ++i)
                for (int r = 0; r < R; ++r)
                    if (fabs(out[i * R + r] - rowsum[i]) > 1e-12 * (1.0 + fabs(rowsum[i]))) {
                        if (fails++ < 10) printf("case %d mode %d row %lld col %d\n", c, d, (long long)i, r);
                    }
            free(out);
            free(rowsum);
        }
        for (int w = 0; w < order; ++w)
            for (int64_t i = 0; i < dims[w] * R; ++i) A[w][i] = (double)(next() % 100) / 50.0 - 1.0;
        const double loss = oracle_cp_loss(order, nnz, idx, val, R, (const double *const *)A, resid);
        double s = 0.0;
        for (int64_t k = 0; k < nnz; ++k) s += resid[k] * resid[k];
        if (fabs(loss - s) > 1e-12 * (1.0 + fabs(s))) {
            if (fails++ < 10) printf("case %d loss %g vs %g\n", c, loss, s);
        }
        for (int w = 0; w < order; ++w) free(A[w]);
        free(idx);
        free(val);
        free(resid);
    }
    printf("60 cases, %d failures\n", fails);
    return fails ? 1 : 0;
}
