/* The C oracle under the sanitizer build: every function on small random
 * tensors, the all-cores loop against the plain one bit for bit (all rows and
 * listed rows), and the rejected arguments.  Exit status 0 = all held. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_mttkrp(int, const int64_t *, int64_t, const int32_t *, const double *, const double *const *, int,
               int, double *);
int orc_lpt(int64_t, const int64_t *, int32_t, int32_t *, int64_t *);
int orc_bucket_rows(int, const int64_t *, int64_t, const int32_t *, int, int64_t *, int64_t *);
int orc_mttkrp_bucketed(int, const int64_t *, int64_t, const int32_t *, const double *, const double *const *,
                        int, int, const int64_t *, const int64_t *, const int64_t *, int64_t, int, double *);

static uint64_t st = 88172645463325252ull;
static uint64_t rnd(void) {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return st;
}

int main(void) {
    int fails = 0;
    const int64_t dims[4] = {17, 9, 30, 4};
    const int N = 4, R = 5;
    const int64_t nnz = 2000;
    int32_t *idx = malloc(sizeof(int32_t) * N * nnz);
    double *val = malloc(sizeof(double) * nnz);
    double *fac[4];
    for (int w = 0; w < N; ++w) {
        fac[w] = malloc(sizeof(double) * dims[w] * R);
        for (int64_t i = 0; i < dims[w] * R; ++i) fac[w][i] = (double)(rnd() % 1000) / 500.0 - 1.0;
        for (int64_t e = 0; e < nnz; ++e) {
            uint64_t u = rnd() % (uint64_t)(dims[w] * dims[w]);
            idx[w * nnz + e] = (int32_t)(dims[w] - 1 - (int64_t)(u / (uint64_t)dims[w]) % dims[w]);
        }
    }
    for (int64_t e = 0; e < nnz; ++e) val[e] = (double)(rnd() % 997) / 997.0;
    for (int d = 0; d < N; ++d) {
        double *a = malloc(sizeof(double) * dims[d] * R), *b = malloc(sizeof(double) * dims[d] * R);
        int64_t *rowptr = malloc(sizeof(int64_t) * (dims[d] + 1)), *perm = malloc(sizeof(int64_t) * nnz);
        fails += orc_mttkrp(N, dims, nnz, idx, val, (const double *const *)fac, R, d, a) != 0;
        fails += orc_bucket_rows(N, dims, nnz, idx, d, rowptr, perm) != 0;
        fails += orc_mttkrp_bucketed(N, dims, nnz, idx, val, (const double *const *)fac, R, d, rowptr, perm, NULL,
                                     0, 3, b) != 0;
        fails += memcmp(a, b, sizeof(double) * dims[d] * R) != 0;
        int64_t rows[3] = {dims[d] - 1, 0, dims[d] / 2};
        fails += orc_mttkrp_bucketed(N, dims, nnz, idx, val, (const double *const *)fac, R, d, rowptr, perm, rows,
                                     3, 2, b) != 0;
        for (int k = 0; k < 3; ++k) fails += memcmp(b + k * R, a + rows[k] * R, sizeof(double) * R) != 0;
        int64_t badrow[1] = {dims[d]};
        fails += orc_mttkrp_bucketed(N, dims, nnz, idx, val, (const double *const *)fac, R, d, rowptr, perm, badrow,
                                     1, 2, b) != -1;
        free(a);
        free(b);
        free(rowptr);
        free(perm);
    }
    int64_t sizes[5] = {3, 3, 2, 2, 2}, loads[2];
    int32_t part[5];
    fails += orc_lpt(5, sizes, 2, part, loads) != 0;
    fails += (loads[0] > loads[1] ? loads[0] : loads[1]) != 7;
    fails += orc_lpt(5, sizes, 0, part, loads) != -1;
    idx[0] = (int32_t)dims[0];
    double out[17 * 5];
    fails += orc_mttkrp(N, dims, nnz, idx, val, (const double *const *)fac, R, 1, out) != -1;
    fails += orc_mttkrp(N, dims, nnz, idx, val, (const double *const *)fac, R, N, out) != -1;
    for (int w = 0; w < N; ++w) free(fac[w]);
    free(idx);
    free(val);
    if (fails) fprintf(stderr, "%d oracle checks failed\n", fails);
    else printf("oracle checks passed\n");
    return fails ? 1 : 0;
}
