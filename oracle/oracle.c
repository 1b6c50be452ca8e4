/*
 * FP64 CPU oracle for sparse MTTKRP and Algorithm 1 (tensor partitioning).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -o liboracle.so oracle.c
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

/*
 * spMTTKRP for one output mode, Eq. (1) of Sec. 2.1.4 evaluated nonzero by
 * nonzero as in the elementwise computation of Sec. 2.1.5 (Alg. 2):
 *
 *   out(i, r) = sum over nonzeros e with i_mode(e) = i of
 *               val(e) * prod_{w != mode} Y_w(i_w(e), r)
 *
 * out is I_mode x rank row-major and is overwritten (rows with no nonzero
 * stay zero).  idx is mode-major [nmodes][nnz]; factors[w] is I_w x rank
 * row-major FP64 (factors[mode] is not read).  Returns 0, or -1 on a bad
 * argument or an index outside its mode.
 */
int orc_mttkrp(int nmodes, const int64_t *dims, int64_t nnz, const int32_t *idx,
               const double *val, const double *const *factors, int rank,
               int mode, double *out)
{
    if (nmodes < 1 || mode < 0 || mode >= nmodes || rank < 1 || nnz < 0)
        return -1;
    memset(out, 0, sizeof(double) * (size_t)dims[mode] * (size_t)rank);
    double *ell = (double *)malloc(sizeof(double) * (size_t)rank);
    if (!ell)
        return -1;
    for (int64_t e = 0; e < nnz; ++e) {
        for (int w = 0; w < nmodes; ++w) {
            int32_t c = idx[(int64_t)w * nnz + e];
            if (c < 0 || c >= dims[w]) {
                free(ell);
                return -1;
            }
        }
        for (int r = 0; r < rank; ++r)
            ell[r] = val[e];
        for (int w = 0; w < nmodes; ++w) {
            if (w == mode)
                continue;
            const double *row = factors[w] + (int64_t)idx[(int64_t)w * nnz + e] * rank;
            for (int r = 0; r < rank; ++r)
                ell[r] *= row[r];
        }
        double *o = out + (int64_t)idx[(int64_t)mode * nnz + e] * rank;
        for (int r = 0; r < rank; ++r)
            o[r] += ell[r];
    }
    free(ell);
    return 0;
}

/*
 * Algorithm 1 (Sec. 3.4) as read here: items (vertices, or pieces of a
 * vertex) arrive already ordered by decreasing number of incident
 * hyperedges; each goes to the least filled of the kappa blocks, where
 * "filled" counts hyperedges (nonzeros) and a tie goes to the block with the
 * lowest id.  part[k] receives the block of item k, loads[] the final
 * number of hyperedges per block.  Plain linear scan for the minimum.
 */
int orc_lpt(int64_t nitems, const int64_t *sizes, int32_t kappa, int32_t *part,
            int64_t *loads)
{
    if (kappa < 1 || nitems < 0)
        return -1;
    for (int32_t w = 0; w < kappa; ++w)
        loads[w] = 0;
    for (int64_t k = 0; k < nitems; ++k) {
        int32_t best = 0;
        for (int32_t w = 1; w < kappa; ++w)
            if (loads[w] < loads[best])
                best = w;
        part[k] = best;
        loads[best] += sizes[k];
    }
    return 0;
}

/*
 * The same sum as orc_mttkrp, evaluated on all host cores.  The nonzeros are
 * first bucketed by output row: a stable counting sort gives, for each row i
 * of the mode, its nonzeros in input order (perm[rowptr[i] .. rowptr[i+1])).
 * Each row is then owned by one thread, which adds its nonzeros in that
 * order.  Every output element therefore receives the same terms in the same
 * order as in orc_mttkrp: the result is identical bit for bit, whatever the
 * thread count, with no atomics.
 *
 * orc_bucket_rows fills rowptr [dims[mode] + 1] and perm [nnz] (untimed
 * preparation); orc_mttkrp_bucketed then computes out (overwritten): all
 * I_mode rows when rows is NULL, else only the nrows listed rows, out row k
 * holding row rows[k] (for checks of sampled rows of large tensors).
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 on a bad
 * argument, an index outside its mode or an allocation failure.
 */
int orc_bucket_rows(int nmodes, const int64_t *dims, int64_t nnz, const int32_t *idx,
                    int mode, int64_t *rowptr, int64_t *perm)
{
    if (nmodes < 1 || mode < 0 || mode >= nmodes || nnz < 0)
        return -1;
    const int64_t I = dims[mode];
    const int32_t *c = idx + (int64_t)mode * nnz;
    for (int64_t i = 0; i <= I; ++i)
        rowptr[i] = 0;
    for (int64_t e = 0; e < nnz; ++e) {
        if (c[e] < 0 || c[e] >= I)
            return -1;
        rowptr[c[e] + 1] += 1;
    }
    for (int64_t i = 0; i < I; ++i)
        rowptr[i + 1] += rowptr[i];
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(I > 0 ? I : 1));
    if (!next)
        return -1;
    for (int64_t i = 0; i < I; ++i)
        next[i] = rowptr[i];
    for (int64_t e = 0; e < nnz; ++e)
        perm[next[c[e]]++] = e;
    free(next);
    return 0;
}

int orc_mttkrp_bucketed(int nmodes, const int64_t *dims, int64_t nnz, const int32_t *idx,
                        const double *val, const double *const *factors, int rank, int mode,
                        const int64_t *rowptr, const int64_t *perm, const int64_t *rows,
                        int64_t nrows, int nthreads, double *out)
{
    if (nmodes < 1 || mode < 0 || mode >= nmodes || rank < 1 || nnz < 0)
        return -1;
    for (int w = 0; w < nmodes; ++w) {
        const int32_t *c = idx + (int64_t)w * nnz;
        for (int64_t e = 0; e < nnz; ++e)
            if (c[e] < 0 || c[e] >= dims[w])
                return -1;
    }
    const int64_t I = dims[mode];
    const int64_t nout = rows ? nrows : I;
    if (rows)
        for (int64_t k = 0; k < nrows; ++k)
            if (rows[k] < 0 || rows[k] >= I)
                return -1;
    int bad = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : omp_get_max_threads()) reduction(| : bad)
    {
        double *ell = (double *)malloc(sizeof(double) * (size_t)rank);
        if (!ell)
            bad = 1;
        /* rows in chunks, handed out as threads free up: the Zipf head rows
         * hold a large share of the nonzeros */
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < nout; ++k) {
            const int64_t i = rows ? rows[k] : k;
            double *o = out + k * rank;
            for (int r = 0; r < rank; ++r)
                o[r] = 0.0;
            if (!ell)
                continue;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int64_t e = perm[k];
                for (int r = 0; r < rank; ++r)
                    ell[r] = val[e];
                for (int w = 0; w < nmodes; ++w) {
                    if (w == mode)
                        continue;
                    const double *row = factors[w] + (int64_t)idx[(int64_t)w * nnz + e] * rank;
                    for (int r = 0; r < rank; ++r)
                        ell[r] *= row[r];
                }
                for (int r = 0; r < rank; ++r)
                    o[r] += ell[r];
            }
        }
        free(ell);
    }
    return bad ? -1 : 0;
}

/* Threads an OpenMP parallel region of the oracle uses by default. */
int orc_max_threads(void)
{
    return omp_get_max_threads();
}
