/*
 * FP64 CPU oracle for sparse MTTKRP and Algorithm 1 (tensor partitioning).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * Build: gcc -O2 -shared -fPIC -o liboracle.so oracle.c
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

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
