// CP-ALS dense step on the device, FP64 for every R x R quantity:
// Grams G_w = Y_w^T Y_w, the normal matrix V = Hadamard of the other Grams,
// its Cholesky factorisation and inverse, Y_d = M_d V^-1, column norms
// lambda and the CP fit.  Reductions are two-stage (block partials, then
// one ordered pass), so results do not depend on scheduling.
#include <algorithm>

#include "kernels.hpp"

// Y = M V^-1 on the FP64 matrix cores (1) or with V^-1 in LDS (0); the
// instruction's lane layout used below was measured on the device.
#ifndef SPT_SOLVE_MFMA
#define SPT_SOLVE_MFMA 1
#endif
// Grams of the caller's factors at the start of a sweep on the FP64 matrix
// cores (rank 8: the LDS kernel)
#ifndef SPT_GRAM_MFMA
#define SPT_GRAM_MFMA 1
#endif

namespace spt {

namespace {

constexpr int kGramRows = 32;

template <int R>
__global__ __launch_bounds__(256) void gram_partial_kernel(const float* __restrict__ Y, int64_t rows,
                                                           double* __restrict__ partial) {
    constexpr int E = R * R;
    constexpr int PER = (E + 255) / 256;
    __shared__ float tile[kGramRows][R];
    const int tid = threadIdx.x;
    const int64_t chunk = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = std::min<int64_t>(rows, (int64_t)blockIdx.x * chunk);
    const int64_t r1 = std::min<int64_t>(rows, r0 + chunk);
    double acc[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) acc[k] = 0.0;
    for (int64_t base = r0; base < r1; base += kGramRows) {
        const int nr = (int)std::min<int64_t>(kGramRows, r1 - base);
        for (int i = tid; i < kGramRows * R; i += 256) {
            const int rr = i / R, cc = i % R;
            tile[rr][cc] = rr < nr ? Y[(base + rr) * R + cc] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            if (e < E) {
                const int r = e / R, c = e % R;
                double s = 0.0;
                for (int i = 0; i < nr; ++i) s += (double)tile[i][r] * (double)tile[i][c];
                acc[k] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = tid + 256 * k;
        if (e < E) partial[(int64_t)blockIdx.x * E + e] = acc[k];
    }
}

// out[e] = sum over b of partial[b][e] for e < E.  Each entry is summed by
// 8 chains (b = c, c+8, ...), each with 4 interleaved accumulators, and the
// chains are combined in a fixed order.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ partial,
                                                              int nblocks, int E,
                                                              double* __restrict__ out) {
    __shared__ double red[8][32];
    const int tid = threadIdx.x;
    const int el = tid % 32, c = tid / 32;
    const int e = blockIdx.x * 32 + el;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (e < E) {
        int b = c;
        for (; b + 24 < nblocks; b += 32) {
            s0 += partial[(int64_t)b * E + e];
            s1 += partial[(int64_t)(b + 8) * E + e];
            s2 += partial[(int64_t)(b + 16) * E + e];
            s3 += partial[(int64_t)(b + 24) * E + e];
        }
        for (; b < nblocks; b += 8) s0 += partial[(int64_t)b * E + e];
    }
    red[c][el] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (tid < 32 && e < E) {
        double t = 0.0;
        for (int k = 0; k < 8; ++k) t += red[k][tid];
        out[e] = t;
    }
}

// V = Hadamard product of the other modes' Grams, plus `ridge` on the diagonal.
template <int R>
__device__ void build_normal(double (*A)[R + 1], const double* __restrict__ grams, int nmodes,
                             int mode, double ridge) {
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
        const int r = e / R, c = e % R;
        double v = 1.0;
        for (int w = 0; w < nmodes; ++w)
            if (w != mode) v *= grams[(int64_t)w * R * R + e];
        A[r][c] = v + (r == c ? ridge : 0.0);
    }
}

// Right-looking Cholesky of A in place (lower triangle), all threads of the
// block; returns false if a pivot is not positive.
template <int R>
__device__ bool cholesky(double (*A)[R + 1]) {
    __shared__ int ok;
    const int tid = threadIdx.x;
    if (tid == 0) ok = 1;
    __syncthreads();
    for (int j = 0; j < R; ++j) {
        if (tid == 0) {
            double d = A[j][j];
            if (!(d > 0.0)) {
                ok = 0;
                d = 1.0;
            }
            A[j][j] = sqrt(d);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < R; i += blockDim.x) A[i][j] /= A[j][j];
        __syncthreads();
        const int m = R - j - 1;
        for (int e = tid; e < m * m; e += blockDim.x) {
            const int i = j + 1 + e / m, k = j + 1 + e % m;
            if (k <= i) A[i][k] -= A[i][j] * A[k][j];
        }
        __syncthreads();
    }
    return ok != 0;
}

// In-place Gauss-Jordan inverse of the SPD matrix in A (no pivoting: the
// pivots are the Schur complements, positive for an SPD matrix).
template <int R>
__device__ void gauss_jordan_inverse(double (*A)[R + 1]) {
    __shared__ double colk[R];
    __shared__ double piv;
    const int tid = threadIdx.x;
    for (int k = 0; k < R; ++k) {
        if (tid < R) colk[tid] = A[tid][k];
        if (tid == 0) piv = A[k][k];
        __syncthreads();
        for (int c = tid; c < R; c += blockDim.x) A[k][c] = (c == k ? 1.0 : A[k][c]) / piv;
        __syncthreads();
        for (int e = tid; e < R * R; e += blockDim.x) {
            const int i = e / R, c = e % R;
            if (i != k) A[i][c] = (c == k ? 0.0 : A[i][c]) - colk[i] * A[k][c];
        }
        __syncthreads();
    }
}

template <int R>
__global__ __launch_bounds__(256) void normal_inverse_kernel(const double* __restrict__ grams,
                                                              int nmodes, int mode,
                                                              double* __restrict__ Vinv,
                                                              int32_t* __restrict__ status) {
    __shared__ double A[R][R + 1];
    __shared__ double ridge;
    const int tid = threadIdx.x;
    build_normal<R>(A, grams, nmodes, mode, 0.0);
    __syncthreads();
    bool ok = cholesky<R>(A);
    double rg = 0.0;
    if (!ok) {
        // one retry with 1e-12 tr(V) / R on the diagonal
        __syncthreads();
        build_normal<R>(A, grams, nmodes, mode, 0.0);
        __syncthreads();
        if (tid == 0) {
            double tr = 0.0;
            for (int j = 0; j < R; ++j) tr += A[j][j];
            ridge = 1e-12 * tr / R;
        }
        __syncthreads();
        rg = ridge;
        build_normal<R>(A, grams, nmodes, mode, rg);
        __syncthreads();
        ok = cholesky<R>(A);
        if (!ok && tid == 0) status[0] |= 1;
    }
    __syncthreads();
    if (!ok) {
        for (int e = tid; e < R * R; e += blockDim.x) Vinv[e] = 0.0;
        return;
    }
    build_normal<R>(A, grams, nmodes, mode, rg);
    __syncthreads();
    gauss_jordan_inverse<R>(A);
    for (int e = tid; e < R * R; e += blockDim.x) Vinv[e] = A[e / R][e % R];
}

template <int R>
__global__ __launch_bounds__(256) void solve_rows_kernel(const float* __restrict__ M,
                                                          const double* __restrict__ Vinv,
                                                          int64_t rows, float* __restrict__ Y,
                                                          double* __restrict__ gpart,
                                                          double* __restrict__ ipart) {
    constexpr int RB = 256 / R;         // rows per batch
    constexpr int E = R * R;
    constexpr int PER = (E + 255) / 256;
    __shared__ double vinv[R][R];
    __shared__ float mt[RB][R];
    __shared__ float yt[RB][R];
    __shared__ double ired[RB][R];
    const int tid = threadIdx.x;
    const int bi = tid / R, col = tid % R;
    for (int e = tid; e < E; e += 256) vinv[e / R][e % R] = Vinv[e];
    const int64_t chunk = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = std::min<int64_t>(rows, (int64_t)blockIdx.x * chunk);
    const int64_t r1 = std::min<int64_t>(rows, r0 + chunk);
    double gacc[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) gacc[k] = 0.0;
    double iacc = 0.0;
    __syncthreads();
    for (int64_t base = r0; base < r1; base += RB) {
        const int nr = (int)std::min<int64_t>(RB, r1 - base);
        const bool valid = bi < nr;
        mt[bi][col] = valid ? M[(base + bi) * R + col] : 0.0f;
        __syncthreads();
        float yf = 0.0f;
        if (valid) {
            double y = 0.0;
#pragma unroll 8
            for (int s = 0; s < R; ++s) y += (double)mt[bi][s] * vinv[s][col];
            yf = (float)y;
            Y[(base + bi) * R + col] = yf;
            iacc += (double)mt[bi][col] * (double)yf;
        }
        yt[bi][col] = yf;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            if (e < E) {
                const int r = e / R, c = e % R;
                double s = 0.0;
                for (int i = 0; i < nr; ++i) s += (double)yt[i][r] * (double)yt[i][c];
                gacc[k] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = tid + 256 * k;
        if (e < E) gpart[(int64_t)blockIdx.x * E + e] = gacc[k];
    }
    ired[bi][col] = iacc;
    __syncthreads();
    if (tid < R) {
        double s = 0.0;
        for (int i = 0; i < RB; ++i) s += ired[i][tid];
        ipart[(int64_t)blockIdx.x * R + tid] = s;
    }
}

// Y = M V^-1 on the FP64 matrix cores (v_mfma_f64_16x16x4f64), for R a
// multiple of 16.  Each wave takes 16-row tiles.  Operand layout of the
// instruction on gfx950 (wave64, checked on the device): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] of a 16x4 by 4x16 step, and
// register v (0..3) of lane l holds D[4 v + l / 16][l % 16] of the 16x16
// result.  The contraction index k of step s for lane group q = l / 16 is
// k = q R/4 + s, so a lane's A values are R/4 consecutive columns of its row
// of M (vector loads) and its B values are the matching rows of V^-1 (held
// in registers for the whole kernel).  The rounded FP32 result feeds the
// Gram of the unnormalised factor with no data movement: for fixed v, the
// four rows 4 v + q of a tile are the k index of one more step, A = column
// tile c0 and B = column tile c1 of those rows.  <M, Y> per column (for the
// fit) is summed in FP64 per lane.
template <int R>
__global__ __launch_bounds__(256) void solve_rows_mfma_kernel(const float* __restrict__ M,
                                                               const double* __restrict__ Vinv,
                                                               int64_t rows, float* __restrict__ Y,
                                                               double* __restrict__ gpart,
                                                               double* __restrict__ ipart) {
    static_assert(R % 16 == 0, "rank");
    typedef double v4d __attribute__((ext_vector_type(4)));
    constexpr int CT = R / 16;             // column tiles
    constexpr int KS = R / 4;              // steps of the solve
    constexpr int NP = CT * (CT + 1) / 2;  // Gram tiles c0 <= c1
    constexpr int E = R * R;
    __shared__ double gsh[E];
    __shared__ double ish[4][4][R];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int rl = lane & 15, q = lane >> 4;

    double bv[CT][KS];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int s = 0; s < KS; ++s) bv[ct][s] = Vinv[(q * KS + s) * R + 16 * ct + rl];
    v4d gacc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) gacc[p] = v4d{0.0, 0.0, 0.0, 0.0};
    double iacc[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) iacc[ct] = 0.0;

    const int64_t tiles = (rows + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < tiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t r0 = tile * 16;
        // every load of the tile is issued before any of it is used: the
        // lane's A values, and M at the lane's result positions for <M, Y>
        float av[KS];
        float mv[CT][4];
        const int64_t ra = r0 + rl;
        if (ra < rows) {
            const float4* src = reinterpret_cast<const float4*>(M + ra * R + q * KS);
#pragma unroll
            for (int j = 0; j < KS / 4; ++j) {
                const float4 x = src[j];
                av[4 * j] = x.x;
                av[4 * j + 1] = x.y;
                av[4 * j + 2] = x.z;
                av[4 * j + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < KS; ++j) av[j] = 0.0f;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = r0 + 4 * v + q;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) mv[ct][v] = row < rows ? M[row * R + 16 * ct + rl] : 0.0f;
        }
        v4d acc[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)av[s], bv[ct][s], acc[ct], 0, 0, 0);
        double yd[CT][4];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = r0 + 4 * v + q;
                const int col = 16 * ct + rl;
                double y = 0.0;
                if (row < rows) {
                    const float yf = (float)acc[ct][v];
                    Y[row * R + col] = yf;
                    y = (double)yf;
                    iacc[ct] += (double)mv[ct][v] * y;
                }
                yd[ct][v] = y;
            }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int p = 0;
#pragma unroll
            for (int c0 = 0; c0 < CT; ++c0)
#pragma unroll
                for (int c1 = c0; c1 < CT; ++c1, ++p)
                    gacc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(yd[c0][v], yd[c1][v], gacc[p], 0, 0, 0);
        }
    }
    // the waves' Gram tiles (and their transposes) summed in LDS in wave
    // order; every entry belongs to one lane of a wave
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
            int p = 0;
#pragma unroll
            for (int c0 = 0; c0 < CT; ++c0)
#pragma unroll
                for (int c1 = c0; c1 < CT; ++c1, ++p)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = 16 * c0 + 4 * v + q, j = 16 * c1 + rl;
                        const double x = gacc[p][v];
                        gsh[i * R + j] = w == 0 ? x : gsh[i * R + j] + x;
                        if (c1 != c0) gsh[j * R + i] = w == 0 ? x : gsh[j * R + i] + x;
                    }
        }
        __syncthreads();
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) ish[wv][q][16 * ct + rl] = iacc[ct];
    __syncthreads();
    for (int e = threadIdx.x; e < E; e += 256) gpart[(int64_t)blockIdx.x * E + e] = gsh[e];
    if (threadIdx.x < R) {
        const int c = threadIdx.x;
        double t = 0.0;
        for (int w = 0; w < 4; ++w)
            for (int g = 0; g < 4; ++g) t += ish[w][g][c];
        ipart[(int64_t)blockIdx.x * R + c] = t;
    }
}

// Partial Grams Y^T Y on the FP64 matrix cores (R a multiple of 16): each
// wave takes 16-row tiles; lane (rl = lane % 16, q = lane / 16) holds
// Y(r0 + 4v + q, 16c + rl), which is both the A operand (column tile c0 of
// Y^T) and the B operand (column tile c1 of Y) of v_mfma_f64_16x16x4f64 for
// the 4 rows r0 + 4v .. r0 + 4v + 3.  The waves' tiles are summed in LDS in
// wave order, and the block writes partial[blockIdx][R*R].
template <int R>
__global__ __launch_bounds__(256) void gram_mfma_kernel(const float* __restrict__ Y, int64_t rows,
                                                         double* __restrict__ partial) {
    static_assert(R % 16 == 0, "rank");
    typedef double v4d __attribute__((ext_vector_type(4)));
    constexpr int CT = R / 16;
    constexpr int NP = CT * (CT + 1) / 2;
    constexpr int E = R * R;
    __shared__ double gsh[E];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int rl = lane & 15, q = lane >> 4;
    v4d gacc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) gacc[p] = v4d{0.0, 0.0, 0.0, 0.0};
    const int64_t tiles = (rows + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < tiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t r0 = tile * 16;
        double yd[CT][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = r0 + 4 * v + q;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) yd[ct][v] = row < rows ? (double)Y[row * R + 16 * ct + rl] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int p = 0;
#pragma unroll
            for (int c0 = 0; c0 < CT; ++c0)
#pragma unroll
                for (int c1 = c0; c1 < CT; ++c1, ++p)
                    gacc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(yd[c0][v], yd[c1][v], gacc[p], 0, 0, 0);
        }
    }
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
            int p = 0;
#pragma unroll
            for (int c0 = 0; c0 < CT; ++c0)
#pragma unroll
                for (int c1 = c0; c1 < CT; ++c1, ++p)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = 16 * c0 + 4 * v + q, j = 16 * c1 + rl;
                        const double x = gacc[p][v];
                        gsh[i * R + j] = w == 0 ? x : gsh[i * R + j] + x;
                        if (c1 != c0) gsh[j * R + i] = w == 0 ? x : gsh[j * R + i] + x;
                    }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < E; e += 256) partial[(int64_t)blockIdx.x * E + e] = gsh[e];
}

template <int R>
__global__ __launch_bounds__(256) void als_finish_kernel(const double* __restrict__ Gun,
                                                          const double* __restrict__ Isum,
                                                          int nmodes, int mode,
                                                          double* __restrict__ grams,
                                                          double* __restrict__ lambda,
                                                          double normX2, int want_fit,
                                                          double* __restrict__ fit) {
    constexpr int E = R * R;
    __shared__ double lam[R];
    __shared__ double red[256];
    const int tid = threadIdx.x;
    if (tid < R) {
        lam[tid] = sqrt(Gun[tid * R + tid]);
        lambda[tid] = lam[tid];
    }
    __syncthreads();
    double* Gm = grams + (int64_t)mode * E;
    for (int e = tid; e < E; e += 256) {
        const int r = e / R, c = e % R;
        const double lr = lam[r], lc = lam[c];
        Gm[e] = (lr > 0.0 && lc > 0.0) ? Gun[e] / (lr * lc) : 0.0;
    }
    if (!want_fit) return;
    __syncthreads();
    // ||Xhat||^2 = lam^T (Hadamard of all Grams) lam, in a fixed order
    double xh = 0.0;
    for (int e = tid; e < E; e += 256) {
        const int r = e / R, c = e % R;
        double h = 1.0;
        for (int w = 0; w < nmodes; ++w) h *= grams[(int64_t)w * E + e];
        xh += lam[r] * h * lam[c];
    }
    red[tid] = xh;
    __syncthreads();
    if (tid == 0) {
        double x = 0.0;
        for (int i = 0; i < 256; ++i) x += red[i];
        double in = 0.0;
        for (int r = 0; r < R; ++r) in += Isum[r];
        double res2 = normX2 + x - 2.0 * in;
        if (res2 < 0.0) res2 = 0.0;
        fit[0] = 1.0 - sqrt(res2) / sqrt(normX2);
    }
}

// Y(i, c) / lambda_c in FP64, rounded once; 4 columns (one 16-byte word) per
// thread, the grid covering the matrix in one sweep where it can.
template <int R>
__global__ void scale_cols_kernel(float* __restrict__ Y, int64_t rows,
                                  const double* __restrict__ lambda) {
    static_assert(R % 4 == 0, "rank");
    const int64_t total4 = rows * (R / 4);
    float4* Y4 = reinterpret_cast<float4*>(Y);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total4;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % (R / 4)) * 4;
        float4 y = Y4[i];
        const double l0 = lambda[c], l1 = lambda[c + 1], l2 = lambda[c + 2], l3 = lambda[c + 3];
        y.x = l0 > 0.0 ? (float)((double)y.x / l0) : 0.0f;
        y.y = l1 > 0.0 ? (float)((double)y.y / l1) : 0.0f;
        y.z = l2 > 0.0 ? (float)((double)y.z / l2) : 0.0f;
        y.w = l3 > 0.0 ? (float)((double)y.w / l3) : 0.0f;
        Y4[i] = y;
    }
}

__global__ void zero_i32_kernel(int32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <template <int> class K, typename... Args>
void by_rank(int rank, dim3 grid, dim3 block, hipStream_t s, Args... args) {
    switch (rank) {
        case 8: hipLaunchKernelGGL(K<8>::fn, grid, block, 0, s, args...); break;
        case 16: hipLaunchKernelGGL(K<16>::fn, grid, block, 0, s, args...); break;
        case 32: hipLaunchKernelGGL(K<32>::fn, grid, block, 0, s, args...); break;
        case 64: hipLaunchKernelGGL(K<64>::fn, grid, block, 0, s, args...); break;
        default: break;
    }
}

template <int R> struct GramP { static constexpr auto fn = gram_partial_kernel<R>; };
template <int R> struct GramMfma { static constexpr auto fn = gram_mfma_kernel<R>; };
template <> struct GramMfma<8> { static constexpr auto fn = gram_partial_kernel<8>; };
template <int R> struct NormInv { static constexpr auto fn = normal_inverse_kernel<R>; };
template <int R> struct Solve { static constexpr auto fn = solve_rows_kernel<R>; };
template <int R> struct SolveMfma { static constexpr auto fn = solve_rows_mfma_kernel<R>; };
template <> struct SolveMfma<8> { static constexpr auto fn = solve_rows_kernel<8>; };
template <int R> struct Finish { static constexpr auto fn = als_finish_kernel<R>; };
template <int R> struct Scale { static constexpr auto fn = scale_cols_kernel<R>; };

}  // namespace

int gram_blocks(int64_t rows) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (rows + 255) / 256));
}

void launch_gram_partial(int rank, const float* Y, int64_t rows, double* partial, hipStream_t s) {
#if SPT_GRAM_MFMA
    by_rank<GramMfma>(rank, dim3(gram_blocks(rows)), dim3(256), s, Y, rows, partial);
#else
    by_rank<GramP>(rank, dim3(gram_blocks(rows)), dim3(256), s, Y, rows, partial);
#endif
}

void launch_reduce_partials(const double* partial, int nblocks, int E, double* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((E + 31) / 32), dim3(256), 0, s, partial, nblocks,
                       E, out);
}

void launch_normal_inverse(int rank, int nmodes, int mode, const double* grams, double* Vinv,
                           int32_t* status, hipStream_t s) {
    by_rank<NormInv>(rank, dim3(1), dim3(256), s, grams, nmodes, mode, Vinv, status);
}

int solve_blocks(int64_t rows) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (rows + 255) / 256));
}

void launch_solve_rows(int rank, const float* M, const double* Vinv, int64_t rows, float* Y,
                       double* gpart, double* ipart, hipStream_t s) {
#if SPT_SOLVE_MFMA
    by_rank<SolveMfma>(rank, dim3(solve_blocks(rows)), dim3(256), s, M, Vinv, rows, Y, gpart, ipart);
#else
    by_rank<Solve>(rank, dim3(solve_blocks(rows)), dim3(256), s, M, Vinv, rows, Y, gpart, ipart);
#endif
}

void launch_als_finish(int rank, int nmodes, int mode, const double* Gun, const double* Isum,
                       double* grams, double* lambda, double normX2, int want_fit, double* fit,
                       hipStream_t s) {
    by_rank<Finish>(rank, dim3(1), dim3(256), s, Gun, Isum, nmodes, mode, grams, lambda, normX2,
                    want_fit, fit);
}

void launch_scale_cols(int rank, float* Y, int64_t rows, const double* lambda, hipStream_t s) {
    const int64_t total4 = rows * (rank / 4);
    if (total4 == 0) return;
    const int64_t blocks = std::min<int64_t>((total4 + 255) / 256, int64_t(1) << 20);
    by_rank<Scale>(rank, dim3((unsigned)blocks), dim3(256), s, Y, rows, lambda);
}

void launch_zero_i32(int32_t* p, int n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

}  // namespace spt
