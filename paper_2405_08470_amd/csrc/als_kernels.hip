// CP-ALS dense step on the device, FP64 for every R x R quantity:
// Grams G_w = Y_w^T Y_w, the normal matrix V = Hadamard of the other Grams,
// its Cholesky factorisation and inverse, Y_d = M_d V^-1, column norms
// lambda and the CP fit.  Reductions are two-stage (block partials, then
// one ordered pass), so results do not depend on scheduling.
#include <algorithm>

#include "kernels.hpp"

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

// In-place Cholesky of the R x R matrix in A (lower triangle); returns
// false if a pivot is not positive.
template <int R>
__device__ bool cholesky(double (*A)[R + 1]) {
    __shared__ int ok;
    const int tid = threadIdx.x;
    if (tid == 0) ok = 1;
    __syncthreads();
    for (int j = 0; j < R; ++j) {
        if (tid == 0) {
            double d = A[j][j];
            for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
            if (!(d > 0.0)) {
                ok = 0;
                d = 1.0;
            }
            A[j][j] = sqrt(d);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < R; i += blockDim.x) {
            double x = A[i][j];
            for (int k = 0; k < j; ++k) x -= A[i][k] * A[j][k];
            A[i][j] = x / A[j][j];
        }
        __syncthreads();
    }
    return ok != 0;
}

template <int R>
__global__ __launch_bounds__(256) void normal_inverse_kernel(const double* __restrict__ grams,
                                                              int nmodes, int mode,
                                                              double* __restrict__ Vinv,
                                                              int32_t* __restrict__ status) {
    __shared__ double A[R][R + 1];
    __shared__ double B[R][R + 1];
    const int tid = threadIdx.x;
    // V = Hadamard product of the other modes' Grams
    for (int e = tid; e < R * R; e += blockDim.x) {
        const int r = e / R, c = e % R;
        double v = 1.0;
        for (int w = 0; w < nmodes; ++w)
            if (w != mode) v *= grams[(int64_t)w * R * R + e];
        A[r][c] = v;
        B[r][c] = v;
    }
    __syncthreads();
    bool ok = cholesky<R>(A);
    if (!ok) {
        __shared__ double ridge;
        if (tid == 0) {
            double tr = 0.0;
            for (int j = 0; j < R; ++j) tr += B[j][j];
            ridge = 1e-12 * tr / R;
        }
        __syncthreads();
        for (int e = tid; e < R * R; e += blockDim.x) {
            const int r = e / R, c = e % R;
            A[r][c] = B[r][c] + (r == c ? ridge : 0.0);
        }
        __syncthreads();
        ok = cholesky<R>(A);
        if (!ok && tid == 0) status[0] |= 1;
    }
    __syncthreads();
    // Linv (lower): column c solves L x = e_c by forward substitution
    for (int c = tid; c < R; c += blockDim.x) {
        for (int i = 0; i < R; ++i) {
            if (i < c) {
                B[i][c] = 0.0;
                continue;
            }
            double x = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) x -= A[i][k] * B[k][c];
            B[i][c] = x / A[i][i];
        }
    }
    __syncthreads();
    // V^-1 = Linv^T Linv
    for (int e = tid; e < R * R; e += blockDim.x) {
        const int r = e / R, c = e % R;
        double s = 0.0;
        for (int k = (r > c ? r : c); k < R; ++k) s += B[k][r] * B[k][c];
        Vinv[e] = ok ? s : 0.0;
    }
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

template <int R>
__global__ void scale_cols_kernel(float* __restrict__ Y, int64_t rows,
                                  const double* __restrict__ lambda) {
    const int64_t total = rows * R;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double l = lambda[i % R];
        Y[i] = l > 0.0 ? (float)((double)Y[i] / l) : 0.0f;
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
template <int R> struct NormInv { static constexpr auto fn = normal_inverse_kernel<R>; };
template <int R> struct Solve { static constexpr auto fn = solve_rows_kernel<R>; };
template <int R> struct Finish { static constexpr auto fn = als_finish_kernel<R>; };
template <int R> struct Scale { static constexpr auto fn = scale_cols_kernel<R>; };

}  // namespace

int gram_blocks(int64_t rows) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (rows + 255) / 256));
}

void launch_gram_partial(int rank, const float* Y, int64_t rows, double* partial, hipStream_t s) {
    by_rank<GramP>(rank, dim3(gram_blocks(rows)), dim3(256), s, Y, rows, partial);
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
    by_rank<Solve>(rank, dim3(solve_blocks(rows)), dim3(256), s, M, Vinv, rows, Y, gpart, ipart);
}

void launch_als_finish(int rank, int nmodes, int mode, const double* Gun, const double* Isum,
                       double* grams, double* lambda, double normX2, int want_fit, double* fit,
                       hipStream_t s) {
    by_rank<Finish>(rank, dim3(1), dim3(256), s, Gun, Isum, nmodes, mode, grams, lambda, normX2,
                    want_fit, fit);
}

void launch_scale_cols(int rank, float* Y, int64_t rows, const double* lambda, hipStream_t s) {
    const int64_t total = rows * rank;
    if (total == 0) return;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
    by_rank<Scale>(rank, dim3((unsigned)blocks), dim3(256), s, Y, rows, lambda);
}

void launch_zero_i32(int32_t* p, int n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

}  // namespace spt
