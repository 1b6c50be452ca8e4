// Forward pass of the gradient-based CP fit over the observed nonzeros:
// model value m_e = sum_r prod_w Y_w(i_w(e), r) at every nonzero of the
// stream, the residual record (the same indices, value m_e - x_e) written to
// a second stream in the same order, and FP64 partial sums of (x_e - m_e)^2.
// The adjoint is the MTTKRP of that residual stream (ec_kernel), since
// d/dY_d of 1/2 sum_e (x_e - m_e)^2 is the MTTKRP of (m_e - x_e).
#include <algorithm>

#include "kernels.hpp"
#include "record.hpp"

namespace spt {

namespace {

template <int W, int RW, int KIND>
__device__ __forceinline__ uint32_t gdecode(const Rec<RW>& r, const int32_t* foff,
                                            const uint32_t* fmask) {
    if constexpr (KIND == kWord32) {
        return rword<W, RW>(r);
    } else if constexpr (KIND == kHalf16) {
        return (rword<W / 2, RW>(r) >> ((W & 1) * 16)) & 0xFFFFu;
    } else {
        const uint64_t lo = ((uint64_t)rword<1, RW>(r) << 32) | rword<0, RW>(r);
        const int o = foff[W];
        if constexpr (RW == 3) {
            return (uint32_t)(lo >> o) & fmask[W];
        } else {
            const uint64_t hi = rword<2, RW>(r);
            const uint64_t x = o >= 64 ? (hi >> (o - 64)) : ((lo >> o) | (o ? (hi << (64 - o)) : 0));
            return (uint32_t)x & fmask[W];
        }
    }
}

// Product over modes of the lane's 4 ranks of each gathered row.
template <int N, int R, int RW, int KIND, int W>
__device__ __forceinline__ void mult_rows(const Rec<RW>& r, const ForwardArgs& a, int li,
                                          float (&p)[4]) {
    if constexpr (W < N) {
        const uint32_t c = gdecode<W, RW, KIND>(r, a.foff, a.fmask);
        const float4 y = *reinterpret_cast<const float4*>(a.fac[W] + (int64_t)c * R + li * 4);
        p[0] *= y.x;
        p[1] *= y.y;
        p[2] *= y.z;
        p[3] *= y.w;
        mult_rows<N, R, RW, KIND, W + 1>(r, a, li, p);
    }
}

// One nonzero per group of L = R/4 lanes; the group's partial dot products
// are summed across its lanes with butterfly shuffles.  The record of the
// group's next nonzero is fetched before the current one's rows are
// gathered, so each iteration waits for one round trip instead of two.
template <int N, int R, int RW, int KIND>
__global__ __launch_bounds__(256) void forward_kernel(const ForwardArgs a) {
    constexpr int L = R / 4;
    constexpr int GPB = 256 / L;  // nonzeros per block per iteration
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int g = tid / L, li = tid % L;
    const int64_t stride = (int64_t)gridDim.x * GPB;
    double loss = 0.0;
    int64_t p = (int64_t)blockIdx.x * GPB + g;
    Rec<RW> r{};
    if (p < a.nnz) load_rec<RW>(a.rec_in, p, r);
    for (; p < a.nnz; p += stride) {
        Rec<RW> rn = r;
        if (p + stride < a.nnz) load_rec<RW>(a.rec_in, p + stride, rn);
        float prod[4] = {1.f, 1.f, 1.f, 1.f};
        mult_rows<N, R, RW, KIND, 0>(r, a, li, prod);
        float m = (prod[0] + prod[1]) + (prod[2] + prod[3]);
#pragma unroll
        for (int off = 1; off < L; off <<= 1) m += __shfl_xor(m, off, L);
        const float x = __uint_as_float(rword<RW - 1, RW>(r));
        const float res = m - x;
        if (li == 0) {
            Rec<RW> o = r;
            o.w[RW - 1] = __float_as_uint(res);
            store_rec<RW>(a.rec_res, p, o);
            loss += 0.5 * (double)res * (double)res;
        }
        r = rn;
    }
    red[tid] = loss;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (tid < s2) red[tid] += red[tid + s2];
        __syncthreads();
    }
    if (tid == 0) a.loss_part[blockIdx.x] = red[0];
}

template <int N, int RW, int KIND>
bool fwd_rank(int rank, int blocks, const ForwardArgs& a, hipStream_t s) {
    switch (rank) {
        case 8: hipLaunchKernelGGL((forward_kernel<N, 8, RW, KIND>), dim3(blocks), dim3(256), 0, s, a); return true;
        case 16: hipLaunchKernelGGL((forward_kernel<N, 16, RW, KIND>), dim3(blocks), dim3(256), 0, s, a); return true;
        case 32: hipLaunchKernelGGL((forward_kernel<N, 32, RW, KIND>), dim3(blocks), dim3(256), 0, s, a); return true;
        case 64: hipLaunchKernelGGL((forward_kernel<N, 64, RW, KIND>), dim3(blocks), dim3(256), 0, s, a); return true;
        default: return false;
    }
}

template <int N>
bool fwd_layout(int rank, int words, int kind, int blocks, const ForwardArgs& a, hipStream_t s) {
    if constexpr (N <= 2) {
        if (words == 3 && kind == kWord32) return fwd_rank<N, 3, kWord32>(rank, blocks, a, s);
        if (words == 4 && kind == kWord32) return fwd_rank<N, 4, kWord32>(rank, blocks, a, s);
    } else if constexpr (N == 3) {
        if (words == 3 && kind == kPacked) return fwd_rank<N, 3, kPacked>(rank, blocks, a, s);
        if (words == 4 && kind == kWord32) return fwd_rank<N, 4, kWord32>(rank, blocks, a, s);
    } else if constexpr (N <= 6) {
        if constexpr (N == 4)
            if (words == 3 && kind == kHalf16) return fwd_rank<N, 3, kHalf16>(rank, blocks, a, s);
        if (words == 3 && kind == kPacked) return fwd_rank<N, 3, kPacked>(rank, blocks, a, s);
        if (words == 4 && kind == kHalf16) return fwd_rank<N, 4, kHalf16>(rank, blocks, a, s);
        if (words == 4 && kind == kPacked) return fwd_rank<N, 4, kPacked>(rank, blocks, a, s);
        if (words == 8 && kind == kWord32) return fwd_rank<N, 8, kWord32>(rank, blocks, a, s);
    } else if constexpr (N == 7) {
        if (words == 3 && kind == kPacked) return fwd_rank<N, 3, kPacked>(rank, blocks, a, s);
        if (words == 8 && kind == kWord32) return fwd_rank<N, 8, kWord32>(rank, blocks, a, s);
    } else {
        if (words == 3 && kind == kPacked) return fwd_rank<N, 3, kPacked>(rank, blocks, a, s);
        if (words == 8 && kind == kHalf16) return fwd_rank<N, 8, kHalf16>(rank, blocks, a, s);
        if (words == 12 && kind == kWord32) return fwd_rank<N, 12, kWord32>(rank, blocks, a, s);
    }
    return false;
}

}  // namespace

int forward_blocks(int64_t nnz) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(2048, (nnz + 255) / 256));
}

bool launch_forward(int nmodes, int rank, int words, int kind, const ForwardArgs& a,
                    hipStream_t s) {
    const int blocks = forward_blocks(a.nnz);
    switch (nmodes) {
        case 2: return fwd_layout<2>(rank, words, kind, blocks, a, s);
        case 3: return fwd_layout<3>(rank, words, kind, blocks, a, s);
        case 4: return fwd_layout<4>(rank, words, kind, blocks, a, s);
        case 5: return fwd_layout<5>(rank, words, kind, blocks, a, s);
        case 6: return fwd_layout<6>(rank, words, kind, blocks, a, s);
        case 7: return fwd_layout<7>(rank, words, kind, blocks, a, s);
        case 8: return fwd_layout<8>(rank, words, kind, blocks, a, s);
        default: return false;
    }
}

}  // namespace spt
