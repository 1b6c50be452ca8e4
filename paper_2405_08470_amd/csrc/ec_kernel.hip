// Launch side of the elementwise kernel (ec_kernel.hpp, instantiated per
// mode count in ec_n2.hip .. ec_n8.hip), the split-row fixup, the BF16 copy
// of the factors and the remap along a chain of next positions.
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "kernels.hpp"
#include "record.hpp"

namespace spt {

EcFnPtr pick_ec_n2(int, int, int, int, bool);
EcFnPtr pick_ec_n3(int, int, int, int, bool);
EcFnPtr pick_ec_n4(int, int, int, int, bool);
EcFnPtr pick_ec_n5(int, int, int, int, bool);
EcFnPtr pick_ec_n6(int, int, int, int, bool);
EcFnPtr pick_ec_n7(int, int, int, int, bool);
EcFnPtr pick_ec_n8(int, int, int, int, bool);

namespace {

// Split rows: one workgroup per row sums its carry slots.  Thread (q, r)
// adds slots q, q + Q, q + 2Q, ... of rank r in four interleaved chains,
// then the Q partials are added in order of q -- a fixed order, so the
// result does not depend on scheduling.  Blocks past the split rows fill
// the rows that have no nonzero with zeros.
template <int R>
__global__ __launch_bounds__(1024) void fixup_kernel(const FixupArgs a, int zero_blocks) {
    constexpr int Q = 1024 / R;
    __shared__ float part[Q][R];
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < a.nsplit) {
        const int j = blockIdx.x;
        const int q = tid / R, r = tid % R;
        const int k0 = a.split_ptr[j], k1 = a.split_ptr[j + 1];
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
        int k = k0 + q;
        for (; k + 3 * Q < k1; k += 4 * Q) {
            s0 += a.carry[(int64_t)k * R + r];
            s1 += a.carry[(int64_t)(k + Q) * R + r];
            s2 += a.carry[(int64_t)(k + 2 * Q) * R + r];
            s3 += a.carry[(int64_t)(k + 3 * Q) * R + r];
        }
        for (; k < k1; k += Q) s0 += a.carry[(int64_t)k * R + r];
        part[q][r] = (s0 + s1) + (s2 + s3);
        __syncthreads();
        if (tid < R) {
            float t = 0.f;
            for (int i = 0; i < Q; ++i) t += part[i][tid];
            a.out[(int64_t)a.split_row[j] * R + tid] = t;
        }
        return;
    }
    // zero rows: float4 per thread
    constexpr int R4 = R / 4;
    const int64_t total = (int64_t)a.nempty * R4;
    const int64_t stride = (int64_t)zero_blocks * 1024;
    for (int64_t i = (int64_t)(blockIdx.x - a.nsplit) * 1024 + tid; i < total; i += stride) {
        const int64_t row = a.empty_rows[i / R4];
        reinterpret_cast<float4*>(a.out + row * R)[i % R4] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

struct NxtChain {
    const int32_t* nxt[8];
};

// FP32 -> BF16 by rounding the bit pattern to nearest, ties to even (add
// 0x7FFF plus the lowest kept bit, truncate); NaNs stay quiet NaNs.
__global__ void to_bf16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t u = __float_as_uint(src[i]);
        if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
            dst[i] = (uint16_t)((u >> 16) | 0x0040u);
        } else {
            u += 0x7FFFu + ((u >> 16) & 1u);
            dst[i] = (uint16_t)(u >> 16);
        }
    }
}

template <int RW>
__global__ void remap_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                             int64_t nnz, NxtChain ch, int hops) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = p;
        for (int h = 0; h < hops; ++h) d = ch.nxt[h][d];
        Rec<RW> r;
        load_rec<RW>(in, p, r);
        store_rec<RW>(out, d, r);
    }
}

EcFnPtr pick_ec(int nmodes, int rank, int fdtype, int words, int kind, bool reuse) {
    switch (nmodes) {
        case 2: return pick_ec_n2(rank, fdtype, words, kind, reuse);
        case 3: return pick_ec_n3(rank, fdtype, words, kind, reuse);
        case 4: return pick_ec_n4(rank, fdtype, words, kind, reuse);
        case 5: return pick_ec_n5(rank, fdtype, words, kind, reuse);
        case 6: return pick_ec_n6(rank, fdtype, words, kind, reuse);
        case 7: return pick_ec_n7(rank, fdtype, words, kind, reuse);
        case 8: return pick_ec_n8(rank, fdtype, words, kind, reuse);
        default: return nullptr;
    }
}

// Workgroups of f one CU holds at once (0 if the query fails).
int resident_blocks(EcFnPtr f) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(f), 64, 0) != hipSuccess)
        return 0;
    return nb;
}

// The elementwise kernel of a combination: the form that reuses the last
// gathered row when it keeps the occupancy of the plain form, else the plain
// form (decided once per combination and device).
EcFnPtr choose_ec(int nmodes, int rank, int fdtype, int words, int kind) {
#ifdef SPT_EC_FORM  // build option: 0 = always the plain form, 1 = always the reuse form
    return pick_ec(nmodes, rank, fdtype, words, kind, SPT_EC_FORM != 0);
#endif
    const EcFnPtr plain = pick_ec(nmodes, rank, fdtype, words, kind, false);
    const EcFnPtr reuse = pick_ec(nmodes, rank, fdtype, words, kind, true);
    if (!plain || !reuse) return plain;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return plain;
    static std::mutex mu;
    static std::map<std::pair<int, EcFnPtr>, EcFnPtr> chosen;
    std::lock_guard<std::mutex> lock(mu);
    auto it = chosen.find({dev, plain});
    if (it != chosen.end()) return it->second;
    const int occ_plain = resident_blocks(plain), occ_reuse = resident_blocks(reuse);
    const EcFnPtr f = occ_reuse > 0 && occ_reuse >= occ_plain ? reuse : plain;
    chosen[{dev, plain}] = f;
    return f;
}

}  // namespace

bool pick_ec_exists(int nmodes, int rank, int fdtype, int words, int kind) {
    return pick_ec(nmodes, rank, fdtype, words, kind, false) != nullptr;
}

bool launch_ec(int nmodes, int rank, int fdtype, int words, int kind, int kappa, const EcArgs& a,
               hipStream_t s) {
    if (kappa <= 0) return pick_ec(nmodes, rank, fdtype, words, kind, false) != nullptr;
    const EcFnPtr f = choose_ec(nmodes, rank, fdtype, words, kind);
    if (!f) return false;
    hipLaunchKernelGGL(f, dim3((unsigned)kappa), dim3(64), 0, s, a);
    return true;
}

void launch_fixup(int rank, const FixupArgs& a, hipStream_t s) {
    const int64_t zero_work = (int64_t)a.nempty * (rank / 4);
    const int zero_blocks = (int)std::min<int64_t>((zero_work + 1023) / 1024, 1024);
    const int blocks = a.nsplit + zero_blocks;
    if (blocks == 0) return;
    switch (rank) {
        case 8: hipLaunchKernelGGL(fixup_kernel<8>, dim3(blocks), dim3(1024), 0, s, a, zero_blocks); break;
        case 16: hipLaunchKernelGGL(fixup_kernel<16>, dim3(blocks), dim3(1024), 0, s, a, zero_blocks); break;
        case 32: hipLaunchKernelGGL(fixup_kernel<32>, dim3(blocks), dim3(1024), 0, s, a, zero_blocks); break;
        case 64: hipLaunchKernelGGL(fixup_kernel<64>, dim3(blocks), dim3(1024), 0, s, a, zero_blocks); break;
        case 128: hipLaunchKernelGGL(fixup_kernel<128>, dim3(blocks), dim3(1024), 0, s, a, zero_blocks); break;
        default: break;
    }
}

void launch_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t s) {
    if (n == 0) return;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
}

void launch_remap(int words, int64_t nnz, const uint32_t* in, uint32_t* out,
                  const int32_t* const* nxt, int hops, hipStream_t s) {
    if (nnz == 0) return;
    NxtChain ch{};
    for (int h = 0; h < hops; ++h) ch.nxt[h] = nxt[h];
    const int threads = 256;
    const int64_t blocks = std::min<int64_t>((nnz + threads - 1) / threads, 8192);
    if (words == 3)
        hipLaunchKernelGGL((remap_kernel<3>), dim3((unsigned)blocks), dim3(threads), 0, s, in, out,
                           nnz, ch, hops);
    else if (words == 4)
        hipLaunchKernelGGL((remap_kernel<4>), dim3((unsigned)blocks), dim3(threads), 0, s, in, out,
                           nnz, ch, hops);
    else if (words == 8)
        hipLaunchKernelGGL((remap_kernel<8>), dim3((unsigned)blocks), dim3(threads), 0, s, in, out,
                           nnz, ch, hops);
    else
        hipLaunchKernelGGL((remap_kernel<12>), dim3((unsigned)blocks), dim3(threads), 0, s, in, out,
                           nnz, ch, hops);
}

}  // namespace spt
