// A record of the nonzero stream: RW 32-bit words (the indices as the
// layout packs them, then the value's bits in the last word).  Records of a
// multiple of 16 bytes move as 16-byte vectors; 12-byte records as three
// dwords (4-byte aligned).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spt {

template <int RW>
struct Rec {
    uint32_t w[RW];
};

template <int W, int RW>
__device__ __forceinline__ uint32_t rword(const Rec<RW>& r) {
    static_assert(W < RW, "word");
    return r.w[W];
}

template <int RW>
__device__ __forceinline__ void load_rec(const uint32_t* __restrict__ base, int64_t p, Rec<RW>& r) {
    if constexpr (RW % 4 == 0) {
        const uint4* src = reinterpret_cast<const uint4*>(base + p * RW);
#pragma unroll
        for (int k = 0; k < RW / 4; ++k) {
            const uint4 v = src[k];
            r.w[4 * k] = v.x;
            r.w[4 * k + 1] = v.y;
            r.w[4 * k + 2] = v.z;
            r.w[4 * k + 3] = v.w;
        }
    } else {
        const uint32_t* src = base + p * RW;
#pragma unroll
        for (int k = 0; k < RW; ++k) r.w[k] = src[k];
    }
}

template <int RW>
__device__ __forceinline__ void store_rec(uint32_t* __restrict__ base, int64_t p, const Rec<RW>& r) {
    if constexpr (RW % 4 == 0) {
        uint4* dst = reinterpret_cast<uint4*>(base + p * RW);
#pragma unroll
        for (int k = 0; k < RW / 4; ++k)
            dst[k] = make_uint4(r.w[4 * k], r.w[4 * k + 1], r.w[4 * k + 2], r.w[4 * k + 3]);
    } else {
        uint32_t* dst = base + p * RW;
#pragma unroll
        for (int k = 0; k < RW; ++k) dst[k] = r.w[k];
    }
}

}  // namespace spt
