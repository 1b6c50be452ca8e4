// Elementwise computation (Alg. 2) and dynamic remapping (Alg. 3) for
// one output mode, mapped to gfx950 wavefronts (the role of Alg. 4).
//
// One workgroup = one wave64 = one partition B_{d,z} of Alg. 1.  A nonzero
// is handled by L = R/4 lanes, each holding 4 consecutive ranks (one 16-byte
// load per gathered factor row per lane, so a row of R FP32 values arrives
// in one request).  The wave splits its partition into G = 64/L contiguous
// sub-ranges, one per lane group; a group walks its sub-range in stream
// order, so runs of equal output row (the stream is grouped by row) are
// summed in registers and each finished row is stored once.  A row that
// crosses a sub-range boundary is finished by a short chain combine in LDS
// at the end.  Rows split across partitions (pieces, see the planner) go to
// a carry slot instead, summed later by the fixup kernel.  No atomics.
//
// Records are fetched one step ahead, one per lane (software pipeline),
// which is also where each record is written to its remap position in the
// next mode's stream (Alg. 3).  Each lane decodes the record it fetched into
// LDS once; the gathers of several nonzeros are issued before any of them is
// consumed.
#pragma once

#include <algorithm>
#include <utility>

#include "kernels.hpp"

// float4 gathers a lane keeps in flight (register budget of the batch)
#ifndef SPT_GATHER_INFLIGHT
#define SPT_GATHER_INFLIGHT 16
#endif

namespace spt {
namespace {

template <int RW>
struct Rec {
    uint4 q[RW / 4];
};

template <int W, int RW>
__device__ __forceinline__ uint32_t rword(const Rec<RW>& r) {
    static_assert(W < RW, "word");
    const uint4& v = r.q[W / 4];
    return (W % 4 == 0) ? v.x : (W % 4 == 1) ? v.y : (W % 4 == 2) ? v.z : v.w;
}

template <int RW>
__device__ __forceinline__ void load_rec(const uint32_t* __restrict__ base, int64_t p, Rec<RW>& r) {
    const uint4* src = reinterpret_cast<const uint4*>(base + p * RW);
#pragma unroll
    for (int k = 0; k < RW / 4; ++k) r.q[k] = src[k];
}

template <int RW>
__device__ __forceinline__ void store_rec(uint32_t* __restrict__ base, int64_t p, const Rec<RW>& r) {
    uint4* dst = reinterpret_cast<uint4*>(base + p * RW);
#pragma unroll
    for (int k = 0; k < RW / 4; ++k) dst[k] = r.q[k];
}

// Index of mode W in a record (layout kinds of the planner).
template <int W, int RW, int KIND>
__device__ __forceinline__ uint32_t decode(const Rec<RW>& r, const EcArgs& a) {
    if constexpr (KIND == kWord32) {
        return rword<W, RW>(r);
    } else if constexpr (KIND == kHalf16) {
        return (rword<W / 2, RW>(r) >> ((W & 1) * 16)) & 0xFFFFu;
    } else {  // packed into the first 96 bits of a 16-byte record
        const uint64_t lo = ((uint64_t)rword<1, RW>(r) << 32) | rword<0, RW>(r);
        const uint64_t hi = rword<2, RW>(r);
        const int o = a.foff[W];
        const uint64_t x = o >= 64 ? (hi >> (o - 64)) : ((lo >> o) | (o ? (hi << (64 - o)) : 0));
        return (uint32_t)x & a.fmask[W];
    }
}

template <int RW, int KIND, int... W>
__device__ __forceinline__ void decode_all(const Rec<RW>& r, const EcArgs& a, uint32_t (*st)[64],
                                           int lane, std::integer_sequence<int, W...>) {
    ((st[W][lane] = decode<W, RW, KIND>(r, a)), ...);
}

// Carry slot of `row` if it is a split row of this partition, else -1.
__device__ __forceinline__ int split_slot(const EcArgs& a, int sp0, int sp1, int row) {
    int slot = -1;
    for (int j = sp0; j < sp1; ++j)
        if (a.psplit_row[j] == row) slot = a.psplit_slot[j];
    return slot;
}

template <int R>
__device__ __forceinline__ float* row_dst(const EcArgs& a, int row, int slot) {
    return slot >= 0 ? a.carry + (int64_t)slot * R : a.out + (int64_t)row * R;
}

// Factor element types.  A lane loads 16 bytes of a factor row at a time:
// 4 FP32 values, or 8 BF16 values (raw 16-bit patterns, widened exactly).
struct FacF32 {
    static constexpr int kPerLoad = 4;
    static constexpr int kBytes = 4;
};
struct FacBF16 {
    static constexpr int kPerLoad = 8;
    static constexpr int kBytes = 2;
};

template <typename FT>
__device__ __forceinline__ void widen(const uint4& u, float (&f)[FT::kPerLoad]) {
    if constexpr (FT::kPerLoad == 4) {
        f[0] = __uint_as_float(u.x);
        f[1] = __uint_as_float(u.y);
        f[2] = __uint_as_float(u.z);
        f[3] = __uint_as_float(u.w);
    } else {
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f[2 * i] = __uint_as_float(w[i] << 16);
            f[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
        }
    }
}

template <int V>
__device__ __forceinline__ void store_vals(float* dst, const float (&v)[V]) {
#pragma unroll
    for (int i = 0; i < V; i += 4)
        *reinterpret_cast<float4*>(dst + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
}

// Value of `v` in lane `src` of the wave (0 <= src < 64; every lane active).
__device__ __forceinline__ uint32_t lane_get(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}
__device__ __forceinline__ float lane_get(float v, int src) {
    return __uint_as_float(lane_get(__float_as_uint(v), src));
}

// Slot of factor row c in a direct-mapped table of h slots (multiplicative
// hash; the host builds the tag tables with the same function).
__device__ __forceinline__ uint32_t hot_slot(uint32_t c, uint32_t h) {
    return __umulhi(c * 0x9E3779B1u, h);
}

// Words of a decoded record: the N indices, the value's bits, the carry slot.
template <int N>
struct Words {
    uint32_t w[N + 2];
};

template <int RW, int KIND, int N, int... W>
__device__ __forceinline__ void decode_words(const Rec<RW>& r, const EcArgs& a, Words<N>& o,
                                             std::integer_sequence<int, W...>) {
    ((o.w[W] = decode<W, RW, KIND>(r, a)), ...);
}

// o.w[idx] for idx < N: an element of a vector value selected at run time
// (a chain of conditional moves; indexing a register array at run time would
// put it in scratch memory)
typedef uint32_t Word8 __attribute__((ext_vector_type(8)));
template <int N>
__device__ __forceinline__ uint32_t pick_word(const Words<N>& o, int idx) {
    Word8 v = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = o.w[i];
    return v[idx & 7];
}

template <int N, int R, int RW, int KIND, typename FT, int WPB>
__global__ __launch_bounds__(64 * WPB) void ec_kernel(const EcArgs a) {
    constexpr int V = FT::kPerLoad;
    constexpr int L = R / V;     // lanes per nonzero
    constexpr int G = 64 / L;    // lane groups = nonzeros in flight
    constexpr int NG = N - 1;    // gathered factor rows per nonzero
    constexpr int RQ = R * FT::kBytes / 16;  // 16-byte words per factor row
    // nonzeros whose gathers are issued together: the largest divisor of L
    // with at most SPT_GATHER_INFLIGHT float4 gathers in flight per lane
    constexpr int BMAX = (SPT_GATHER_INFLIGHT / NG) > 0 ? SPT_GATHER_INFLIGHT / NG : 1;
    constexpr int B = L <= BMAX ? L : (L / 2 <= BMAX ? L / 2 : (L / 4 <= BMAX ? L / 4 : (L / 8 <= BMAX ? L / 8 : 1)));
    static_assert(R % V == 0 && L >= 1 && 64 % L == 0 && L % B == 0 && RQ == L, "rank");
    constexpr uint32_t kHot = 0x80000000u;  // marks an LDS slot in place of a row
    constexpr uint32_t kNone = 0xFFFFFFFFu;

    // the hot rows of the gathered factors: tags, then rows
    HIP_DYNAMIC_SHARED(uint4, hot_lds)

    const int wv = threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    const int g = lane / L;
    const int li = lane % L;
    const int mode = a.rot[0];
    constexpr auto seq = std::make_integer_sequence<int, N>{};

    // ---- gathered mode k (1..N-1) keeps hot_h[k] rows in LDS: all rows of
    // the mode (hot_full: slot = row), or a direct-mapped table whose tag
    // says which row each slot holds (-1: none)
    int32_t* const tags = reinterpret_cast<int32_t*>(hot_lds);
#pragma unroll
    for (int k = 1; k < N; ++k) {
        const int h = a.hot_h[k];
        if (h == 0) continue;
        if (!a.hot_full[k])
            for (int i = threadIdx.x; i < h; i += 64 * WPB) tags[a.hot_tag_off[k] + i] = a.hot_tag[k][i];
        const uint4* src = static_cast<const uint4*>(a.fac[k]);
        for (int i = threadIdx.x; i < h * RQ; i += 64 * WPB) {
            const int sl = i / RQ;
            const int row = a.hot_full[k] ? sl : a.hot_tag[k][sl];
            if (row >= 0) hot_lds[a.hot_row_off[k] + i] = src[(int64_t)row * RQ + i % RQ];
        }
    }
    __syncthreads();

    // ---- the wave's partitions: z = block + grid * (wave + WPB * j)
    for (int64_t z = blockIdx.x + (int64_t)gridDim.x * wv; z < a.kappa; z += (int64_t)gridDim.x * WPB) {
        const int64_t s = a.ptr[z];
        const int64_t n = a.ptr[z + 1] - s;
        if (n == 0) continue;
        // rows of this partition split across partitions, one per lane
        const int sp0 = a.psplit_ptr[z], sp1 = a.psplit_ptr[z + 1];
        const int nsp = sp1 - sp0;
        const bool sp_reg = nsp <= 64;
        int32_t my_srow = -1, my_sslot = -1;
        if (sp_reg && lane < nsp) {
            my_srow = a.psplit_row[sp0 + lane];
            my_sslot = a.psplit_slot[sp0 + lane];
        }
        // carry slot of a row of this partition (-1: not a split row)
        auto slot_of = [&](uint32_t row) {
            int slot = -1;
            if (sp_reg) {
                for (int j = 0; j < nsp; ++j) {
                    const uint32_t r = (uint32_t)__builtin_amdgcn_readlane(my_srow, j);
                    const int sl = __builtin_amdgcn_readlane(my_sslot, j);
                    if (r == row) slot = sl;
                }
            } else {
                slot = split_slot(a, sp0, sp1, (int)row);
            }
            return slot;
        };

        const int64_t q = n / G, rm = n % G;
        const int64_t gs = s + g * q + (g < rm ? g : rm);
        const int gn = (int)(q + (g < rm ? 1 : 0));
        const int64_t ge = gs + gn;

        // output rows around the group's sub-range: before, first, last, after
        uint32_t brow[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t p = j == 0 ? gs - 1 : j == 1 ? gs : j == 2 ? ge - 1 : ge;
            brow[j] = kNone;
            if (gn > 0 && p >= s && p < s + n) {
                Rec<RW> r;
                load_rec<RW>(a.rec_in, p, r);
                Words<N> wd;
                decode_words<RW, KIND>(r, a, wd, seq);
                brow[j] = pick_word(wd, mode);
            }
        }
        const bool open_left = gn > 0 && brow[0] != kNone && brow[0] == brow[1];
        const bool open_right = gn > 0 && brow[3] != kNone && brow[3] == brow[2];

        float acc[V], head[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            acc[v] = 0.0f;
            head[v] = 0.0f;
        }
        int cur_row = -1, cur_slot = -1, head_row = -1;
        bool first_seg = true;
        const int steps = (int)(q + (rm > 0 ? 1 : 0));
        const bool remap_inline = a.rec_out != nullptr;

        // One step: commit the record fetched for this step (remap store,
        // decode), prefetch the next step's record into the other buffer
        // after the first gathers, then run the lane groups over their L
        // nonzeros of this step.  Two record buffers alternate, so a prefetch
        // never overwrites the registers of a remap store still in flight.
        Rec<RW> ra, rb;
        int32_t na = 0, nb = 0;
        if (li < gn) {
            load_rec<RW>(a.rec_in, gs + li, ra);
            if (remap_inline) na = a.nxt[gs + li];
        }
        // the lane's record: indices in rotated mode order (w[k] = index of
        // mode (d + k) mod N), then the value's bits and the carry slot
        Words<N> mine;
#pragma unroll
        for (int k = 0; k < N + 2; ++k) mine.w[k] = 0u;
        auto step = [&](int step0, Rec<RW>& cur, int32_t& ncur, Rec<RW>& nxt_rec, int32_t& nnext) {
            if (step0 + li < gn) {
                if (remap_inline) store_rec<RW>(a.rec_out, ncur, cur);
                Words<N> dec;
                decode_words<RW, KIND>(cur, a, dec, seq);
#pragma unroll
                for (int k = 0; k < N; ++k) mine.w[k] = pick_word(dec, a.rot[k]);
                mine.w[N] = rword<RW - 1, RW>(cur);
            }
            // every lane (the lookup reads other lanes); lanes past the
            // group's range look up a stale row and never use it
            mine.w[N + 1] = (uint32_t)slot_of(mine.w[0]);
            const int cnt = gn - step0;
#pragma unroll
            for (int kb = 0; kb < L; kb += B) {
                // each gathered row: its LDS slot (with kHot) when it is hot,
                // else its row in memory
                uint32_t c[B][NG];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int src = g * L + kb + b;
#pragma unroll
                    for (int k = 0; k < NG; ++k) {
                        const uint32_t row = lane_get(mine.w[k + 1], src);
                        const int h = a.hot_h[k + 1];
                        uint32_t cc = row;
                        if (h > 0) {
                            if (a.hot_full[k + 1]) {
                                cc = kHot | row;
                            } else {
                                const uint32_t sl = hot_slot(row, (uint32_t)h);
                                if (tags[a.hot_tag_off[k + 1] + sl] == (int32_t)row) cc = kHot | sl;
                            }
                        }
                        c[b][k] = cc;
                    }
                }
                uint4 y[B][NG];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const bool live = kb + b < cnt;
#pragma unroll
                    for (int k = 0; k < NG; ++k) {
                        if (live) {
                            if (c[b][k] & kHot)
                                y[b][k] = hot_lds[a.hot_row_off[k + 1] + (int)(c[b][k] & ~kHot) * RQ + li];
                            else
                                y[b][k] = static_cast<const uint4*>(a.fac[k + 1])[(int64_t)c[b][k] * RQ + li];
                        }
                    }
                }
                if (kb == 0 && step0 + L + li < gn) {
                    load_rec<RW>(a.rec_in, gs + step0 + L + li, nxt_rec);
                    if (remap_inline) nnext = a.nxt[gs + step0 + L + li];
                }
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int src = g * L + kb + b;
                    const int row = (int)lane_get(mine.w[0], src);
                    const float val = __uint_as_float(lane_get(mine.w[N], src));
                    const int rslot = (int)lane_get(mine.w[N + 1], src);
                    if (kb + b < cnt) {
                        if (row != cur_row) {
                            if (cur_row >= 0) {
                                if (first_seg && open_left) {
#pragma unroll
                                    for (int v = 0; v < V; ++v) head[v] = acc[v];
                                    head_row = cur_row;
                                } else {
                                    store_vals<V>(row_dst<R>(a, cur_row, cur_slot) + li * V, acc);
                                }
                                first_seg = false;
                            }
                            cur_row = row;
                            cur_slot = rslot;
#pragma unroll
                            for (int v = 0; v < V; ++v) acc[v] = 0.0f;
                        }
                        float prod[V];
                        widen<FT>(y[b][0], prod);
#pragma unroll
                        for (int k = 1; k < NG; ++k) {
                            float f[V];
                            widen<FT>(y[b][k], f);
#pragma unroll
                            for (int v = 0; v < V; ++v) prod[v] *= f[v];
                        }
#pragma unroll
                        for (int v = 0; v < V; ++v) acc[v] = fmaf(prod[v], val, acc[v]);
                    }
                }
            }
        };
        for (int t = 0; t < steps; t += 2 * L) {
            step(t, ra, na, rb, nb);
            if (t + L < steps) step(t + L, rb, nb, ra, na);
        }

        // the group's last segment: kept (the tail) when the next group or
        // the head chain continues it, else stored
        int tail_row = -1, tail_slot = -1;
        if (cur_row >= 0) {
            if (open_right || (first_seg && open_left)) {
                tail_row = cur_row;
                tail_slot = cur_slot;
            } else {
                store_vals<V>(row_dst<R>(a, cur_row, cur_slot) + li * V, acc);
            }
        }

        // chain combine across groups in group order (every group computes
        // it, group 0 stores): a row that crosses sub-range boundaries is the
        // tail of one group, whole groups, and the head of another
        const int flags = (open_left ? 1 : 0) | (open_right ? 2 : 0) | (gn > 0 ? 4 : 0);
        float csum[V];
#pragma unroll
        for (int v = 0; v < V; ++v) csum[v] = 0.0f;
        int crow = -1, cslot = -1;
        auto flush = [&]() {
            if (crow >= 0 && g == 0) store_vals<V>(row_dst<R>(a, crow, cslot) + li * V, csum);
        };
        for (int h = 0; h < G; ++h) {
            const int f = (int)lane_get((uint32_t)flags, h * L);
            const int hr = (int)lane_get((uint32_t)head_row, h * L);
            const int tr = (int)lane_get((uint32_t)tail_row, h * L);
            const int ts = (int)lane_get((uint32_t)tail_slot, h * L);
            float hv[V], tv[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                hv[v] = lane_get(head[v], h * L + li);
                tv[v] = lane_get(acc[v], h * L + li);
            }
            if (!(f & 4)) continue;
            if (f & 1) {
                if (hr >= 0) {
#pragma unroll
                    for (int v = 0; v < V; ++v) csum[v] += hv[v];
                    flush();
                    crow = -1;
#pragma unroll
                    for (int v = 0; v < V; ++v) csum[v] = 0.0f;
                    if (tr >= 0) {
                        crow = tr;
                        cslot = ts;
#pragma unroll
                        for (int v = 0; v < V; ++v) csum[v] = tv[v];
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) csum[v] += tv[v];
                    if (!(f & 2)) {
                        flush();
                        crow = -1;
#pragma unroll
                        for (int v = 0; v < V; ++v) csum[v] = 0.0f;
                    }
                }
            } else if (tr >= 0) {
                crow = tr;
                cslot = ts;
#pragma unroll
                for (int v = 0; v < V; ++v) csum[v] = tv[v];
            }
        }
    }  // partitions
}

using EcFn = EcFnPtr;

template <int N, int RW, int KIND>
EcFn pick_rank(int rank, int fdtype) {
    if (fdtype == 0) {
        switch (rank) {
            case 8: return ec_kernel<N, 8, RW, KIND, FacF32, ec_waves(N, 8, 4)>;
            case 16: return ec_kernel<N, 16, RW, KIND, FacF32, ec_waves(N, 16, 4)>;
            case 32: return ec_kernel<N, 32, RW, KIND, FacF32, ec_waves(N, 32, 4)>;
            case 64: return ec_kernel<N, 64, RW, KIND, FacF32, ec_waves(N, 64, 4)>;
            case 128: return ec_kernel<N, 128, RW, KIND, FacF32, ec_waves(N, 128, 4)>;
            default: return nullptr;
        }
    }
    switch (rank) {
        case 8: return ec_kernel<N, 8, RW, KIND, FacBF16, ec_waves(N, 8, 2)>;
        case 16: return ec_kernel<N, 16, RW, KIND, FacBF16, ec_waves(N, 16, 2)>;
        case 32: return ec_kernel<N, 32, RW, KIND, FacBF16, ec_waves(N, 32, 2)>;
        case 64: return ec_kernel<N, 64, RW, KIND, FacBF16, ec_waves(N, 64, 2)>;
        case 128: return ec_kernel<N, 128, RW, KIND, FacBF16, ec_waves(N, 128, 2)>;
        default: return nullptr;
    }
}

// (record words, layout kind) pairs the planner can choose for N modes
template <int N>
EcFn pick_layout(int rank, int fdtype, int words, int kind) {
    if constexpr (N <= 3) {
        if (words == 4 && kind == kWord32) return pick_rank<N, 4, kWord32>(rank, fdtype);
    } else if constexpr (N <= 6) {
        if (words == 4 && kind == kHalf16) return pick_rank<N, 4, kHalf16>(rank, fdtype);
        if (words == 4 && kind == kPacked) return pick_rank<N, 4, kPacked>(rank, fdtype);
        if (words == 8 && kind == kWord32) return pick_rank<N, 8, kWord32>(rank, fdtype);
    } else if constexpr (N == 7) {
        if (words == 8 && kind == kWord32) return pick_rank<N, 8, kWord32>(rank, fdtype);
    } else {
        if (words == 8 && kind == kHalf16) return pick_rank<N, 8, kHalf16>(rank, fdtype);
        if (words == 12 && kind == kWord32) return pick_rank<N, 12, kWord32>(rank, fdtype);
    }
    return nullptr;
}

}  // namespace
}  // namespace spt
