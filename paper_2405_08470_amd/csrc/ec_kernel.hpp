// Fused elementwise computation (Alg. 2) and dynamic remapping (Alg. 3) for
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
#include "record.hpp"

// float4 gathers a lane keeps in flight (register budget of the batch)
#ifndef SPT_GATHER_INFLIGHT
#define SPT_GATHER_INFLIGHT 16
#endif
namespace spt {
namespace {

// Index of mode W in a record (layout kinds of the planner).
template <int W, int RW, int KIND>
__device__ __forceinline__ uint32_t decode(const Rec<RW>& r, const EcArgs& a) {
    if constexpr (KIND == kWord32) {
        return rword<W, RW>(r);
    } else if constexpr (KIND == kHalf16) {
        return (rword<W / 2, RW>(r) >> ((W & 1) * 16)) & 0xFFFFu;
    } else {  // bit fields in the first 64 bits (12-byte record) or 96 bits (16-byte)
        const uint64_t lo = ((uint64_t)rword<1, RW>(r) << 32) | rword<0, RW>(r);
        const int o = a.foff[W];
        if constexpr (RW == 3) {
            return (uint32_t)(lo >> o) & a.fmask[W];
        } else {
            const uint64_t hi = rword<2, RW>(r);
            const uint64_t x = o >= 64 ? (hi >> (o - 64)) : ((lo >> o) | (o ? (hi << (64 - o)) : 0));
            return (uint32_t)x & a.fmask[W];
        }
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

// REUSE: the last gathered mode's row (mode d-1, the second key of mode d's
// stream order, so consecutive nonzeros often share it) is fetched once per
// run of consecutive nonzeros that share it and their output row and kept in
// registers; every nonzero still multiplies it into its product in the same
// order, so both forms give the same bits.  Without REUSE every nonzero
// fetches all its gathered rows.  REUSE costs registers; the launch takes it
// only where it keeps the occupancy.
template <int N, int R, int RW, int KIND, typename FT, bool REUSE>
__global__ __launch_bounds__(64) void ec_kernel(const EcArgs a) {
    constexpr int V = FT::kPerLoad;
    constexpr int L = R / V;     // lanes per nonzero
    constexpr int G = 64 / L;    // lane groups = nonzeros in flight
    constexpr int NG = N - 1;    // gathered factor rows per nonzero
    // nonzeros whose gathers are issued together: the largest divisor of L
    // with at most SPT_GATHER_INFLIGHT float4 gathers in flight per lane
    constexpr int BMAX = (SPT_GATHER_INFLIGHT / NG) > 0 ? SPT_GATHER_INFLIGHT / NG : 1;
    constexpr int B = L <= BMAX ? L : (L / 2 <= BMAX ? L / 2 : (L / 4 <= BMAX ? L / 4 : (L / 8 <= BMAX ? L / 8 : 1)));
    static_assert(R % V == 0 && L >= 1 && 64 % L == 0 && L % B == 0, "rank");
    // staged words per nonzero: indices in mode order, value, carry slot
    constexpr int SW = N + 2;
    constexpr int MAXSPLIT = 64;  // split rows of a partition kept in LDS

    __shared__ uint32_t stage[SW][64];
    __shared__ float part[2][G][R];   // [0] head, [1] tail partial of a group
    __shared__ int32_t prow[2][G];
    __shared__ int32_t pslot[2][G];
    __shared__ int32_t gflag[G];      // bit 0 open-left, bit 1 open-right, bit 2 non-empty
    __shared__ uint32_t brow[G][4];   // rows at the sub-range boundaries
    __shared__ int32_t srow[MAXSPLIT], sslot[MAXSPLIT];

    const int z = blockIdx.x;
    const int lane = threadIdx.x;
    const int g = lane / L;
    const int li = lane % L;
    const int64_t s = a.ptr[z];
    const int64_t n = a.ptr[z + 1] - s;
    if (n == 0) return;
    const int sp0 = a.psplit_ptr[z], sp1 = a.psplit_ptr[z + 1];
    const int nsp = sp1 - sp0;
    const bool sp_lds = nsp <= MAXSPLIT;
    if (sp_lds && lane < nsp) {
        srow[lane] = a.psplit_row[sp0 + lane];
        sslot[lane] = a.psplit_slot[sp0 + lane];
    }
    const int mode = a.rot[0];
    constexpr auto seq = std::make_integer_sequence<int, N>{};

    const int64_t q = n / G, rm = n % G;
    const int64_t gs = s + g * q + (g < rm ? g : rm);
    const int gn = (int)(q + (g < rm ? 1 : 0));
    const int64_t ge = gs + gn;

    // output rows around the group's sub-range: before, first, last, after
    for (int j = li; j < 4; j += L) {
        const int64_t p = j == 0 ? gs - 1 : j == 1 ? gs : j == 2 ? ge - 1 : ge;
        uint32_t row = 0xFFFFFFFFu;
        if (gn > 0 && p >= s && p < s + n) {
            Rec<RW> r;
            load_rec<RW>(a.rec_in, p, r);
            decode_all<RW, KIND>(r, a, stage, lane, seq);
            row = stage[mode][lane];
        }
        brow[g][j] = row;
    }
    __syncthreads();
    const bool open_left = gn > 0 && brow[g][0] != 0xFFFFFFFFu && brow[g][0] == brow[g][1];
    const bool open_right = gn > 0 && brow[g][3] != 0xFFFFFFFFu && brow[g][3] == brow[g][2];
    if (li == 0) {
        gflag[g] = (open_left ? 1 : 0) | (open_right ? 2 : 0) | (gn > 0 ? 4 : 0);
        prow[0][g] = -1;
        prow[1][g] = -1;
    }
    __syncthreads();

    // acc: the output row's sum so far; ylast (REUSE): the last gathered
    // mode's row of the current run of equal (output row, last gathered row)
    float acc[V], ylast[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        acc[v] = 0.0f;
        ylast[v] = 0.0f;
    }
    int cur_row = -1, cur_slot = -1;
    uint32_t cur_lrow = 0xFFFFFFFFu;  // last gathered mode's row of the current run
    bool first_seg = true;
    const int steps = (int)(q + (rm > 0 ? 1 : 0));
    const bool remap = a.rec_out != nullptr;
    const bool remap_inline = remap;

    // carry slot of a row of this partition (-1: not a split row)
    auto slot_of = [&](int row) {
        int slot = -1;
        if (sp_lds) {
            for (int j = 0; j < nsp; ++j)
                if (srow[j] == row) slot = sslot[j];
        } else {
            slot = split_slot(a, sp0, sp1, row);
        }
        return slot;
    };

    // One step: commit the record fetched for this step (remap store,
    // decode), prefetch the next step's record into the other buffer after
    // the first gathers, then run the lane groups over their L nonzeros of
    // this step.  Two record buffers alternate, so a prefetch never
    // overwrites the registers of a remap store still in flight.
    Rec<RW> ra, rb;
    int32_t na = 0, nb = 0;
    if (li < gn) {
        load_rec<RW>(a.rec_in, gs + li, ra);
        if (remap_inline) na = a.nxt[gs + li];
    }
    auto step = [&](int step0, Rec<RW>& cur, int32_t& ncur, Rec<RW>& nxt_rec, int32_t& nnext) {
        if (step0 + li < gn) {
            if (remap_inline) store_rec<RW>(a.rec_out, ncur, cur);
            decode_all<RW, KIND>(cur, a, stage, lane, seq);
            stage[N][lane] = rword<RW - 1, RW>(cur);
            stage[N + 1][lane] = (uint32_t)slot_of((int)stage[mode][lane]);
        }
        __syncthreads();
        const int cnt = gn - step0;
        #pragma unroll
        for (int kb = 0; kb < L; kb += B) {
            // the batch's rows first (one LDS wait for all of them), then its
            // gathers back to back; a nonzero past the group's range gathers
            // row 0 (always a valid row) instead of branching around the load
            uint32_t orow[B], rix[B][NG];
            #pragma unroll
            for (int b = 0; b < B; ++b) {
                const int slot = g * L + kb + b;
                orow[b] = stage[mode][slot];
                #pragma unroll
                for (int k = 0; k < NG; ++k) rix[b][k] = stage[a.rot[k + 1]][slot];
            }
            // the last gathered mode's row is fetched only where a run of
            // equal (output row, last gathered row) starts: the same test the
            // accumulation below makes, against the previous nonzero
            bool fresh[B];
            #pragma unroll
            for (int b = 0; b < B; ++b) {
                const uint32_t po = b == 0 ? (uint32_t)cur_row : orow[b - 1];
                const uint32_t pl = b == 0 ? cur_lrow : rix[b - 1][NG - 1];
                fresh[b] = !REUSE || orow[b] != po || rix[b][NG - 1] != pl;
            }
            uint4 y[B][NG];
            #pragma unroll
            for (int b = 0; b < B; ++b) {
                const bool live = kb + b < cnt;
                #pragma unroll
                for (int k = 0; k < NG; ++k) {
                    const uint4* src = reinterpret_cast<const uint4*>(
                        static_cast<const char*>(a.fac[k + 1]) +
                        ((int64_t)(live ? rix[b][k] : 0u) * R + li * V) * FT::kBytes);
                    if (!REUSE || k < NG - 1) {
                        y[b][k] = *src;
                    } else if (live && fresh[b]) {
                        y[b][k] = *src;
                    }
                }
            }
            if (kb == 0 && step0 + L + li < gn) {
                load_rec<RW>(a.rec_in, gs + step0 + L + li, nxt_rec);
                if (remap_inline) nnext = a.nxt[gs + step0 + L + li];
            }
            #pragma unroll
            for (int b = 0; b < B; ++b) {
                if (kb + b < cnt) {
                    const int slot = g * L + kb + b;
                    const int row = (int)orow[b];
                    if (REUSE && fresh[b]) {
                        widen<FT>(y[b][NG - 1], ylast);
                        cur_lrow = rix[b][NG - 1];
                    }
                    if (row != cur_row) {
                        if (cur_row >= 0) {
                            if (first_seg && open_left) {
                                store_vals<V>(&part[0][g][li * V], acc);
                                if (li == 0) {
                                    prow[0][g] = cur_row;
                                    pslot[0][g] = cur_slot;
                                }
                            } else {
                                store_vals<V>(row_dst<R>(a, cur_row, cur_slot) + li * V, acc);
                            }
                            first_seg = false;
                        }
                        cur_row = row;
                        cur_slot = (int)stage[N + 1][slot];
                        #pragma unroll
                        for (int v = 0; v < V; ++v) acc[v] = 0.0f;
                    }
                    const float val = __uint_as_float(stage[N][slot]);
                    if constexpr (REUSE) {
                        // the product of the gathered rows in mode order, the
                        // last one from the registers of its run
                        float prod[V];
                        if constexpr (NG == 1) {
                            #pragma unroll
                            for (int v = 0; v < V; ++v) prod[v] = ylast[v];
                        } else {
                            widen<FT>(y[b][0], prod);
                            #pragma unroll
                            for (int k = 1; k < NG - 1; ++k) {
                                float f[V];
                                widen<FT>(y[b][k], f);
                                #pragma unroll
                                for (int v = 0; v < V; ++v) prod[v] *= f[v];
                            }
                            #pragma unroll
                            for (int v = 0; v < V; ++v) prod[v] *= ylast[v];
                        }
                        #pragma unroll
                        for (int v = 0; v < V; ++v) acc[v] = fmaf(prod[v], val, acc[v]);
                    } else {
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
        }
        __syncthreads();
    
    };
    for (int t = 0; t < steps; t += 2 * L) {
        step(t, ra, na, rb, nb);
        if (t + L < steps) step(t + L, rb, nb, ra, na);
    }

    // the group's last segment
    if (cur_row >= 0) {
        if (open_right || (first_seg && open_left)) {
            store_vals<V>(&part[1][g][li * V], acc);
            if (li == 0) {
                prow[1][g] = cur_row;
                pslot[1][g] = cur_slot;
            }
        } else {
            store_vals<V>(row_dst<R>(a, cur_row, cur_slot) + li * V, acc);
        }
    }
    __syncthreads();

    // chain combine across groups, lanes over ranks, in group order
    for (int r0 = 0; r0 < R; r0 += 64) {
        const int rk = r0 + lane;
        const bool active = rk < R;
        float csum = 0.0f;
        int crow = -1, cslot = -1;
        for (int h = 0; h < G; ++h) {
            const int f = gflag[h];
            if (!(f & 4)) continue;
            const bool ol = f & 1, orr = f & 2;
            auto flush = [&](int row, int slot, float x) {
                if (row < 0) return;
                if (active) row_dst<R>(a, row, slot)[rk] = x;
            };
            if (ol) {
                if (prow[0][h] >= 0) {
                    csum += active ? part[0][h][rk] : 0.0f;
                    flush(crow, cslot, csum);
                    crow = -1;
                    csum = 0.0f;
                    if (prow[1][h] >= 0) {
                        crow = prow[1][h];
                        cslot = pslot[1][h];
                        csum = active ? part[1][h][rk] : 0.0f;
                    }
                } else {
                    csum += active ? part[1][h][rk] : 0.0f;
                    if (!orr) {
                        flush(crow, cslot, csum);
                        crow = -1;
                        csum = 0.0f;
                    }
                }
            } else if (prow[1][h] >= 0) {
                crow = prow[1][h];
                cslot = pslot[1][h];
                csum = active ? part[1][h][rk] : 0.0f;
            }
        }
    }
}

using EcFn = EcFnPtr;

template <int N, int RW, int KIND, bool REUSE>
EcFn pick_rank(int rank, int fdtype) {
    if (fdtype == 0) {
        switch (rank) {
            case 8: return ec_kernel<N, 8, RW, KIND, FacF32, REUSE>;
            case 16: return ec_kernel<N, 16, RW, KIND, FacF32, REUSE>;
            case 32: return ec_kernel<N, 32, RW, KIND, FacF32, REUSE>;
            case 64: return ec_kernel<N, 64, RW, KIND, FacF32, REUSE>;
            case 128: return ec_kernel<N, 128, RW, KIND, FacF32, REUSE>;
            default: return nullptr;
        }
    }
    switch (rank) {
        case 8: return ec_kernel<N, 8, RW, KIND, FacBF16, REUSE>;
        case 16: return ec_kernel<N, 16, RW, KIND, FacBF16, REUSE>;
        case 32: return ec_kernel<N, 32, RW, KIND, FacBF16, REUSE>;
        case 64: return ec_kernel<N, 64, RW, KIND, FacBF16, REUSE>;
        case 128: return ec_kernel<N, 128, RW, KIND, FacBF16, REUSE>;
        default: return nullptr;
    }
}

template <int N, int RW, int KIND>
EcFn pick_rank(int rank, int fdtype, bool reuse) {
    return reuse ? pick_rank<N, RW, KIND, true>(rank, fdtype) : pick_rank<N, RW, KIND, false>(rank, fdtype);
}

// (record words, layout kind) pairs the planner can choose for N modes
template <int N>
EcFn pick_layout(int rank, int fdtype, int words, int kind, bool reuse) {
    if constexpr (N <= 2) {
        if (words == 3 && kind == kWord32) return pick_rank<N, 3, kWord32>(rank, fdtype, reuse);
        if (words == 4 && kind == kWord32) return pick_rank<N, 4, kWord32>(rank, fdtype, reuse);
    } else if constexpr (N == 3) {
        if (words == 3 && kind == kPacked) return pick_rank<N, 3, kPacked>(rank, fdtype, reuse);
        if (words == 4 && kind == kWord32) return pick_rank<N, 4, kWord32>(rank, fdtype, reuse);
    } else if constexpr (N <= 6) {
        if constexpr (N == 4)
            if (words == 3 && kind == kHalf16) return pick_rank<N, 3, kHalf16>(rank, fdtype, reuse);
        if (words == 3 && kind == kPacked) return pick_rank<N, 3, kPacked>(rank, fdtype, reuse);
        if (words == 4 && kind == kHalf16) return pick_rank<N, 4, kHalf16>(rank, fdtype, reuse);
        if (words == 4 && kind == kPacked) return pick_rank<N, 4, kPacked>(rank, fdtype, reuse);
        if (words == 8 && kind == kWord32) return pick_rank<N, 8, kWord32>(rank, fdtype, reuse);
    } else if constexpr (N == 7) {
        if (words == 3 && kind == kPacked) return pick_rank<N, 3, kPacked>(rank, fdtype, reuse);
        if (words == 8 && kind == kWord32) return pick_rank<N, 8, kWord32>(rank, fdtype, reuse);
    } else {
        if (words == 3 && kind == kPacked) return pick_rank<N, 3, kPacked>(rank, fdtype, reuse);
        if (words == 8 && kind == kHalf16) return pick_rank<N, 8, kHalf16>(rank, fdtype, reuse);
        if (words == 12 && kind == kWord32) return pick_rank<N, 12, kWord32>(rank, fdtype, reuse);
    }
    return nullptr;
}

}  // namespace
}  // namespace spt
