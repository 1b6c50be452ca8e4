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
// Records are fetched 64 at a time, one per lane, which is also where each
// record is written to its remap position in the next mode's stream
// (Alg. 3): consecutive records bound for the same (row, source partition)
// in the next stream land in consecutive slots.
#include <algorithm>

#include "kernels.hpp"

namespace spt {

namespace {

template <int W>
__device__ __forceinline__ uint32_t pick_word(const uint32_t (&r)[W], int k) {
    uint32_t v = r[0];
#pragma unroll
    for (int i = 1; i < W; ++i) v = (k == i) ? r[i] : v;
    return v;
}

template <int RW>
__device__ __forceinline__ uint32_t field(const uint32_t (&r)[RW], int wi, int sh, uint32_t mask) {
    // indices occupy words 0 .. RW-2; word RW-1 is the value
    uint32_t lo = pick_word<RW - 1>(reinterpret_cast<const uint32_t(&)[RW - 1]>(r), wi);
    uint32_t hi = pick_word<RW - 1>(reinterpret_cast<const uint32_t(&)[RW - 1]>(r), wi + 1);
    hi = (wi + 1 < RW - 1) ? hi : 0u;
    return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)sh) & mask;
}

template <int RW>
__device__ __forceinline__ void load_record(const uint32_t* __restrict__ base, int64_t p,
                                            uint32_t (&r)[RW]) {
    const uint4* q = reinterpret_cast<const uint4*>(base + p * RW);
#pragma unroll
    for (int k = 0; k < RW / 4; ++k) {
        uint4 v = q[k];
        r[4 * k + 0] = v.x;
        r[4 * k + 1] = v.y;
        r[4 * k + 2] = v.z;
        r[4 * k + 3] = v.w;
    }
}

template <int RW>
__device__ __forceinline__ void store_record(uint32_t* __restrict__ base, int64_t p,
                                             const uint32_t (&r)[RW]) {
    uint4* q = reinterpret_cast<uint4*>(base + p * RW);
#pragma unroll
    for (int k = 0; k < RW / 4; ++k)
        q[k] = make_uint4(r[4 * k + 0], r[4 * k + 1], r[4 * k + 2], r[4 * k + 3]);
}

// Carry slot of `row` if it is a split row of this partition, else -1.
__device__ __forceinline__ int split_slot(const EcArgs& a, int sp0, int sp1, int row) {
    int slot = -1;
    for (int j = sp0; j < sp1; ++j)
        if (a.psplit_row[j] == row) slot = a.psplit_slot[j];
    return slot;
}

template <int N, int R, int RW>
__global__ __launch_bounds__(64) void ec_kernel(const EcArgs a) {
    constexpr int V = 4;
    constexpr int L = R / V;     // lanes per nonzero
    constexpr int G = 64 / L;    // lane groups = nonzeros in flight
    constexpr int SW = N + 1;    // staged words: rotated indices, value
    static_assert(R % V == 0 && 64 % L == 0, "rank");

    __shared__ uint32_t stage[SW][64];
    __shared__ float part[2][G][R];   // [0] head, [1] tail partial of a group
    __shared__ int32_t prow[2][G];
    __shared__ int32_t gflag[G];      // bit 0 open-left, bit 1 open-right, bit 2 non-empty

    const int z = blockIdx.x;
    const int lane = threadIdx.x;
    const int g = lane / L;
    const int li = lane % L;
    const int64_t s = a.ptr[z];
    const int64_t n = a.ptr[z + 1] - s;
    if (n == 0) return;
    const int sp0 = a.psplit_ptr[z], sp1 = a.psplit_ptr[z + 1];

    const int64_t q = n / G, rm = n % G;
    const int64_t gs = s + g * q + (g < rm ? g : rm);
    const int64_t gn = q + (g < rm ? 1 : 0);
    const int64_t ge = gs + gn;

    // Does the group's first / last row continue from / into a neighbour?
    bool open_left = false, open_right = false;
    if (gn > 0) {
        uint32_t r0[RW], r1[RW];
        load_record<RW>(a.rec_in, gs, r0);
        load_record<RW>(a.rec_in, ge - 1, r1);
        const uint32_t first_row = field<RW>(r0, a.fword[0], a.fshift[0], a.fmask[0]);
        const uint32_t last_row = field<RW>(r1, a.fword[0], a.fshift[0], a.fmask[0]);
        if (gs > s) {
            uint32_t rp[RW];
            load_record<RW>(a.rec_in, gs - 1, rp);
            open_left = field<RW>(rp, a.fword[0], a.fshift[0], a.fmask[0]) == first_row;
        }
        if (ge < s + n) {
            uint32_t rn[RW];
            load_record<RW>(a.rec_in, ge, rn);
            open_right = field<RW>(rn, a.fword[0], a.fshift[0], a.fmask[0]) == last_row;
        }
    }
    if (li == 0) {
        gflag[g] = (open_left ? 1 : 0) | (open_right ? 2 : 0) | (gn > 0 ? 4 : 0);
        prow[0][g] = -1;
        prow[1][g] = -1;
    }

    float acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0f;
    int cur_row = -1;
    bool first_seg = true;
    const int64_t steps = q + (rm > 0 ? 1 : 0);

    for (int64_t t = 0; t < steps; t += L) {
        // stage: lane li of group g fetches nonzero gs + t + li
        if (t + li < gn) {
            const int64_t p = gs + t + li;
            uint32_t r[RW];
            load_record<RW>(a.rec_in, p, r);
            if (a.rec_out) store_record<RW>(a.rec_out, a.nxt[p], r);
#pragma unroll
            for (int k = 0; k < N; ++k)
                stage[k][lane] = field<RW>(r, a.fword[k], a.fshift[k], a.fmask[k]);
            stage[N][lane] = r[RW - 1];
        }
        __syncthreads();
        const int64_t cnt = gn - t;
#pragma unroll
        for (int kk = 0; kk < L; ++kk) {
            if (kk < cnt) {
                const int slot = g * L + kk;
                const int row = (int)stage[0][slot];
                if (row != cur_row) {
                    if (cur_row >= 0) {
                        if (first_seg && open_left) {
#pragma unroll
                            for (int v = 0; v < V; ++v) part[0][g][li * V + v] = acc[v];
                            if (li == 0) prow[0][g] = cur_row;
                        } else {
                            const int sl = split_slot(a, sp0, sp1, cur_row);
                            float* dst = sl >= 0 ? a.carry + (int64_t)sl * R
                                                 : a.out + (int64_t)cur_row * R;
                            *reinterpret_cast<float4*>(dst + li * V) =
                                make_float4(acc[0], acc[1], acc[2], acc[3]);
                        }
                        first_seg = false;
                    }
                    cur_row = row;
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[v] = 0.0f;
                }
                const float val = __uint_as_float(stage[N][slot]);
                float4 prod = *reinterpret_cast<const float4*>(
                    a.fac[1] + (int64_t)stage[1][slot] * R + li * V);
#pragma unroll
                for (int k = 2; k < N; ++k) {
                    const float4 y = *reinterpret_cast<const float4*>(
                        a.fac[k] + (int64_t)stage[k][slot] * R + li * V);
                    prod.x *= y.x;
                    prod.y *= y.y;
                    prod.z *= y.z;
                    prod.w *= y.w;
                }
                acc[0] = fmaf(prod.x, val, acc[0]);
                acc[1] = fmaf(prod.y, val, acc[1]);
                acc[2] = fmaf(prod.z, val, acc[2]);
                acc[3] = fmaf(prod.w, val, acc[3]);
            }
        }
        __syncthreads();
    }

    // the group's last segment
    if (cur_row >= 0) {
        if (open_right || (first_seg && open_left)) {
#pragma unroll
            for (int v = 0; v < V; ++v) part[1][g][li * V + v] = acc[v];
            if (li == 0) prow[1][g] = cur_row;
        } else {
            const int sl = split_slot(a, sp0, sp1, cur_row);
            float* dst = sl >= 0 ? a.carry + (int64_t)sl * R : a.out + (int64_t)cur_row * R;
            *reinterpret_cast<float4*>(dst + li * V) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        }
    }
    __syncthreads();

    // chain combine across groups, lanes over ranks, in group order
    for (int r0 = 0; r0 < R; r0 += 64) {
        const int rk = r0 + lane;
        const bool active = rk < R;
        float csum = 0.0f;
        int crow = -1;
        for (int h = 0; h < G; ++h) {
            const int f = gflag[h];
            if (!(f & 4)) continue;
            const bool ol = f & 1, orr = f & 2;
            auto flush = [&](int row, float x) {
                if (row < 0) return;
                const int sl = split_slot(a, sp0, sp1, row);
                float* dst = sl >= 0 ? a.carry + (int64_t)sl * R : a.out + (int64_t)row * R;
                if (active) dst[rk] = x;
            };
            if (ol) {
                if (prow[0][h] >= 0) {
                    csum += active ? part[0][h][rk] : 0.0f;
                    flush(crow, csum);
                    crow = -1;
                    csum = 0.0f;
                    if (prow[1][h] >= 0) {
                        crow = prow[1][h];
                        csum = active ? part[1][h][rk] : 0.0f;
                    }
                } else {
                    csum += active ? part[1][h][rk] : 0.0f;
                    if (!orr) {
                        flush(crow, csum);
                        crow = -1;
                        csum = 0.0f;
                    }
                }
            } else if (prow[1][h] >= 0) {
                crow = prow[1][h];
                csum = active ? part[1][h][rk] : 0.0f;
            }
        }
    }
}

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

template <int RW>
__global__ void remap_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                             int64_t nnz, NxtChain ch, int hops) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = p;
        for (int h = 0; h < hops; ++h) d = ch.nxt[h][d];
        uint32_t r[RW];
        load_record<RW>(in, p, r);
        store_record<RW>(out, d, r);
    }
}

template <int N, int R, int RW>
void launch_one(int kappa, const EcArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((ec_kernel<N, R, RW>), dim3(kappa), dim3(64), 0, s, a);
}

template <int N, int RW>
bool by_rank(int rank, int kappa, const EcArgs& a, hipStream_t s) {
    switch (rank) {
        case 8: launch_one<N, 8, RW>(kappa, a, s); return true;
        case 16: launch_one<N, 16, RW>(kappa, a, s); return true;
        case 32: launch_one<N, 32, RW>(kappa, a, s); return true;
        case 64: launch_one<N, 64, RW>(kappa, a, s); return true;
        case 128: launch_one<N, 128, RW>(kappa, a, s); return true;
        default: return false;
    }
}

template <int N>
bool by_words(int rank, int words, int kappa, const EcArgs& a, hipStream_t s) {
    if (words == 4) return by_rank<N, 4>(rank, kappa, a, s);
    if (words == 8) return by_rank<N, 8>(rank, kappa, a, s);
    return false;
}

}  // namespace

bool launch_ec(int nmodes, int rank, int words, int kappa, const EcArgs& a, hipStream_t s) {
    switch (nmodes) {
        case 2: return by_words<2>(rank, words, kappa, a, s);
        case 3: return by_words<3>(rank, words, kappa, a, s);
        case 4: return by_words<4>(rank, words, kappa, a, s);
        case 5: return by_words<5>(rank, words, kappa, a, s);
        case 6: return by_words<6>(rank, words, kappa, a, s);
        case 7: return by_words<7>(rank, words, kappa, a, s);
        case 8: return by_words<8>(rank, words, kappa, a, s);
        default: return false;
    }
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

void launch_remap(int words, int64_t nnz, const uint32_t* in, uint32_t* out,
                  const int32_t* const* nxt, int hops, hipStream_t s) {
    if (nnz == 0) return;
    NxtChain ch{};
    for (int h = 0; h < hops; ++h) ch.nxt[h] = nxt[h];
    const int threads = 256;
    const int64_t blocks = std::min<int64_t>((nnz + threads - 1) / threads, 8192);
    if (words == 4)
        hipLaunchKernelGGL((remap_kernel<4>), dim3((unsigned)blocks), dim3(threads), 0, s, in, out,
                           nnz, ch, hops);
    else
        hipLaunchKernelGGL((remap_kernel<8>), dim3((unsigned)blocks), dim3(threads), 0, s, in, out,
                           nnz, ch, hops);
}

}  // namespace spt
