// Dynamic remapping (Alg. 3) as its own pass, chunk by chunk in destination
// order.
//
// The fused form stores each record at its next-mode position while the
// elementwise computation runs (one 16-byte store to a random address per
// nonzero).  Here the stream is cut into chunks of C consecutive records, and
// the records of each chunk are written in the order of their destinations:
// consecutive threads take consecutive table slots, so records of one chunk
// that land next to each other in the next mode's stream go out in the same
// store instruction and share memory transactions.  Each chunk (64 KB of
// records) is read in that order too; all workgroups of a chunk run on one XCD,
// so its lines are fetched once into that XCD's L2 and then hit there.  The next mode's stream is the same as the fused form's, bit for bit.
//
// Tables (built once at load, per mode d, from the next positions nxt_d):
//   ddst[c*C + j] = j-th smallest destination among the records of chunk c
//   doff[c*C + j] = offset inside chunk c of the record that goes there
// Destinations are distinct (nxt_d is a permutation), so the sorted order is
// unique and does not depend on how it is computed.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "kernels.hpp"

// Records per chunk for 16-byte records (32-byte: half, 48-byte: a quarter);
// a power of two.
#ifndef SPT_STAGE_CHUNK16
#define SPT_STAGE_CHUNK16 4096
#endif

namespace spt {
namespace {

constexpr int kStageThreads = 256;  // table sort
constexpr int kRemapThreads = 256;
constexpr int kChunk16 = SPT_STAGE_CHUNK16;
static_assert((kChunk16 & (kChunk16 - 1)) == 0 && kChunk16 >= 1024 && kChunk16 <= 16384, "chunk");

// One workgroup per chunk: bitonic sort of (destination, offset) pairs in LDS.
template <int C>
__global__ __launch_bounds__(kStageThreads) void stage_tables_kernel(const int32_t* __restrict__ nxt,
                                                                      int64_t nnz, int32_t* __restrict__ ddst,
                                                                      uint16_t* __restrict__ doff) {
    __shared__ int32_t key[C];
    __shared__ uint16_t pay[C];
    const int64_t base = (int64_t)blockIdx.x * C;
    const int cnt = (int)((nnz - base) < C ? (nnz - base) : C);
    for (int i = threadIdx.x; i < C; i += kStageThreads) {
        key[i] = i < cnt ? nxt[base + i] : INT_MAX;  // padding sorts last
        pay[i] = (uint16_t)i;
    }
    __syncthreads();
    for (int k = 2; k <= C; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < C; i += kStageThreads) {
                const int l = i ^ j;
                if (l > i) {
                    const bool ascending = (i & k) == 0;
                    const int32_t a = key[i], b = key[l];
                    if ((a > b) == ascending) {
                        key[i] = b;
                        key[l] = a;
                        const uint16_t t = pay[i];
                        pay[i] = pay[l];
                        pay[l] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < cnt; i += kStageThreads) {
        ddst[base + i] = key[i];
        doff[base + i] = pay[i];
    }
}

// One record per thread: slot j of the tables, read from its chunk in L2.
template <int RW, int C>
__global__ __launch_bounds__(kRemapThreads) void remap_flat_kernel(const uint32_t* __restrict__ in,
                                                                    uint32_t* __restrict__ out,
                                                                    const int32_t* __restrict__ ddst,
                                                                    const uint16_t* __restrict__ doff,
                                                                    int64_t nnz) {
    constexpr int Q = RW / 4;
    // the grid is a multiple of 8 chunks; block b runs on XCD b % 8 and takes
    // the (b / 8)-th block of that XCD's chunks c = x, x + 8, x + 16, ...
    constexpr unsigned BPC = C / kRemapThreads;  // workgroups per chunk
    const unsigned b = blockIdx.x, x = b % 8u, r = b / 8u;
    const unsigned v = ((r / BPC) * 8u + x) * BPC + r % BPC;
    const int64_t j = (int64_t)v * kRemapThreads + threadIdx.x;
    if (j >= nnz) return;
    const int64_t p = (j / C) * C + doff[j];
    const int64_t q = ddst[j];
    const uint4* src = reinterpret_cast<const uint4*>(in);
    uint4* dst = reinterpret_cast<uint4*>(out);
#pragma unroll
    for (int w = 0; w < Q; ++w) dst[q * Q + w] = src[p * Q + w];
}

}  // namespace

int stage_chunk(int words) {
    // 64 KB of LDS per workgroup at most; a power of two for the bitonic sort
    return words == 4 ? kChunk16 : words == 8 ? kChunk16 / 2 : kChunk16 / 4;
}

void launch_stage_tables(int words, const int32_t* nxt, int64_t nnz, int32_t* ddst, uint16_t* doff,
                         hipStream_t s) {
    if (nnz == 0) return;
    const int C = stage_chunk(words);
    const unsigned blocks = (unsigned)((nnz + C - 1) / C);
    if (C == kChunk16)
        hipLaunchKernelGGL(stage_tables_kernel<kChunk16>, dim3(blocks), dim3(kStageThreads), 0, s, nxt, nnz, ddst,
                           doff);
    else if (C == kChunk16 / 2)
        hipLaunchKernelGGL(stage_tables_kernel<kChunk16 / 2>, dim3(blocks), dim3(kStageThreads), 0, s, nxt, nnz,
                           ddst, doff);
    else
        hipLaunchKernelGGL(stage_tables_kernel<kChunk16 / 4>, dim3(blocks), dim3(kStageThreads), 0, s, nxt, nnz,
                           ddst, doff);
}

void launch_remap_staged(int words, int64_t nnz, const uint32_t* in, uint32_t* out, const int32_t* ddst,
                         const uint16_t* doff, hipStream_t s) {
    if (nnz == 0) return;
    const int C = stage_chunk(words);
    const int64_t nchunks = (nnz + C - 1) / C;
    const unsigned blocks = (unsigned)(((nchunks + 7) / 8) * 8 * (C / kRemapThreads));
    if (words == 4)
        hipLaunchKernelGGL((remap_flat_kernel<4, kChunk16>), dim3(blocks), dim3(kRemapThreads), 0, s, in, out,
                           ddst, doff, nnz);
    else if (words == 8)
        hipLaunchKernelGGL((remap_flat_kernel<8, kChunk16 / 2>), dim3(blocks), dim3(kRemapThreads), 0, s, in,
                           out, ddst, doff, nnz);
    else
        hipLaunchKernelGGL((remap_flat_kernel<12, kChunk16 / 4>), dim3(blocks), dim3(kRemapThreads), 0, s, in,
                           out, ddst, doff, nnz);
}

}  // namespace spt
