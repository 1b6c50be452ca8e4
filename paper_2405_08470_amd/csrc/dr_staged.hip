// Dynamic remapping (Alg. 3) as its own pass, chunk by chunk in destination
// order.
//
// The fused form stores each record at its next-mode position while the
// elementwise computation runs (one 12- or 16-byte store to a random address
// per nonzero).  Here the stream is cut into chunks of C consecutive records
// (the largest power of two of records within 2 MB: 131072 records of 12 or
// 16 bytes), and the records of each chunk are
// written in the order of their destinations: consecutive threads take
// consecutive table slots, so records of one chunk that land next to each
// other in the next mode's stream go out in the same store instruction and
// share cache lines.  In the next mode's order the records one source
// partition sends to one row are consecutive, so the longer the chunk, the
// longer these runs and the fewer lines the pass writes partially.  Each
// chunk is read in destination order too; all workgroups of a chunk run on one
// XCD, so its lines are fetched once into that XCD's L2 and then hit there.
// The next mode's stream is the same as the fused form's, bit for bit.
//
// Tables (built once at load, per mode d, from the next positions nxt_d):
//   ddst[c*C + j] = j-th smallest destination among the records of chunk c,
//                   in its low dbits bits (dbits = the bits of nnz - 1)
//   doff[c*C + j] = offset inside chunk c of the record that goes there: its
//                   low 16 bits; the offset's higher bits sit in ddst above
//                   the destination (chunks beyond 65536 records need them)
// Destinations are distinct (nxt_d is a permutation), so the sorted order is
// unique and does not depend on how it is computed: sub-runs of kSub records
// are sorted in LDS, then each chunk's sub-runs are merged by rank.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "kernels.hpp"
#include "record.hpp"

// Bytes of records per chunk (the chunk holds the largest power of two of
// records that fits, at least kSub, and no more than the bits ddst has to
// spare above the destinations can address).
#ifndef SPT_STAGE_CHUNK_BYTES
#define SPT_STAGE_CHUNK_BYTES (2 << 20)
#endif

namespace spt {
namespace {

constexpr int kStageThreads = 256;  // table sort
// remap workgroups of 16 waves: a quarter of the workgroups of 4-wave ones to
// dispatch for the same records (5-7 % faster per pass on the MI355X)
constexpr int kRemapThreads = 1024;
constexpr int kSub = 4096;           // entries sorted in LDS by one workgroup

// One workgroup per run of C consecutive entries: bitonic sort of (destination,
// offset) pairs in LDS.
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

// Merge of the sorted sub-runs of each chunk of 2^cshift entries: an entry's
// place in its chunk is its place in its own sub-run plus the number of
// smaller destinations in the chunk's other sub-runs (binary searches;
// destinations are distinct).  Offsets become offsets inside the chunk.
__global__ __launch_bounds__(kStageThreads) void merge_runs_kernel(const int32_t* __restrict__ sdst,
                                                                   const uint16_t* __restrict__ soff,
                                                                   int64_t nnz, int cshift, int dbits,
                                                                   int32_t* __restrict__ ddst,
                                                                   uint16_t* __restrict__ doff) {
    const int64_t i = blockIdx.x * (int64_t)kStageThreads + threadIdx.x;
    if (i >= nnz) return;
    const int64_t c0 = (i >> cshift) << cshift;
    const int64_t r0 = (i / kSub) * kSub;
    const int64_t cend = (c0 + (int64_t(1) << cshift)) < nnz ? c0 + (int64_t(1) << cshift) : nnz;
    const int32_t key = sdst[i];
    int64_t pos = i - r0;
    for (int64_t rs = c0; rs < cend; rs += kSub) {
        if (rs == r0) continue;
        int64_t lo = rs, hi = (rs + kSub) < cend ? rs + kSub : cend;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (sdst[mid] < key) lo = mid + 1; else hi = mid;
        }
        pos += lo - rs;
    }
    const uint32_t off = (uint32_t)((r0 - c0) + soff[i]);
    ddst[c0 + pos] = (int32_t)((uint32_t)key | ((off >> 16) << dbits));
    doff[c0 + pos] = (uint16_t)(off & 0xFFFFu);
}

// One record per thread: slot j of the tables, read from its chunk in L2.
template <int RW>
__global__ __launch_bounds__(kRemapThreads) void remap_flat_kernel(const uint32_t* __restrict__ in,
                                                                    uint32_t* __restrict__ out,
                                                                    const int32_t* __restrict__ ddst,
                                                                    const uint16_t* __restrict__ doff,
                                                                    int64_t nnz, int cshift, int dbits) {
    // the grid is a multiple of 8 chunks; block b runs on XCD b % 8 and takes
    // the (b / 8)-th block of that XCD's chunks c = x, x + 8, x + 16, ...
    const unsigned bpc = (1u << cshift) / kRemapThreads;  // workgroups per chunk
    const unsigned b = blockIdx.x, x = b % 8u, r = b / 8u;
    const unsigned v = ((r / bpc) * 8u + x) * bpc + r % bpc;
    const int64_t j = (int64_t)v * kRemapThreads + threadIdx.x;
    if (j >= nnz) return;
    const uint32_t t = (uint32_t)ddst[j];
    const int64_t p = ((j >> cshift) << cshift) + doff[j] + ((int64_t)(t >> dbits) << 16);
    const int64_t q = t & ((1u << dbits) - 1u);
    Rec<RW> rec;
    load_rec<RW>(in, p, rec);
    store_rec<RW>(out, q, rec);
}

// Bits of a destination (0 .. nnz - 1), at least 1.
int dest_bits(int64_t nnz) {
    int b = 1;
    while (b < 31 && (int64_t(1) << b) < nnz) ++b;
    return b;
}

// log2 of the records per chunk: the bytes target, at least kSub, at most
// what 16 bits of doff and the 32 - dbits spare bits of ddst address.
int chunk_shift(int words, int64_t nnz) {
    const int maxsh = 16 + (32 - dest_bits(nnz));
    int sh = 12;
    while (sh < maxsh && sh < 24 && ((int64_t(1) << (sh + 1)) * words * 4 <= (int64_t)SPT_STAGE_CHUNK_BYTES)) ++sh;
    return sh;
}

}  // namespace

int stage_chunk(int words, int64_t nnz) { return 1 << chunk_shift(words, nnz); }

void launch_stage_tables(int words, const int32_t* nxt, int64_t nnz, int32_t* ddst, uint16_t* doff,
                         int32_t* tmp_dst, uint16_t* tmp_off, hipStream_t s) {
    if (nnz == 0) return;
    const int cshift = chunk_shift(words, nnz);
    const unsigned subs = (unsigned)((nnz + kSub - 1) / kSub);
    hipLaunchKernelGGL(stage_tables_kernel<kSub>, dim3(subs), dim3(kStageThreads), 0, s, nxt, nnz, tmp_dst,
                       tmp_off);
    const unsigned blocks = (unsigned)((nnz + kStageThreads - 1) / kStageThreads);
    hipLaunchKernelGGL(merge_runs_kernel, dim3(blocks), dim3(kStageThreads), 0, s, (const int32_t*)tmp_dst,
                       (const uint16_t*)tmp_off, nnz, cshift, dest_bits(nnz), ddst, doff);
}

void launch_remap_staged(int words, int64_t nnz, const uint32_t* in, uint32_t* out, const int32_t* ddst,
                         const uint16_t* doff, hipStream_t s) {
    if (nnz == 0) return;
    const int cshift = chunk_shift(words, nnz), dbits = dest_bits(nnz);
    const int64_t nchunks = (nnz + (int64_t(1) << cshift) - 1) >> cshift;
    const unsigned blocks = (unsigned)(((nchunks + 7) / 8) * 8 * ((int64_t(1) << cshift) / kRemapThreads));
    if (words == 3)
        hipLaunchKernelGGL((remap_flat_kernel<3>), dim3(blocks), dim3(kRemapThreads), 0, s, in, out, ddst, doff,
                           nnz, cshift, dbits);
    else if (words == 4)
        hipLaunchKernelGGL((remap_flat_kernel<4>), dim3(blocks), dim3(kRemapThreads), 0, s, in, out, ddst, doff,
                           nnz, cshift, dbits);
    else if (words == 8)
        hipLaunchKernelGGL((remap_flat_kernel<8>), dim3(blocks), dim3(kRemapThreads), 0, s, in, out, ddst, doff,
                           nnz, cshift, dbits);
    else
        hipLaunchKernelGGL((remap_flat_kernel<12>), dim3(blocks), dim3(kRemapThreads), 0, s, in, out, ddst, doff,
                           nnz, cshift, dbits);
}

}  // namespace spt
