// Launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace spt {

// Arguments of the fused elementwise-computation / remapping kernel for one
// output mode d.  Everything "rotated" is indexed k = 0..N-1 for mode
// (d + k) mod N, so k = 0 is the output mode.
struct EcArgs {
    const uint32_t* rec_in;    // records of mode d's stream
    uint32_t* rec_out;         // remap target in mode d+1's order, or nullptr
    const int32_t* nxt;        // [nnz] position in mode d+1 of the record at p
    const int64_t* ptr;        // [kappa+1] partition offsets of mode d
    const int32_t* psplit_ptr; // [kappa+1] split rows of each partition
    const int32_t* psplit_row;
    const int32_t* psplit_slot;
    float* out;                // I_d x R
    float* carry;              // nslots x R partial sums of split rows
    const void* fac[8];        // rotated: fac[k] = factor of mode (d + k) mod N
    int32_t rot[8];            // rot[k] = (d + k) mod N
    int32_t foff[8];           // bit offset of each mode's index (packed layout)
    uint32_t fmask[8];         // width mask of each mode's index (packed layout)
};

// Forward pass of the gradient fit (grad_kernel.hip).
struct ForwardArgs {
    const uint32_t* rec_in;    // records of a stream
    uint32_t* rec_res;         // same records with value m_e - x_e, same order
    const float* fac[8];       // factors in mode order
    double* loss_part;         // [forward_blocks(nnz)] partial sums of (x-m)^2 / 2
    int64_t nnz;
    int32_t foff[8];           // bit offset of each mode's index (packed layout)
    uint32_t fmask[8];
};

struct FixupArgs {
    float* out;
    const float* carry;
    const int32_t* split_row;  // [nsplit]
    const int32_t* split_ptr;  // [nsplit+1]
    const int32_t* empty_rows; // [nempty]
    int32_t nsplit;
    int32_t nempty;
};

using EcFnPtr = void (*)(EcArgs);

// fdtype 0: FP32 factors, 1: BF16 factors.  Returns false if the combination
// (nmodes, rank, factor type, record words, layout kind) has no kernel.  One
// single-wave workgroup per partition (kappa of them).
bool launch_ec(int nmodes, int rank, int fdtype, int words, int kind, int kappa, const EcArgs& a,
               hipStream_t s);
// true if the combination has an elementwise kernel
bool pick_ec_exists(int nmodes, int rank, int fdtype, int words, int kind);
int forward_blocks(int64_t nnz);
bool launch_forward(int nmodes, int rank, int words, int kind, const ForwardArgs& a,
                    hipStream_t s);
// dst[i] = src[i] rounded to the nearest BF16 (ties to even), i < n
void launch_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t s);
void launch_fixup(int rank, const FixupArgs& a, hipStream_t s);
// Moves every record of the stream from position p to the position reached by
// following `hops` next-position arrays (nxt[0] first).
void launch_remap(int words, int64_t nnz, const uint32_t* in, uint32_t* out,
                  const int32_t* const* nxt, int hops, hipStream_t s);
// Staged remapping (dr_staged.hip): records in chunks of stage_chunk(words,
// nnz) consecutive stream positions; per chunk, the destinations in
// increasing order (ddst) and the offset inside the chunk of the record for
// each (doff, with the offset's bits above 16 stored in ddst above the
// destination's bits).  The build needs nnz-entry temporaries tmp_dst /
// tmp_off.
int stage_chunk(int words, int64_t nnz);
void launch_stage_tables(int words, const int32_t* nxt, int64_t nnz, int32_t* ddst, uint16_t* doff,
                         int32_t* tmp_dst, uint16_t* tmp_off, hipStream_t s);
// out[ddst[j]] = in[chunk(j) * C + doff[j]] for every j < nnz
void launch_remap_staged(int words, int64_t nnz, const uint32_t* in, uint32_t* out, const int32_t* ddst,
                         const uint16_t* doff, hipStream_t s);

// ---- CP-ALS dense step (FP64 for everything R x R) ----
int gram_blocks(int64_t rows);
// partial[b][R*R] for b < gram_blocks(rows)
void launch_gram_partial(int rank, const float* Y, int64_t rows, double* partial, hipStream_t s);
// out[e] = sum_b partial[b][e] (fixed order), e < E
void launch_reduce_partials(const double* partial, int nblocks, int E, double* out, hipStream_t s);
// V = Hadamard of grams[w] (w != mode); Cholesky; Vinv.  status[0] |= 1 on
// failure after one ridge retry.
void launch_normal_inverse(int rank, int nmodes, int mode, const double* grams, double* Vinv,
                           int32_t* status, hipStream_t s);
// Y = M Vinv (FP32 out); partial Grams of Y and partial column sums of M.*Y
int solve_blocks(int64_t rows);
void launch_solve_rows(int rank, const float* M, const double* Vinv, int64_t rows, float* Y,
                       double* gpart, double* ipart, hipStream_t s);
// From the reduced sums G_un (R x R) and Isum (R): lambda = sqrt(diag G_un),
// grams[mode] = D^-1 G_un D^-1; if want_fit, fit[0] from all grams, lambda,
// Isum and normX2.
void launch_als_finish(int rank, int nmodes, int mode, const double* Gun, const double* Isum,
                       double* grams, double* lambda, double normX2, int want_fit, double* fit,
                       hipStream_t s);
void launch_scale_cols(int rank, float* Y, int64_t rows, const double* lambda, hipStream_t s);
// dst[0..bytes) = src[0..bytes), bytes a multiple of 16 (probe.hip)
void launch_copy_probe(const void* src, void* dst, int64_t bytes, hipStream_t s);
// The fixed per-device buffer of spt_mttkrp_noalloc (noalloc.hip): its size,
// and its device address on the current device (looked up once per device).
constexpr int64_t kNoAllocScratchBytes = int64_t(16) << 20;
hipError_t noalloc_scratch(void** ptr);
// p[0..n) = 0 with a kernel (no memset node when a caller captures a graph)
void launch_zero_i32(int32_t* p, int n, hipStream_t s);

}  // namespace spt
